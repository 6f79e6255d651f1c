/*
 * FP64 CPU oracle of the GL-ECSIM particle pass and field step
 * (Chen, Zhou & Toth, "Suppressing spurious oscillations and particle noise
 * in particle-in-cell simulations", arXiv 2506.11320).
 *
 * TEST INFRASTRUCTURE ONLY.  Plain, slow, obviously correct loops in double
 * precision.  Only the tests, the smoke check and the benchmark's CPU-baseline
 * leg use it; the product path never does.  It shares no code with the GPU
 * library.
 *
 * Mesh (Sec. 2.1): E on nodes, B at cell centres.  Node (i,j,k) sits at
 * (i dx, j dy, k dz); cell (i,j,k) has its centre at ((i+1/2) dx, ...).  The
 * active axes are periodic, except an x axis closed by walls (see "Walled x
 * axis" below).  Fields are stored component-major, [3][N], with linear index
 * i + nx*(j + ny*k); nodes and cells share the index space (as many nodes as
 * cells; a walled x axis stores one more point).
 *
 * Each function names the passage of the paper it follows.  Readings of
 * passages that are silent or garbled are marked READING.
 *
 * Parity unpinned (no closed form, printed value or invariant fixes them;
 * the GPU path implements the same reading): the multi-dimensional form of
 * the LF coefficients and their diffusion speed (or_kappa_E / or_kappa_B
 * beyond 1D), and which lag of the E limiter the paper's code uses.  The node
 * average of B (or_node_avg) is pinned by its exactness on linear fields;
 * where B is interpolated to the particles stays a reading.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "glecsim_oracle.h"

static int64_t nnodes(const or_grid* G) {
  int64_t N = 1;
  for (int d = 0; d < G->dim; ++d) N *= G->n[d];
  return N;
}
static double cellvol(const or_grid* G) {
  double v = 1.0;
  for (int d = 0; d < G->dim; ++d) v *= G->dx[d];
  return v;
}
static void unflat(const or_grid* G, int64_t g, int ic[3]) {
  ic[0] = ic[1] = ic[2] = 0;
  for (int d = 0; d < G->dim; ++d) { ic[d] = (int)(g % G->n[d]); g /= G->n[d]; }
}
static int64_t flat(const or_grid* G, const int ic[3]) {
  int64_t g = 0;
  for (int d = G->dim - 1; d >= 0; --d) {
    int i = ic[d] % G->n[d];
    if (i < 0) i += G->n[d];
    g = g * G->n[d] + i;
  }
  return g;
}
/* index of a neighbour shifted by o[3] (periodic) */
static int64_t shifted(const or_grid* G, int64_t g, const int o[3]) {
  int ic[3]; unflat(G, g, ic);
  int jc[3] = {ic[0] + o[0], ic[1] + o[1], ic[2] + o[2]};
  return flat(G, jc);
}

int64_t or_nnodes(const or_grid* G) { return nnodes(G); }

/* ---------------------------------------------------------------------- */
/* Walled x axis (READING: the paper's shock runs are driven flows against a
 * boundary, Sec. 4.3-4.4, whose discretisation it does not print).  A
 * conducting wall is the mirror of the domain: under x -> -x the tangential
 * E and the normal B are odd (they vanish on the wall) and the normal E and
 * the tangential B are even.  At the inflow plane E is held at its upstream
 * value and the ghost cell beyond it holds the upstream B.
 * Storage: n[0] = nx + 1 points along x (nodes 0..nx; cells 0..nx-1 and the
 * ghost cell nx). */
enum { OR_PERIODIC = 0, OR_WALL = 1, OR_INFLOW = 2 };
static int walled(const or_grid* G) { return G->bc_lo != OR_PERIODIC; }
static int nxp(const or_grid* G) { return G->n[0] - 1; } /* physical cells along x when walled */
/* cell (i, j, k), i possibly beyond the walls: value of component comp of a
 * cell field; odd: the component changes sign under the mirror */
static double cell_val(const or_grid* G, const double* F, int comp, int i, int j, int k, int odd) {
  int64_t N = nnodes(G);
  double sg = 1.0;
  if (walled(G)) {
    int nx = nxp(G);
    if (i < 0) { i = -1 - i; sg = odd ? -1.0 : 1.0; }
    else if (i >= nx && G->bc_hi == OR_WALL) { i = 2 * nx - 1 - i; sg = odd ? -1.0 : 1.0; }
  }
  int ic[3] = {i, j, k};
  return sg * F[comp * N + flat(G, ic)];
}
/* node (i, j, k) of a node field with the wall mirror (i in [-nx, 2 nx]) */
static double node_val(const or_grid* G, const double* F, int comp, int i, int j, int k, int odd) {
  int64_t N = nnodes(G);
  double sg = 1.0;
  if (walled(G)) {
    int nx = nxp(G);
    if (i < 0) { i = -i; sg = odd ? -1.0 : 1.0; }
    else if (i > nx) { i = 2 * nx - i; sg = odd ? -1.0 : 1.0; }
  }
  int ic[3] = {i, j, k};
  return sg * F[comp * N + flat(G, ic)];
}
/* parity of vector components under the x mirror: B-like (pseudo-vector:
 * normal odd) and E-like / velocity-like (normal even, tangential odd for E;
 * the velocity's normal component is odd) */
static int odd_B(int comp) { return comp == 0; }
static int odd_u(int comp) { return comp == 0; }
/* E^{n+theta} components held at a node: the tangential components on a wall,
 * all three on the inflow plane */
static int dirichlet(const or_grid* G, int i, int comp) {
  if (!walled(G)) return 0;
  int nx = nxp(G);
  if (i == 0) return comp != 0;
  if (i == nx) return G->bc_hi == OR_INFLOW ? 1 : comp != 0;
  return 0;
}

/* ---------------------------------------------------------------------- */
/* Shape function (linear, cloud-in-cell).  READING: the paper does not name
 * the shape order; the workloads use linear shapes.
 * W(x_p - x_g) = prod_d max(0, 1 - |x_p,d - x_g,d| / dx_d), the distance taken
 * on the periodic domain.  Returns the 2^dim nodes with their weights. */
int or_shape(const or_grid* G, const double x[3], int64_t nodes[8], double W[8]) {
  int base[3] = {0, 0, 0};
  for (int d = 0; d < G->dim; ++d) base[d] = (int)floor(x[d] / G->dx[d]);
  int nc = 1 << G->dim;
  for (int a = 0; a < nc; ++a) {
    int ic[3] = {0, 0, 0};
    double w = 1.0;
    for (int d = 0; d < G->dim; ++d) {
      int i = base[d] + ((a >> d) & 1);
      double L = G->n[d] * G->dx[d];
      double dist = fabs(x[d] - i * G->dx[d]);
      dist = fmod(dist, L);
      if (dist > 0.5 * L) dist = L - dist;
      double t = 1.0 - dist / G->dx[d];
      w *= (t > 0.0) ? t : 0.0;
      ic[d] = i;
    }
    nodes[a] = flat(G, ic);
    W[a] = w;
  }
  return nc;
}

/* ---------------------------------------------------------------------- */
/* Rotation matrix alpha (Sec. 3.1, the definition of alpha^n_p):
 *   alpha = (I - beta I x B + beta^2 B B) / (1 + beta^2 |B|^2).
 * READING of the sign of "I x B": alpha w = (w + beta w x B + beta^2 (w.B) B)
 * / (1 + beta^2 B^2), the inverse of (I - beta [. x B]); it is the only sign
 * for which the paper's identity alpha (u + beta E_M) = u with E_M = -u x B
 * holds.  Stored row-major: alpha[3*i + j]. */
void or_alpha(double beta, const double B[3], double alpha[9]) {
  double b2 = B[0] * B[0] + B[1] * B[1] + B[2] * B[2];
  double den = 1.0 + beta * beta * b2;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      /* (w x B)_i = eps_{i j k} w_j B_k, so the matrix of w -> w x B has
         entry [i][j] = eps_{i j k} B_k */
      double cross = 0.0;
      for (int k = 0; k < 3; ++k) {
        int e = (i == j || j == k || i == k) ? 0 : (((j - i + 3) % 3 == 1) ? 1 : -1);
        cross += e * B[k];
      }
      alpha[3 * i + j] = ((i == j ? 1.0 : 0.0) + beta * cross + beta * beta * B[i] * B[j]) / den;
    }
}

static void matvec3(const double A[9], const double x[3], double y[3]) {
  for (int i = 0; i < 3; ++i) y[i] = A[3 * i] * x[0] + A[3 * i + 1] * x[1] + A[3 * i + 2] * x[2];
}

/* B at nodes: the mean of B over the 2^dim cells that touch node g.
 * READING: the paper leaves the location at which B is interpolated to the
 * particle unstated; B is averaged to nodes and gathered with the same
 * linear weights as E. */
void or_node_avg(const or_grid* G, const double* Bc, double* Bn) {
  int64_t N = nnodes(G);
  int nc = 1 << G->dim;
  for (int64_t g = 0; g < N; ++g) {
    int ic[3]; unflat(G, g, ic);
    for (int comp = 0; comp < 3; ++comp) {
      double s = 0.0;
      for (int a = 0; a < nc; ++a) {
        int o[3] = {0, 0, 0};
        for (int d = 0; d < G->dim; ++d) o[d] = -((a >> d) & 1);
        s += cell_val(G, Bc, comp, ic[0] + o[0], ic[1] + o[1], ic[2] + o[2], odd_B(comp));
      }
      Bn[comp * N + g] = s / nc;
    }
  }
}

static void gather(const or_grid* G, const double* F, const int64_t nodes[8], const double W[8], int nc,
                   double out[3]) {
  int64_t N = nnodes(G);
  for (int comp = 0; comp < 3; ++comp) {
    double s = 0.0;
    for (int a = 0; a < nc; ++a) s += W[a] * F[comp * N + nodes[a]];
    out[comp] = s;
  }
}

/* offset index in the full 27-point stencil */
static int off27(const int o[3]) { return (o[0] + 1) + 3 * (o[1] + 1) + 9 * (o[2] + 1); }

/* ---------------------------------------------------------------------- */
/* Deposit of one species (Sec. 3.1).  Accumulates into caller-zeroed arrays:
 *   J[3][N]      += (1/dV) sum_p q_p alpha_p (v_p - u(x_p)) W_pg
 *                   (u_node == NULL: lab frame, u = 0; else the comoving
 *                   current J_C of Sec. 3.1 with u(x_p) = sum_g W_pg u_g)
 *   M[27][9][N]  += sum_p q_p alpha_p W_pg W_pg'   at g, offset g' - g
 *                   (mass matrix M_{s,gg'}, all 27 offsets, no symmetry used)
 *   rho[N]       += (1/dV) sum_p q_p W_pg
 *   mm[3][N]     += m_s sum_p w_p v_p W_pg            (mass-weighted momentum)
 *   mass[N]      += m_s sum_p w_p W_pg
 * q_p = q_s w_p.  Particles: x[3*p + d] global positions, v[3*p + d]. */
void or_deposit_species(const or_grid* G, double qs, double ms, double beta_s, int64_t np,
                        const double* x, const double* v, const double* w, const double* Bn,
                        const double* u_node, double* J, double* M, double* rho, double* mm,
                        double* mass) {
  int64_t N = nnodes(G);
  double dV = cellvol(G);
  for (int64_t p = 0; p < np; ++p) {
    int64_t nodes[8]; double W[8];
    int nc = or_shape(G, &x[3 * p], nodes, W);
    double Bp[3]; gather(G, Bn, nodes, W, nc, Bp);
    double al[9]; or_alpha(beta_s, Bp, al);
    double qp = qs * w[p];
    double vc[3] = {v[3 * p], v[3 * p + 1], v[3 * p + 2]};
    if (u_node) {
      double up[3]; gather(G, u_node, nodes, W, nc, up);
      for (int d = 0; d < 3; ++d) vc[d] -= up[d];
    }
    double av[3]; matvec3(al, vc, av);
    for (int a = 0; a < nc; ++a) {
      int64_t g = nodes[a];
      for (int d = 0; d < 3; ++d) J[d * N + g] += qp * av[d] * W[a] / dV;
      rho[g] += qp * W[a] / dV;
      for (int d = 0; d < 3; ++d) mm[d * N + g] += ms * w[p] * v[3 * p + d] * W[a];
      mass[g] += ms * w[p] * W[a];
      for (int b = 0; b < nc; ++b) {
        int o[3] = {0, 0, 0};
        for (int d = 0; d < G->dim; ++d) o[d] = ((b >> d) & 1) - ((a >> d) & 1);
        int oi = off27(o);
        for (int e = 0; e < 9; ++e) M[((int64_t)oi * 9 + e) * N + g] += qp * al[e] * W[a] * W[b];
      }
    }
  }
}

/* u = mass-weighted bulk velocity (Sec. 3.1: "the plasma velocity").
 * READING: u_g = sum_s m_s sum_p w_p v_p W_pg / sum_s m_s sum_p w_p W_pg, and
 * u_g = 0 where no particle touches node g. */
void or_bulk_velocity(const or_grid* G, const double* mm, const double* mass, double* u) {
  int64_t N = nnodes(G);
  for (int64_t g = 0; g < N; ++g)
    for (int d = 0; d < 3; ++d) u[d * N + g] = (mass[g] > 0.0) ? mm[d * N + g] / mass[g] : 0.0;
}

/* Digital filter of Sec. 2.4, one pass along one axis with stride d:
 *   v*_i = phi v_i + (1 - phi)/2 (v_{i-d} + v_{i+d}), periodic. */
void or_filter_axis(const or_grid* G, double* f, int ncomp, double phi, int stride, int axis) {
  int64_t N = nnodes(G);
  double* tmp = (double*)malloc(sizeof(double) * N);
  for (int c = 0; c < ncomp; ++c) {
    for (int64_t g = 0; g < N; ++g) {
      int om[3] = {0, 0, 0}, op[3] = {0, 0, 0};
      om[axis] = -stride; op[axis] = stride;
      double lo, hi;
      if (axis == 0 && walled(G)) {
        /* READING: mirror at the walls (a 3-component field is a velocity or
           a current: its normal component is odd) */
        int ic[3]; unflat(G, g, ic);
        int odd = ncomp == 3 && odd_u(c);
        lo = node_val(G, f, c, ic[0] - stride, ic[1], ic[2], odd);
        hi = node_val(G, f, c, ic[0] + stride, ic[1], ic[2], odd);
      } else {
        lo = f[c * N + shifted(G, g, om)];
        hi = f[c * N + shifted(G, g, op)];
      }
      tmp[g] = phi * f[c * N + g] + 0.5 * (1.0 - phi) * (lo + hi);
    }
    memcpy(&f[c * N], tmp, sizeof(double) * N);
  }
  free(tmp);
}

/* Smoothing of u (Sec. 3.1): npass passes with phi, the stride alternating
 * 1, 2, 1, 2, ...  READING: each pass sweeps x, then y, then z. */
void or_smooth(const or_grid* G, double* f, int ncomp, int npass, double phi) {
  for (int k = 0; k < npass; ++k)
    for (int axis = 0; axis < G->dim; ++axis) or_filter_axis(G, f, ncomp, phi, (k % 2 == 0) ? 1 : 2, axis);
}

/* Motional electric field E_M = -u x B (Sec. 3.1), at nodes with B averaged
 * to nodes. */
void or_motional(const or_grid* G, const double* u, const double* Bn, double* EM) {
  int64_t N = nnodes(G);
  for (int64_t g = 0; g < N; ++g) {
    double a[3] = {u[g], u[N + g], u[2 * N + g]}, b[3] = {Bn[g], Bn[N + g], Bn[2 * N + g]};
    EM[g] = -(a[1] * b[2] - a[2] * b[1]);
    EM[N + g] = -(a[2] * b[0] - a[0] * b[2]);
    EM[2 * N + g] = -(a[0] * b[1] - a[1] * b[0]);
  }
}

/* y[3][N] = sum_{g'} M[g, g'] x[g'] with M in the full 27-offset layout. */
void or_mass_apply(const or_grid* G, const double* M, const double* x, double* y) {
  int64_t N = nnodes(G);
  for (int64_t g = 0; g < N; ++g) {
    double acc[3] = {0, 0, 0};
    for (int oz = -1; oz <= 1; ++oz)
      for (int oy = -1; oy <= 1; ++oy)
        for (int ox = -1; ox <= 1; ++ox) {
          int o[3] = {ox, oy, oz};
          if ((G->dim < 2 && oy) || (G->dim < 3 && oz)) continue;
          int64_t h = shifted(G, g, o);
          int oi = off27(o);
          for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) acc[i] += M[((int64_t)oi * 9 + 3 * i + j) * N + g] * x[j * N + h];
        }
    for (int i = 0; i < 3; ++i) y[i * N + g] = acc[i];
  }
}

/* Effective explicit current of the comoving E system (Sec. 3.1, the
 * modified E equation): J_eff = J_C - (1/dV) sum_{s,g'} beta_s M_{s,gg'} E_M,g'. */
void or_current_eff(const or_grid* G, const double* JC, const double* Mtilde, const double* EM, double* Jeff) {
  int64_t N = nnodes(G);
  double dV = cellvol(G);
  double* t = (double*)malloc(sizeof(double) * 3 * N);
  or_mass_apply(G, Mtilde, EM, t);
  for (int64_t i = 0; i < 3 * N; ++i) Jeff[i] = JC[i] - t[i] / dV;
  free(t);
}

/* ---------------------------------------------------------------------- */
/* Generalised MC limiter of van Leer (Sec. 2.2):
 *   phi(r, beta) = max(0, min(beta r, (1 + r)/2, beta)),
 * with r = num / den.  READING for den = 0: r = 1 when num = 0 as well (a
 * locally constant profile is smooth), r = +inf (phi = beta) for num > 0 and
 * r = -inf (phi = 0) for num < 0.  beta = 0 gives phi = 0 everywhere (the
 * unlimited first-order scheme of Sec. 2.2). */
double or_limiter(double num, double den, double beta) {
  double r;
  if (den == 0.0) {
    if (num == 0.0) r = 1.0;
    else return (num > 0.0) ? beta : 0.0;
  } else {
    r = num / den;
  }
  double a = beta * r, b = 0.5 * (1.0 + r), c = beta;
  double m = a < b ? a : b;
  m = m < c ? m : c;
  return m > 0.0 ? m : 0.0;
}

/* Diffusion coefficients of the E operator (Sec. 2.2, the numerical flux d
 * of the implicit E diffusion).  For component m and axis d, the flux between
 * node g and g + e_d is stored at index g:
 *   kappa = (1 - phi_E) a / 2,
 *   r = (E_g - E_{g-e_d}) / (E_{g+e_d} - E_g).
 * READINGS: the ratio is lagged to E^n (the paper uses the unknown E^{n+theta},
 * which would make the system nonlinear); the multi-dimensional form applies
 * the 1D formula axis by axis and component by component; a at the flux is
 * the mean of a over the two nodes it joins.  a_node[N] is the diffusion
 * speed at nodes (c for light-wave runs, |u| for plasma runs).
 * Layout kappa[(d*3 + m)*N + g]. */
void or_kappa_E(const or_grid* G, const double* E, const double* a_node, double beta, double* kappa) {
  int64_t N = nnodes(G);
  memset(kappa, 0, sizeof(double) * 9 * N);
  for (int d = 0; d < G->dim; ++d) {
    int om[3] = {0, 0, 0}, op[3] = {0, 0, 0};
    om[d] = -1; op[d] = 1;
    for (int m = 0; m < 3; ++m)
      for (int64_t g = 0; g < N; ++g) {
        int64_t gm = shifted(G, g, om), gp = shifted(G, g, op);
        double phi = or_limiter(E[m * N + g] - E[m * N + gm], E[m * N + gp] - E[m * N + g], beta);
        double a = 0.5 * (a_node[g] + a_node[gp]);
        if (d == 0 && walled(G)) {
          /* READING: no flux through the boundary planes; at the face next to
             the lower wall the ratio would need a value beyond it: phi = 0 */
          int ic[3]; unflat(G, g, ic);
          if (ic[0] == nxp(G)) { kappa[(d * 3 + m) * N + g] = 0.0; continue; }
          if (ic[0] == 0) phi = 0.0;
        }
        kappa[(d * 3 + m) * N + g] = 0.5 * (1.0 - phi) * a;
      }
  }
}

/* Diffusion coefficients of the B update (Sec. 2.2, the flux f_B): for
 * component m and axis d, the face between cell c and c + e_d, stored at c:
 *   kappa = (1 - phi_B) a / 2,  r = (B_c - B_{c-e_d}) / (B_{c+e_d} - B_c).
 * a at the face is the mean of a_node over the 2^(dim-1) nodes of the face
 * (READING, as for E). */
void or_kappa_B(const or_grid* G, const double* B, const double* a_node, double beta, double* kappa) {
  int64_t N = nnodes(G);
  memset(kappa, 0, sizeof(double) * 9 * N);
  int nf = 1 << (G->dim - 1);
  for (int d = 0; d < G->dim; ++d) {
    int om[3] = {0, 0, 0}, op[3] = {0, 0, 0};
    om[d] = -1; op[d] = 1;
    for (int64_t c = 0; c < N; ++c) {
      /* nodes of the face between c and c + e_d: node index c + e_d + t
         with t_d = 0 and t_e in {0,1} for the other axes */
      double asum = 0.0;
      int k = 0;
      for (int t = 0; t < (1 << G->dim); ++t) {
        if ((t >> d) & 1) continue;
        int o[3] = {0, 0, 0};
        for (int e = 0; e < G->dim; ++e) o[e] = (t >> e) & 1;
        o[d] = 1;
        asum += a_node[shifted(G, c, o)];
        ++k;
      }
      (void)k;
      double a = asum / nf;
      int64_t cm = shifted(G, c, om), cp = shifted(G, c, op);
      int ic[3]; unflat(G, c, ic);
      for (int m = 0; m < 3; ++m) {
        double phi = or_limiter(B[m * N + c] - B[m * N + cm], B[m * N + cp] - B[m * N + c], beta);
        if (walled(G)) {
          /* READING: no flux through the boundary faces and none on the ghost
             cells; next to the lower wall the ratio is not defined: phi = 0 */
          if (ic[0] >= nxp(G) - (d == 0)) { kappa[(d * 3 + m) * N + c] = 0.0; continue; }
          if (d == 0 && ic[0] == 0) phi = 0.0;
        }
        kappa[(d * 3 + m) * N + c] = 0.5 * (1.0 - phi) * a;
      }
    }
  }
}

/* ---------------------------------------------------------------------- */
/* Discrete curls (READING: only the 1D stencil is printed, Sec. 2.1).
 * Partial derivative along d from nodes to a cell: the difference of the
 * means over the cell's upper and lower faces (2^(dim-1) nodes each).
 * From cells to a node: the difference of the means over the cells on the
 * upper and lower side of the node.  Along inactive axes the derivative is 0. */
static double dnc(const or_grid* G, const double* F, int64_t c, int d) {
  if (d >= G->dim) return 0.0;
  int nc = 1 << G->dim;
  double up = 0.0, lo = 0.0;
  for (int a = 0; a < nc; ++a) {
    int o[3] = {0, 0, 0};
    for (int e = 0; e < G->dim; ++e) o[e] = (a >> e) & 1;
    double val = F[shifted(G, c, o)];
    if ((a >> d) & 1) up += val; else lo += val;
  }
  return (up - lo) / (nc / 2) / G->dx[d];
}
static double dcn(const or_grid* G, const double* F, int64_t g, int d) {
  if (d >= G->dim) return 0.0;
  int nc = 1 << G->dim;
  double up = 0.0, lo = 0.0;
  for (int a = 0; a < nc; ++a) {
    int o[3] = {0, 0, 0};
    for (int e = 0; e < G->dim; ++e) o[e] = -((a >> e) & 1);
    double val = F[shifted(G, g, o)];
    /* cell g - a lies on the upper side along d when a_d = 0 */
    if ((a >> d) & 1) lo += val; else up += val;
  }
  return (up - lo) / (nc / 2) / G->dx[d];
}

void or_curl_nc(const or_grid* G, const double* E, double* out) {
  int64_t N = nnodes(G);
  for (int64_t c = 0; c < N; ++c) {
    out[c] = dnc(G, &E[2 * N], c, 1) - dnc(G, &E[N], c, 2);
    out[N + c] = dnc(G, &E[0], c, 2) - dnc(G, &E[2 * N], c, 0);
    out[2 * N + c] = dnc(G, &E[N], c, 0) - dnc(G, &E[0], c, 1);
    if (walled(G)) {
      int ic[3]; unflat(G, c, ic);
      if (ic[0] == nxp(G)) out[c] = out[N + c] = out[2 * N + c] = 0.0;  /* the ghost cell */
    }
  }
}
/* cell -> node derivative of component comp along d with the wall mirror */
static double dcn_w(const or_grid* G, const double* B, int comp, int64_t g, int d) {
  if (d >= G->dim) return 0.0;
  int nc = 1 << G->dim;
  int ic[3]; unflat(G, g, ic);
  double up = 0.0, lo = 0.0;
  for (int a = 0; a < nc; ++a) {
    int o[3] = {0, 0, 0};
    for (int e = 0; e < G->dim; ++e) o[e] = -((a >> e) & 1);
    double val = cell_val(G, B, comp, ic[0] + o[0], ic[1] + o[1], ic[2] + o[2], odd_B(comp));
    if ((a >> d) & 1) lo += val; else up += val;
  }
  return (up - lo) / (nc / 2) / G->dx[d];
}
void or_curl_cn(const or_grid* G, const double* B, double* out) {
  int64_t N = nnodes(G);
  for (int64_t g = 0; g < N; ++g) {
    if (walled(G)) {
      out[g] = dcn_w(G, B, 2, g, 1) - dcn_w(G, B, 1, g, 2);
      out[N + g] = dcn_w(G, B, 0, g, 2) - dcn_w(G, B, 2, g, 0);
      out[2 * N + g] = dcn_w(G, B, 1, g, 0) - dcn_w(G, B, 0, g, 1);
      continue;
    }
    out[g] = dcn(G, &B[2 * N], g, 1) - dcn(G, &B[N], g, 2);
    out[N + g] = dcn(G, &B[0], g, 2) - dcn(G, &B[2 * N], g, 0);
    out[2 * N + g] = dcn(G, &B[N], g, 0) - dcn(G, &B[0], g, 1);
  }
}
/* divergence of a node field at cells */
void or_div_nc(const or_grid* G, const double* E, double* out) {
  int64_t N = nnodes(G);
  for (int64_t c = 0; c < N; ++c) out[c] = dnc(G, &E[0], c, 0) + dnc(G, &E[N], c, 1) + dnc(G, &E[2 * N], c, 2);
}

/* Gauss's law residual.  Sec. 2.1 writes Maxwell's equations; Gauss's law
 * div E = 4 pi rho is the constraint the GL correction named in Sec. 1 restores
 * (the correction itself is not described there).  READING: the residual is
 * taken at cell centres, where div_NC lives, against the cell mean of the
 * node charge density (rho_node summed over species, mean over the cell's
 * 2^dim nodes):
 *   out[0] = sum_c (div_NC E - 4 pi rho_c)^2,   out[1] = sum_c (4 pi rho_c)^2,
 * so that the relative residual is sqrt(out[0] / out[1]). */
void or_gauss_sums(const or_grid* G, const double* E, const double* rho_node, double out[2]) {
  int64_t N = nnodes(G);
  int nc = 1 << G->dim;
  double* div = (double*)malloc(sizeof(double) * N);
  or_div_nc(G, E, div);
  out[0] = out[1] = 0.0;
  for (int64_t c = 0; c < N; ++c) {
    if (walled(G)) {
      int ic[3]; unflat(G, c, ic);
      if (ic[0] == nxp(G)) continue;  /* the ghost cell */
    }
    double rc = 0.0;
    for (int a = 0; a < nc; ++a) {
      int o[3] = {0, 0, 0};
      for (int e = 0; e < G->dim; ++e) o[e] = (a >> e) & 1;
      rc += rho_node[shifted(G, c, o)];
    }
    double r4 = 4.0 * M_PI * rc / nc;
    out[0] += (div[c] - r4) * (div[c] - r4);
    out[1] += r4 * r4;
  }
  free(div);
}

/* Diffusion operator D applied to a field F (node or cell, same stencil):
 *   (D F)_g = sum_d (1/dx_d) [k_{g}(F_{g+e_d} - F_g) - k_{g-e_d}(F_g - F_{g-e_d})]
 * with kappa stored at the lower point of each flux. */
void or_diffusion(const or_grid* G, const double* kappa, const double* F, double* out) {
  int64_t N = nnodes(G);
  for (int m = 0; m < 3; ++m)
    for (int64_t g = 0; g < N; ++g) {
      double s = 0.0;
      for (int d = 0; d < G->dim; ++d) {
        int om[3] = {0, 0, 0}, op[3] = {0, 0, 0};
        om[d] = -1; op[d] = 1;
        int64_t gm = shifted(G, g, om), gp = shifted(G, g, op);
        double kp = kappa[(d * 3 + m) * N + g], km = kappa[(d * 3 + m) * N + gm];
        s += (kp * (F[m * N + gp] - F[m * N + g]) - km * (F[m * N + g] - F[m * N + gm])) / G->dx[d];
      }
      out[m * N + g] = s;
    }
}

/* ---------------------------------------------------------------------- */
/* The implicit E operator (Sec. 2.1 ECSIM-E, with the mass term of Sec. 3.1
 * and the implicit LF diffusion of Sec. 2.2):
 *   A x = x + (c theta dt)^2 curl_CN curl_NC x
 *           + (4 pi theta dt / dV) sum_g' Mtilde_{gg'} x_g'
 *           - theta dt D_E x.
 * READINGS: grad div - laplacian is discretised as curl_CN(curl_NC); the
 * printed mass-term coefficient 4 pi/(c dV) is read as 4 pi theta dt / dV (the
 * value obtained by substituting the predicted current into ECSIM-E); the
 * diffusion enters with the sign that makes it dissipative.  Mtilde or kappa
 * may be NULL (term absent). */
void or_apply_A(const or_grid* G, const or_params* P, const double* Mtilde, const double* kappaE,
                const double* x, double* y) {
  int64_t N = nnodes(G);
  double dV = cellvol(G);
  double ctd = P->c * P->theta * P->dt;
  double* cc = (double*)malloc(sizeof(double) * 3 * N);
  double* t = (double*)malloc(sizeof(double) * 3 * N);
  or_curl_nc(G, x, cc);
  or_curl_cn(G, cc, t);
  for (int64_t i = 0; i < 3 * N; ++i) y[i] = x[i] + ctd * ctd * t[i];
  if (Mtilde) {
    or_mass_apply(G, Mtilde, x, t);
    for (int64_t i = 0; i < 3 * N; ++i) y[i] += 4.0 * M_PI * P->theta * P->dt / dV * t[i];
  }
  if (kappaE) {
    or_diffusion(G, kappaE, x, t);
    for (int64_t i = 0; i < 3 * N; ++i) y[i] -= P->theta * P->dt * t[i];
  }
  if (walled(G))
    for (int64_t g = 0; g < N; ++g) {
      int ic[3]; unflat(G, g, ic);
      for (int m = 0; m < 3; ++m)
        if (dirichlet(G, ic[0], m)) y[m * N + g] = x[m * N + g];  /* held components: identity rows */
    }
  free(cc);
  free(t);
}

/* Right-hand side (Sec. 2.1 ECSIM-E; Sec. 3.1):
 *   b = E^n + c theta dt curl_CN B^n - 4 pi theta dt J_eff. */
void or_rhs(const or_grid* G, const or_params* P, const double* En, const double* Bc, const double* Jeff,
            double* b) {
  int64_t N = nnodes(G);
  double* t = (double*)malloc(sizeof(double) * 3 * N);
  or_curl_cn(G, Bc, t);
  for (int64_t i = 0; i < 3 * N; ++i)
    b[i] = En[i] + P->c * P->theta * P->dt * t[i] - 4.0 * M_PI * P->theta * P->dt * Jeff[i];
  if (walled(G))
    for (int64_t g = 0; g < N; ++g) {
      int ic[3]; unflat(G, g, ic);
      for (int m = 0; m < 3; ++m)
        if (dirichlet(G, ic[0], m)) b[m * N + g] = En[m * N + g];  /* E^{n+theta} = E^n there */
    }
  free(t);
}

/* B update (Sec. 2.1 theta-B with Sec. 2.2's diffusive flux):
 *   B^{n+1} = B^n - c dt curl_NC E^{n+theta} + dt D_B B^n.
 * READING: the printed factor c theta dt in ECSIM-B is read as c dt, as in
 * theta-B and in the 1D update. */
void or_update_B(const or_grid* G, const or_params* P, const double* Bc, const double* Eth,
                 const double* kappaB, double* Bnew) {
  int64_t N = nnodes(G);
  double* t = (double*)malloc(sizeof(double) * 3 * N);
  or_curl_nc(G, Eth, t);
  for (int64_t i = 0; i < 3 * N; ++i) Bnew[i] = Bc[i] - P->c * P->dt * t[i];
  if (kappaB) {
    or_diffusion(G, kappaB, Bc, t);
    for (int64_t i = 0; i < 3 * N; ++i) Bnew[i] += P->dt * t[i];
  }
  if (walled(G))
    for (int64_t c = 0; c < N; ++c) {
      int ic[3]; unflat(G, c, ic);
      if (ic[0] == nxp(G))
        for (int m = 0; m < 3; ++m) Bnew[m * N + c] = Bc[m * N + c];  /* the ghost cell keeps its value */
    }
  free(t);
}

/* E^{n+1} from E^{n+theta} = (1 - theta) E^n + theta E^{n+1} (Sec. 2.1). */
void or_update_E(int64_t n3, double theta, const double* En, const double* Eth, double* Enew) {
  for (int64_t i = 0; i < n3; ++i) Enew[i] = (Eth[i] - (1.0 - theta) * En[i]) / theta;
}

/* ---------------------------------------------------------------------- */
/* Implicit mover (Sec. 3.1; READING of the time-centring, whose details the
 * paper leaves to the ECSIM reference): positions at n+1/2, velocities at n.
 *   vbar = alpha_p (v^n + beta_s E_p),  E_p = sum_g W_pg E^{n+theta}_g,
 *   v^{n+1} = 2 vbar - v^n,  x^{n+3/2} = x^{n+1/2} + dt v^{n+1}  (periodic).
 * alpha_p uses B at x^{n+1/2}, the same as in the deposit. */
void or_push_species(const or_grid* G, double beta_s, double dt, int64_t np, const double* x, const double* v,
                     const double* Eth, const double* Bn, double* xnew, double* vnew, int* keep) {
  for (int64_t p = 0; p < np; ++p) {
    if (keep) keep[p] = 1;
    int64_t nodes[8]; double W[8];
    int nc = or_shape(G, &x[3 * p], nodes, W);
    double Ep[3], Bp[3];
    gather(G, Eth, nodes, W, nc, Ep);
    gather(G, Bn, nodes, W, nc, Bp);
    double al[9]; or_alpha(beta_s, Bp, al);
    double t[3] = {v[3 * p] + beta_s * Ep[0], v[3 * p + 1] + beta_s * Ep[1], v[3 * p + 2] + beta_s * Ep[2]};
    double vb[3]; matvec3(al, t, vb);
    for (int d = 0; d < 3; ++d) {
      vnew[3 * p + d] = 2.0 * vb[d] - v[3 * p + d];
      double xn = x[3 * p + d];
      if (d == 0 && walled(G)) {
        /* READING: specular reflection on a wall (x -> -x, v_x -> -v_x about
           the wall plane); a particle crossing the inflow plane leaves */
        double L = nxp(G) * G->dx[0];
        xn += dt * vnew[3 * p];
        if (xn < 0.0) {
          xn = -xn;
          vnew[3 * p] = -vnew[3 * p];
        } else if (xn >= L) {
          if (G->bc_hi == OR_WALL) {
            xn = 2.0 * L - xn;
            vnew[3 * p] = -vnew[3 * p];
          } else if (keep) {
            keep[p] = 0;
          }
        }
      } else if (d < G->dim) {
        double L = G->n[d] * G->dx[d];
        xn += dt * vnew[3 * p + d];
        xn = fmod(xn, L);
        if (xn < 0.0) xn += L;
        if (xn >= L) xn -= L;
      }
      xnew[3 * p + d] = xn;
    }
  }
}

/* ---------------------------------------------------------------------- */
/* Restarted GMRES(m) with modified Gram-Schmidt and Givens rotations, all in
 * FP64, for A of or_apply_A.  Stops when ||b - A x|| <= tol ||b||, checked on
 * the true residual at each restart.  Returns iterations, or -1 if maxit was
 * reached. */
typedef struct { const or_grid* G; const or_params* P; const double* Mt; const double* kE; } opctx;
static void opA(const opctx* C, const double* x, double* y) { or_apply_A(C->G, C->P, C->Mt, C->kE, x, y); }
static double dot(int64_t n, const double* a, const double* b) {
  double s = 0.0;
  for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
  return s;
}

int or_gmres(const or_grid* G, const or_params* P, const double* Mtilde, const double* kappaE, const double* b,
             double* x, double tol, int maxit, int restart, double* relres_out) {
  opctx C = {G, P, Mtilde, kappaE};
  int64_t n = 3 * nnodes(G);
  int m = restart;
  double* V = (double*)malloc(sizeof(double) * n * (m + 1));
  double* H = (double*)calloc((size_t)(m + 1) * m, sizeof(double));
  double* cs = (double*)malloc(sizeof(double) * m);
  double* sn = (double*)malloc(sizeof(double) * m);
  double* s = (double*)malloc(sizeof(double) * (m + 1));
  double* r = (double*)malloc(sizeof(double) * n);
  double* w = (double*)malloc(sizeof(double) * n);
  double bn = sqrt(dot(n, b, b));
  if (bn == 0.0) bn = 1.0;
  int it = 0, conv = 0;
  double rel = 0.0;
  while (it < maxit) {
    opA(&C, x, r);
    for (int64_t i = 0; i < n; ++i) r[i] = b[i] - r[i];
    double beta = sqrt(dot(n, r, r));
    rel = beta / bn;
    if (rel <= tol) { conv = 1; break; }
    for (int64_t i = 0; i < n; ++i) V[i] = r[i] / beta;
    memset(s, 0, sizeof(double) * (m + 1));
    s[0] = beta;
    int j;
    for (j = 0; j < m && it < maxit; ++j, ++it) {
      opA(&C, &V[j * n], w);
      for (int i = 0; i <= j; ++i) {
        double h = dot(n, w, &V[i * n]);
        H[i * m + j] = h;
        for (int64_t k = 0; k < n; ++k) w[k] -= h * V[i * n + k];
      }
      double hn = sqrt(dot(n, w, w));
      H[(j + 1) * m + j] = hn;
      if (hn > 0.0)
        for (int64_t k = 0; k < n; ++k) V[(j + 1) * n + k] = w[k] / hn;
      for (int i = 0; i < j; ++i) {
        double t0 = cs[i] * H[i * m + j] + sn[i] * H[(i + 1) * m + j];
        double t1 = -sn[i] * H[i * m + j] + cs[i] * H[(i + 1) * m + j];
        H[i * m + j] = t0; H[(i + 1) * m + j] = t1;
      }
      double a = H[j * m + j], bb = H[(j + 1) * m + j];
      double den = sqrt(a * a + bb * bb);
      cs[j] = den > 0 ? a / den : 1.0;
      sn[j] = den > 0 ? bb / den : 0.0;
      H[j * m + j] = den; H[(j + 1) * m + j] = 0.0;
      s[j + 1] = -sn[j] * s[j];
      s[j] = cs[j] * s[j];
      if (fabs(s[j + 1]) / bn <= tol || hn == 0.0) { ++j; ++it; break; }
    }
    /* back substitution y = H^{-1} s, x += V y */
    int k = j;
    double* yv = (double*)malloc(sizeof(double) * (k > 0 ? k : 1));
    for (int i = k - 1; i >= 0; --i) {
      double t = s[i];
      for (int l = i + 1; l < k; ++l) t -= H[i * m + l] * yv[l];
      yv[i] = t / H[i * m + i];
    }
    for (int i = 0; i < k; ++i)
      for (int64_t q = 0; q < n; ++q) x[q] += yv[i] * V[i * n + q];
    free(yv);
  }
  if (!conv) {
    opA(&C, x, r);
    for (int64_t i = 0; i < n; ++i) r[i] = b[i] - r[i];
    rel = sqrt(dot(n, r, r)) / bn;
    conv = rel <= tol;
  }
  if (relres_out) *relres_out = rel;
  free(V); free(H); free(cs); free(sn); free(s); free(r); free(w);
  return conv ? it : -1;
}

/* Dense operator (columns = A applied to unit vectors) and a Gaussian
 * elimination solve with partial pivoting, for tiny grids only. */
void or_dense_A(const or_grid* G, const or_params* P, const double* Mtilde, const double* kappaE, double* Ad) {
  int64_t n = 3 * nnodes(G);
  double* e = (double*)calloc(n, sizeof(double));
  double* col = (double*)malloc(sizeof(double) * n);
  for (int64_t j = 0; j < n; ++j) {
    e[j] = 1.0;
    or_apply_A(G, P, Mtilde, kappaE, e, col);
    e[j] = 0.0;
    for (int64_t i = 0; i < n; ++i) Ad[i * n + j] = col[i];
  }
  free(e); free(col);
}

int or_dense_solve(int64_t n, const double* Ain, const double* b, double* x) {
  double* A = (double*)malloc(sizeof(double) * n * n);
  memcpy(A, Ain, sizeof(double) * n * n);
  memcpy(x, b, sizeof(double) * n);
  for (int64_t k = 0; k < n; ++k) {
    int64_t piv = k;
    for (int64_t i = k + 1; i < n; ++i)
      if (fabs(A[i * n + k]) > fabs(A[piv * n + k])) piv = i;
    if (A[piv * n + k] == 0.0) { free(A); return -1; }
    if (piv != k) {
      for (int64_t j = 0; j < n; ++j) { double t = A[k * n + j]; A[k * n + j] = A[piv * n + j]; A[piv * n + j] = t; }
      double t = x[k]; x[k] = x[piv]; x[piv] = t;
    }
    for (int64_t i = k + 1; i < n; ++i) {
      double f = A[i * n + k] / A[k * n + k];
      for (int64_t j = k; j < n; ++j) A[i * n + j] -= f * A[k * n + j];
      x[i] -= f * x[k];
    }
  }
  for (int64_t i = n - 1; i >= 0; --i) {
    double t = x[i];
    for (int64_t j = i + 1; j < n; ++j) t -= A[i * n + j] * x[j];
    x[i] = t / A[i * n + i];
  }
  free(A);
  return 0;
}

/* ---------------------------------------------------------------------- */
/* Scalar linear advection u_t + c u_x = 0 (c > 0) with the flux of Sec. 2.2:
 *   f_{i+1/2} = c (u_i + u_{i+1})/2 - (1 - phi_{i+1/2}) a/2 (u_{i+1} - u_i),
 * a = c, phi from the MC limiter with r = (u_i - u_{i-1})/(u_{i+1} - u_i);
 * forward Euler in time, periodic.  'phi_override' >= 0 fixes phi (1: FTCS). */
void or_advect(int n, double* u, double nu, double beta, int nsteps, double phi_override) {
  double* f = (double*)malloc(sizeof(double) * n);
  double* un = (double*)malloc(sizeof(double) * n);
  for (int s = 0; s < nsteps; ++s) {
    for (int i = 0; i < n; ++i) {
      int im = (i - 1 + n) % n, ip = (i + 1) % n;
      double phi = phi_override >= 0.0 ? phi_override : or_limiter(u[i] - u[im], u[ip] - u[i], beta);
      f[i] = 0.5 * (u[i] + u[ip]) - 0.5 * (1.0 - phi) * (u[ip] - u[i]); /* flux / c */
    }
    for (int i = 0; i < n; ++i) un[i] = u[i] - nu * (f[i] - f[(i - 1 + n) % n]);
    memcpy(u, un, sizeof(double) * n);
  }
  free(f); free(un);
}
