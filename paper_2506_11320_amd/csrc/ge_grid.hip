// Grid-side kernels of the GL-ECSIM step on gfx950: node assembly of the
// deposited sums, bulk velocity and its digital filter, motional field,
// comoving current, limited Lax-Friedrichs coefficients, right-hand side, the
// implicit E operator and the field updates.  Fields are FP64, [comp][N].
#include <cmath>
#include <cstring>

#include "ge_internal.h"

namespace {

constexpr double FOUR_PI = 12.566370614359172953850573533118;

template <int DIM>
struct Gd {
  static constexpr int NC = 1 << DIM;
  static constexpr int NR = DIM == 3 ? 27 : (DIM == 2 ? 9 : 3);
};

__device__ inline int ax_bit(int a, int d) { return (a >> d) & 1; }

// ----------------------------------------------------------------- node average of B
// value of component q of a cell field at cell (i, j, k), i possibly beyond
// a wall (mirror: odd components change sign)
__device__ inline double cellv(const DGrid& G, const double* __restrict__ F, int q, int i, int j, int k, bool odd) {
  double sg;
  const int im = cell_mirror(G, i, sg, odd);
  return sg * F[q * G.N + flat3(G, im, j, k)];
}

template <int DIM>
__global__ void k_node_avg(DGrid G, const double* __restrict__ B, double* __restrict__ Bn) {
  int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= G.N) return;
  if (walled(G)) {
    int gx, gy, gz;
    unflat3(G, g, gx, gy, gz);
    for (int q = 0; q < 3; ++q) {
      double s = 0;
      for (int a = 0; a < Gd<DIM>::NC; ++a)
        s += cellv(G, B, q, gx - ax_bit(a, 0), gy - (DIM >= 2 ? ax_bit(a, 1) : 0), gz - (DIM >= 3 ? ax_bit(a, 2) : 0),
                   q == 0);
      Bn[q * G.N + g] = s / Gd<DIM>::NC;
    }
    return;
  }
  for (int q = 0; q < 3; ++q) {
    double s = 0;
    for (int a = 0; a < Gd<DIM>::NC; ++a)
      s += B[q * G.N + nbr3(G, g, -ax_bit(a, 0), DIM >= 2 ? -ax_bit(a, 1) : 0, DIM >= 3 ? -ax_bit(a, 2) : 0)];
    s /= Gd<DIM>::NC;
    Bn[q * G.N + g] = s;
  }
}

// node8[g][4 half + q] = src[q][g] in the particle precision, [4 half + 3] = 0
template <typename T>
__global__ void k_pack_node8(int64_t N, const double* __restrict__ src, int half, T* __restrict__ node8) {
  int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= N) return;
  typedef T t4 __attribute__((ext_vector_type(4)));
  reinterpret_cast<t4*>(node8)[2 * g + half] = t4{(T)src[g], (T)src[N + g], (T)src[2 * N + g], (T)0};
}

// ----------------------------------------------------------------- assembly
// Sum the per-cell quadratic-row sums into the node-pair half stencil and the
// per-cell corner sums into nodes, in a fixed order (deterministic).  Node g
// and g + o are corners a and a + o of the cells g - a; that pair's weight
// product is quadratic row (2 a_d + o_d) along each axis d.
// Values k0 .. k0 + 8 of one cell's sums (qc = the cell's value 0), read as
// the 3 or 4 aligned 4-value vectors that hold them (k0 is a compile-time
// constant at every call, so the picks below are fixed register moves).
template <typename T>
__device__ inline void load_run9(const T* __restrict__ qc, int k0, T out[9]) {
  typedef T t4 __attribute__((ext_vector_type(4)));
  const int kb0 = k0 >> 2, nb = ((k0 + 8) >> 2) - kb0 + 1;
  t4 blk[4];
#pragma unroll
  for (int j = 0; j < 4; ++j)
    if (j < nb) blk[j] = *reinterpret_cast<const t4*>(qc + cq_off(4 * (kb0 + j)));
#pragma unroll
  for (int e = 0; e < 9; ++e) out[e] = blk[((k0 + e) >> 2) - kb0][(k0 + e) & 3];
}

template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_assemble(DGrid G, const T* __restrict__ Q, int Qn, int nsp, T* __restrict__ Mt,
                                                  T* __restrict__ M0, double* __restrict__ Jlab, double* __restrict__ mm,
                                                  double* __restrict__ mass, double* __restrict__ rho) {
  constexpr int NC = Gd<DIM>::NC, NR = Gd<DIM>::NR;
  using HS = HalfStencil<DIM>;
  const int64_t t = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (t >= G.N) return;
  const int64_t N = G.N;
  int gi, gj, gk;
  const int64_t g = visit_order(G, (unsigned)t, gi, gj, gk);
  int64_t cells[NC];
#pragma unroll
  for (int a = 0; a < NC; ++a)
    cells[a] = flat3(G, gi - ax_bit(a, 0), gj - (DIM >= 2 ? ax_bit(a, 1) : 0), gk - (DIM >= 3 ? ax_bit(a, 2) : 0));
#pragma unroll
  for (int h = 0; h < HS::NH; ++h) {
    double smt[9], sm0[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) smt[e] = sm0[e] = 0.0;
#pragma unroll
    for (int a = 0; a < NC; ++a) {
      bool ok = true;
      int r = 0, mul = 1;
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        const int bd = ax_bit(a, d) + HS::o[h][d];
        ok = ok && bd >= 0 && bd <= 1;
        r += (2 * ax_bit(a, d) + HS::o[h][d]) * mul;
        mul *= 3;
      }
      if (!ok) continue;
      const T* qc = Q + cq_index(cells[a], 0, Qn);
      T v[9];
      load_run9(qc, r * 9, v);
#pragma unroll
      for (int e = 0; e < 9; ++e) smt[e] += (double)v[e];
      load_run9(qc, 9 * NR + r * 9, v);
#pragma unroll
      for (int e = 0; e < 9; ++e) sm0[e] += (double)v[e];
    }
#pragma unroll
    for (int e = 0; e < 9; ++e) {
      Mt[(int64_t)(h * 9 + e) * N + g] = (T)smt[e];
      M0[(int64_t)(h * 9 + e) * N + g] = (T)sm0[e];
    }
  }
  const double idV = 1.0 / G.dV;
  const int NK = 7 + nsp;
  for (int k = 0; k < NK; ++k) {
    double s = 0;
#pragma unroll
    for (int a = 0; a < NC; ++a) s += (double)Q[cq_index(cells[a], 18 * NR + k * NC + a, Qn)];
    if (k < 3) Jlab[k * N + g] = s * idV;
    else if (k < 6) mm[(k - 3) * N + g] = s;
    else if (k == 6) mass[g] = s;
    else rho[(k - 7) * N + g] = s * idV;
  }
}

// ----------------------------------------------------------------- bulk velocity, filter, E_M
__global__ void k_bulk_u(int64_t N, const double* __restrict__ mm, const double* __restrict__ mass, double* __restrict__ u) {
  int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= N) return;
  double m = mass[g];
  for (int q = 0; q < 3; ++q) u[q * N + g] = m > 0 ? mm[q * N + g] / m : 0.0;
}

// One pass of the digital filter (Sec. 2.4) along 'axis' with stride d:
// v* = phi v + (1 - phi)/2 (v_{-d} + v_{+d}).
// Along a walled x axis the neighbours mirror about the wall planes; the
// field is a velocity or a current, whose normal (x) component is odd.
__global__ void k_filter(DGrid G, const double* __restrict__ src, double* __restrict__ dst, int axis, int d, double phi) {
  int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= G.N) return;
  const double half = 0.5 * (1.0 - phi);
  if (axis == 0 && walled(G)) {
    int gx, gy, gz;
    unflat3(G, g, gx, gy, gz);
    for (int q = 0; q < 3; ++q) {
      double sm, sp;
      const int im = node_mirror(G, gx - d, sm, q == 0), ip = node_mirror(G, gx + d, sp, q == 0);
      dst[q * G.N + g] = phi * src[q * G.N + g] +
                         half * (sm * src[q * G.N + flat3(G, im, gy, gz)] + sp * src[q * G.N + flat3(G, ip, gy, gz)]);
    }
    return;
  }
  int o[3] = {0, 0, 0};
  o[axis] = d;
  int64_t gp = nbr3(G, g, o[0], o[1], o[2]);
  int64_t gm = nbr3(G, g, -o[0], -o[1], -o[2]);
  for (int q = 0; q < 3; ++q) dst[q * G.N + g] = phi * src[q * G.N + g] + half * (src[q * G.N + gm] + src[q * G.N + gp]);
}

// E_M = -u x B (Sec. 3.1) and the diffusion speed at nodes (Sec. 2.2).
__global__ void k_motional(int64_t N, const double* __restrict__ u, const double* __restrict__ Bn, double* __restrict__ EM,
                           double* __restrict__ anode, int a_mode, double a_const) {
  int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= N) return;
  double ux = u[g], uy = u[N + g], uz = u[2 * N + g];
  double bx = Bn[g], by = Bn[N + g], bz = Bn[2 * N + g];
  EM[g] = -(uy * bz - uz * by);
  EM[N + g] = -(uz * bx - ux * bz);
  EM[2 * N + g] = -(ux * by - uy * bx);
  anode[g] = a_mode == GE_A_LIGHT ? a_const : sqrt(ux * ux + uy * uy + uz * uz);
}

// y_g = sum over the 3^DIM neighbours g' of M_{g,g'} x_{g'}, half stencil:
// the stored block at g serves offset +o, the block stored at g - o serves -o.
template <typename T, int DIM>
__device__ inline void apply_half(const DGrid& G, const T* __restrict__ M, const double* __restrict__ x, int64_t g,
                                  int gx, int gy, int gz, double y[3]) {
  using HS = HalfStencil<DIM>;
  const int64_t N = G.N;
  y[0] = y[1] = y[2] = 0;
#pragma unroll
  for (int h = 0; h < HS::NH; ++h) {
    const int64_t gp = flat3(G, gx + HS::o[h][0], gy + HS::o[h][1], gz + HS::o[h][2]);
    const double xp[3] = {x[gp], x[N + gp], x[2 * N + gp]};
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) y[i] += (double)M[(int64_t)(h * 9 + 3 * i + j) * N + g] * xp[j];
    if (h == 0) continue;
    const int64_t gm = flat3(G, gx - HS::o[h][0], gy - HS::o[h][1], gz - HS::o[h][2]);
    const double xm[3] = {x[gm], x[N + gm], x[2 * N + gm]};
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) y[i] += (double)M[(int64_t)(h * 9 + 3 * i + j) * N + gm] * xm[j];
  }
}

// J_eff = J_lab - (1/dV)(M0 u + Mtilde E_M)  (Sec. 3.1, comoving frame).
// PART 0: both terms, Jout = Jin - (1/dV)(M0 u + Mtilde E_M); PART 1: the
// comoving-frame current J_C = Jin - (1/dV) M0 u; PART 2: the E_M term alone,
// Jout = Jin - (1/dV) Mtilde E_M (J_C is smoothed between parts 1 and 2).
template <typename T, int DIM, int PART>
__global__ __launch_bounds__(256) void k_comoving(DGrid G, const T* __restrict__ Mt, const T* __restrict__ M0,
                                                  const double* __restrict__ u, const double* __restrict__ EM,
                                                  const double* __restrict__ Jin, double* __restrict__ Jout) {
  const int64_t t = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (t >= G.N) return;
  int gx, gy, gz;
  const int64_t g = visit_order(G, (unsigned)t, gx, gy, gz);
  double a[3] = {0, 0, 0}, b[3] = {0, 0, 0};
  if (PART != 2) apply_half<T, DIM>(G, M0, u, g, gx, gy, gz, a);
  if (PART != 1) apply_half<T, DIM>(G, Mt, EM, g, gx, gy, gz, b);
  const double idV = 1.0 / G.dV;
  for (int q = 0; q < 3; ++q) {
    const double corr = PART == 0 ? a[q] + b[q] : (PART == 1 ? a[q] : b[q]);
    Jout[q * G.N + g] = Jin[q * G.N + g] - idV * corr;
  }
}

// Divergence cleaning (Sec. 2.3): psi = (psi - dt c_h^2 div B) decay with the
// central-difference divergence of the cell-centred B at cell centres.
template <int DIM>
__global__ void k_dedner_psi(DGrid G, const double* __restrict__ B, double* __restrict__ psi, double dtch2,
                             double decay) {
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= G.N) return;
  double div = 0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const int64_t cp = nbr3(G, c, d == 0, d == 1, d == 2), cm = nbr3(G, c, -(d == 0), -(d == 1), -(d == 2));
    div += (B[d * G.N + cp] - B[d * G.N + cm]) / (2.0 * G.dx[d]);
  }
  psi[c] = (psi[c] - dtch2 * div) * decay;
}

// ----------------------------------------------------------------- limited LF coefficients
// Generalised MC limiter (Sec. 2.2) of r = num/den: max(0, min(beta r,
// (1+r)/2, beta)); den = 0 reads r = 1 (num = 0), +inf (num > 0) or -inf.
__device__ inline double mc_limiter(double num, double den, double beta) {
  double r;
  if (den == 0.0) {
    if (num == 0.0) r = 1.0;
    else return num > 0.0 ? beta : 0.0;
  } else {
    r = num / den;
  }
  double m = fmin(fmin(beta * r, 0.5 * (1.0 + r)), beta);
  return m > 0.0 ? m : 0.0;
}

// E: flux between node g and g + e_d (stored at g); ratio lagged to E^n.
// kEf (FP32 path, else null): the same values rounded to float, which the
// interior field operator reads (half the bytes per matvec).
template <int DIM>
__global__ void k_kappa_E(DGrid G, const double* __restrict__ E, const double* __restrict__ anode, double beta,
                          double* __restrict__ kE, float* __restrict__ kEf) {
  int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= G.N) return;
  const int64_t N = G.N;
  for (int d = 0; d < 3; ++d) {
    if (d >= DIM) {
      for (int m = 0; m < 3; ++m) {
        kE[(d * 3 + m) * N + g] = 0.0;
        if (kEf) kEf[(d * 3 + m) * N + g] = 0.0f;
      }
      continue;
    }
    int o[3] = {0, 0, 0};
    o[d] = 1;
    int64_t gp = nbr3(G, g, o[0], o[1], o[2]), gm = nbr3(G, g, -o[0], -o[1], -o[2]);
    double a = 0.5 * (anode[g] + anode[gp]);
    // walled x: no flux through the boundary planes; phi = 0 next to the lower wall
    int bx = -1;
    if (d == 0 && walled(G)) {
      int gy, gz;
      unflat3(G, g, bx, gy, gz);
      if (bx == G.nxp) a = 0.0;
    }
    for (int m = 0; m < 3; ++m) {
      double phi = mc_limiter(E[m * N + g] - E[m * N + gm], E[m * N + gp] - E[m * N + g], beta);
      if (bx == 0) phi = 0.0;
      const double k = 0.5 * (1.0 - phi) * a;
      kE[(d * 3 + m) * N + g] = k;
      if (kEf) kEf[(d * 3 + m) * N + g] = (float)k;
    }
  }
}

// B: face between cell c and c + e_d (stored at c); a = mean over the face's nodes.
template <int DIM>
__global__ void k_kappa_B(DGrid G, const double* __restrict__ B, const double* __restrict__ anode, double beta,
                          double* __restrict__ kB) {
  int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= G.N) return;
  const int64_t N = G.N;
  for (int d = 0; d < 3; ++d) {
    if (d >= DIM) {
      for (int m = 0; m < 3; ++m) kB[(d * 3 + m) * N + c] = 0.0;
      continue;
    }
    double asum = 0;
    int nf = 0;
    for (int t = 0; t < (1 << DIM); ++t) {
      if (ax_bit(t, d)) continue;
      int o[3] = {0, 0, 0};
      for (int e = 0; e < DIM; ++e) o[e] = ax_bit(t, e);
      o[d] = 1;
      asum += anode[nbr3(G, c, o[0], o[1], o[2])];
      ++nf;
    }
    double a = asum / nf;
    int o[3] = {0, 0, 0};
    o[d] = 1;
    int64_t cp = nbr3(G, c, o[0], o[1], o[2]), cm = nbr3(G, c, -o[0], -o[1], -o[2]);
    // walled x: no flux through the boundary faces nor on the ghost cells;
    // phi = 0 on the face next to the lower wall
    int bx = -1;
    if (walled(G)) {
      int cy, cz;
      unflat3(G, c, bx, cy, cz);
      if (bx >= G.nxp - (d == 0)) a = 0.0;
    }
    for (int m = 0; m < 3; ++m) {
      double phi = mc_limiter(B[m * N + c] - B[m * N + cm], B[m * N + cp] - B[m * N + c], beta);
      if (d == 0 && bx == 0) phi = 0.0;
      kB[(d * 3 + m) * N + c] = 0.5 * (1.0 - phi) * a;
    }
  }
}

// ----------------------------------------------------------------- curls
// Node -> cell derivative along d: difference of the means over the cell's
// upper and lower faces.  Cell -> node: difference of the means over the
// cells on the node's upper and lower side.
template <int DIM>
__global__ void k_curl_nc(DGrid G, const double* __restrict__ E, double* __restrict__ C) {
  int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= G.N) return;
  const int64_t N = G.N;
  constexpr int NC = Gd<DIM>::NC;
  double up[3][3] = {{0}}, lo[3][3] = {{0}};  // [axis][comp]
  for (int a = 0; a < NC; ++a) {
    int64_t g = nbr3(G, c, ax_bit(a, 0), DIM >= 2 ? ax_bit(a, 1) : 0, DIM >= 3 ? ax_bit(a, 2) : 0);
    double e0 = E[g], e1 = E[N + g], e2 = E[2 * N + g];
    for (int d = 0; d < DIM; ++d) {
      if (ax_bit(a, d)) { up[d][0] += e0; up[d][1] += e1; up[d][2] += e2; }
      else { lo[d][0] += e0; lo[d][1] += e1; lo[d][2] += e2; }
    }
  }
  double D[3][3] = {{0}};  // D[d][comp] = d comp / d x_d
  const double inv = 2.0 / NC;
  for (int d = 0; d < DIM; ++d)
    for (int q = 0; q < 3; ++q) D[d][q] = (up[d][q] - lo[d][q]) * inv * G.idx[d];
  C[c] = D[1][2] - D[2][1];
  C[N + c] = D[2][0] - D[0][2];
  C[2 * N + c] = D[0][1] - D[1][0];
  if (walled(G)) {
    int cx, cy, cz;
    unflat3(G, c, cx, cy, cz);
    if (cx == G.nxp) C[c] = C[N + c] = C[2 * N + c] = 0.0;  // the ghost cell
  }
}

template <int DIM>
__device__ inline void curl_cn_at(const DGrid& G, const double* __restrict__ B, int64_t g, double out[3]) {
  const int64_t N = G.N;
  constexpr int NC = Gd<DIM>::NC;
  double up[3][3] = {{0}}, lo[3][3] = {{0}};
  int gx = 0, gy = 0, gz = 0;
  const bool w = walled(G);
  if (w) unflat3(G, g, gx, gy, gz);
  for (int a = 0; a < NC; ++a) {
    double b0, b1, b2;
    if (w) {
      // cells beyond a wall are the mirror images (B_x odd, B_y, B_z even)
      const int ci = gx - ax_bit(a, 0), cj = gy - (DIM >= 2 ? ax_bit(a, 1) : 0), ck = gz - (DIM >= 3 ? ax_bit(a, 2) : 0);
      b0 = cellv(G, B, 0, ci, cj, ck, true);
      b1 = cellv(G, B, 1, ci, cj, ck, false);
      b2 = cellv(G, B, 2, ci, cj, ck, false);
    } else {
      int64_t cc = nbr3(G, g, -ax_bit(a, 0), DIM >= 2 ? -ax_bit(a, 1) : 0, DIM >= 3 ? -ax_bit(a, 2) : 0);
      b0 = B[cc]; b1 = B[N + cc]; b2 = B[2 * N + cc];
    }
    for (int d = 0; d < DIM; ++d) {
      if (ax_bit(a, d)) { lo[d][0] += b0; lo[d][1] += b1; lo[d][2] += b2; }
      else { up[d][0] += b0; up[d][1] += b1; up[d][2] += b2; }
    }
  }
  double D[3][3] = {{0}};
  const double inv = 2.0 / NC;
  for (int d = 0; d < DIM; ++d)
    for (int q = 0; q < 3; ++q) D[d][q] = (up[d][q] - lo[d][q]) * inv * G.idx[d];
  out[0] = D[1][2] - D[2][1];
  out[1] = D[2][0] - D[0][2];
  out[2] = D[0][1] - D[1][0];
}

// Diffusion term (D F)_g for component m: sum_d [k_g (F_{g+e}-F_g) - k_{g-e} (F_g - F_{g-e})] / dx_d
template <int DIM>
__device__ inline double diffusion_at(const DGrid& G, const double* __restrict__ kap, const double* __restrict__ F,
                                      int64_t g, int m) {
  const int64_t N = G.N;
  double s = 0;
  for (int d = 0; d < DIM; ++d) {
    int o[3] = {0, 0, 0};
    o[d] = 1;
    int64_t gp = nbr3(G, g, o[0], o[1], o[2]), gm = nbr3(G, g, -o[0], -o[1], -o[2]);
    double f0 = F[m * N + g];
    s += (kap[(d * 3 + m) * N + g] * (F[m * N + gp] - f0) - kap[(d * 3 + m) * N + gm] * (f0 - F[m * N + gm])) * G.idx[d];
  }
  return s;
}

// b = E^n + c theta dt curl_CN B^n - 4 pi theta dt J_eff
template <int DIM>
__global__ void k_rhs(DGrid G, const double* __restrict__ E, const double* __restrict__ B, const double* __restrict__ J,
                      double ctd, double ftd, double* __restrict__ b) {
  int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= G.N) return;
  double cb[3];
  curl_cn_at<DIM>(G, B, g, cb);
  int gx = -1, gy, gz;
  if (walled(G)) unflat3(G, g, gx, gy, gz);
  for (int q = 0; q < 3; ++q)
    b[q * G.N + g] = (gx >= 0 && held(G, gx, q)) ? E[q * G.N + g]  // E^{n+theta} = E^n on held components
                                                  : E[q * G.N + g] + ctd * cb[q] - ftd * J[q * G.N + g];
}

// curl_NC of a node field at physical cell (i, j, k)
template <int DIM>
__device__ inline void curl_nc_cell(const DGrid& G, const double* __restrict__ E, int i, int j, int k, double C[3]) {
  constexpr int NC = Gd<DIM>::NC;
  const int64_t N = G.N;
  double up[3][3] = {{0}}, lo[3][3] = {{0}};
  for (int a = 0; a < NC; ++a) {
    const int64_t g = flat3(G, i + ax_bit(a, 0), j + (DIM >= 2 ? ax_bit(a, 1) : 0), k + (DIM >= 3 ? ax_bit(a, 2) : 0));
    const double e[3] = {E[g], E[N + g], E[2 * N + g]};
    for (int d = 0; d < DIM; ++d)
      for (int q = 0; q < 3; ++q) (ax_bit(a, d) ? up : lo)[d][q] += e[q];
  }
  double D[3][3] = {{0}};
  const double inv = 2.0 / NC;
  for (int d = 0; d < DIM; ++d)
    for (int q = 0; q < 3; ++q) D[d][q] = (up[d][q] - lo[d][q]) * inv * G.idx[d];
  C[0] = D[1][2] - D[2][1];
  C[1] = D[2][0] - D[0][2];
  C[2] = D[0][1] - D[1][0];
}

// A x = x + (c theta dt)^2 curl_CN curl_NC x + (4 pi theta dt / dV) Mtilde x
//       - theta dt D_E x, in one pass over the 3^DIM neighbours of each node.
// curl_CN curl_NC is a constant 3^DIM-point stencil (a sum of tensor products
// of 1D differences and averages), precomputed on the host into K:
// K.k[o][3 m + j] multiplies x_j at offset o for output component m.
// curl_CN (curl_NC x) at an interior node as a 27-point stencil of 3x3
// blocks (Sec. 2.1 discretisation), built on the host (curl_curl_stencil)
struct CurlCurl {
  double k[27][9];
};

// A x at every node; on a walled x axis k_apply_A_planes then rewrites the
// rows of the two boundary node planes, where this kernel's periodic stencil
// does not apply.  Keeping the mirror-cell curl-curl out of this kernel, and
// this kernel free of an early exit, keeps it at 65 registers per thread.
template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_apply_A(DGrid G, const double* __restrict__ x, const T* __restrict__ Mt,
                                                 const T* __restrict__ kE, CurlCurl K, double k2, double mcoef,
                                                 double tdt, double* __restrict__ y) {
  const int64_t t = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  const int64_t N = G.N;
  if (t >= N) return;
  int gx, gy, gz;
  const int64_t g = visit_order(G, (unsigned)t, gx, gy, gz);
  double acc[3] = {x[g], x[N + g], x[2 * N + g]};
  const double x0[3] = {acc[0], acc[1], acc[2]};
  {
    constexpr int RY = DIM >= 2 ? 1 : 0, RZ = DIM >= 3 ? 1 : 0;
#pragma unroll
    for (int oz = -RZ; oz <= RZ; ++oz)
#pragma unroll
      for (int oy = -RY; oy <= RY; ++oy)
#pragma unroll
        for (int ox = -1; ox <= 1; ++ox) {
          const int oi = (ox + 1) + 3 * (oy + 1) + 9 * (oz + 1);
          const int64_t h = flat3(G, gx + ox, gy + oy, gz + oz);
          const double xv[3] = {x[h], x[N + h], x[2 * N + h]};
#pragma unroll
          for (int m = 0; m < 3; ++m)
            acc[m] += k2 * (K.k[oi][3 * m] * xv[0] + K.k[oi][3 * m + 1] * xv[1] + K.k[oi][3 * m + 2] * xv[2]);
        }
  }
  if (Mt) {
    double mx[3];
    apply_half<T, DIM>(G, Mt, x, g, gx, gy, gz, mx);
#pragma unroll
    for (int m = 0; m < 3; ++m) acc[m] += mcoef * mx[m];
  }
  if (kE) {
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const int64_t gp = flat3(G, gx + (d == 0), gy + (d == 1), gz + (d == 2));
      const int64_t gm = flat3(G, gx - (d == 0), gy - (d == 1), gz - (d == 2));
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        const double kp = (double)kE[(d * 3 + m) * N + g], km = (double)kE[(d * 3 + m) * N + gm];
        acc[m] -= tdt * G.idx[d] * (kp * (x[m * N + gp] - x0[m]) - km * (x0[m] - x[m * N + gm]));
      }
    }
  }
#pragma unroll
  for (int m = 0; m < 3; ++m) y[m * N + g] = acc[m];
}

// Rows of A x at the node planes x = 0 and x = nxp of a walled grid, written
// after k_apply_A.  Held components are identity rows (all three on an inflow
// plane, the tangential ones on a wall).  The normal row of a wall node takes
// curl_CN over the cells around the node, those beyond the wall being mirror
// images of curl_NC x (a pseudo-vector: x component odd; the ghost cell of an
// inflow plane carries zero), plus row 0 of the half-stencil mass term and
// the diffusion term.  The plane's nodes lie n[0] apart in memory, so each
// load touches its own cache line; 8 lanes share a node to keep many loads in
// flight: lane p takes cell p of the curl-curl, mass-matrix blocks p and
// p + 8 and, for p < DIM, the diffusion along axis p, and the 8 parts are
// summed in a fixed order.  One group of 8 lanes per node of the two planes.
template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_apply_A_planes(DGrid G, const double* __restrict__ x,
                                                        const T* __restrict__ Mt, const double* __restrict__ kE,
                                                        double k2, double mcoef, double tdt, double* __restrict__ y) {
  constexpr int NC = Gd<DIM>::NC;
  using HS = HalfStencil<DIM>;
  const int64_t N = G.N;
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int p = (int)(threadIdx.x & 7);
  const int64_t node = t >> 3, plane = (int64_t)G.n[1] * G.n[2];
  const bool live = node < 2 * plane;  // every lane takes part in the sums below
  const int64_t r = !live ? 0 : (node < plane ? node : node - plane);
  const int gx = live && node >= plane ? G.nxp : 0;
  const int gy = (int)(r % G.n[1]), gz = (int)(r / G.n[1]);
  const int64_t g = flat3(G, gx, gy, gz);
  const double x0 = x[g];
  double s = 0.0;
  if (live && !held(G, gx, 0)) {
    if (p < NC) {
      // cell p below/above the node along each axis; D[1][2] - D[2][1] of
      // curl_CN takes its curl with the sign of its side
      const int ci = gx - ax_bit(p, 0), cj = gy - (DIM >= 2 ? ax_bit(p, 1) : 0),
                ck = gz - (DIM >= 3 ? ax_bit(p, 2) : 0);
      double sg;
      const int cm = cell_mirror(G, ci, sg, true);
      if (cm < G.nxp) {
        double C[3];
        curl_nc_cell<DIM>(G, x, cm, cj, ck, C);  // C[0] (odd) is not used by the normal row
        const double inv = 2.0 / NC;
        double cc = 0.0;
        if (DIM >= 2) cc += (ax_bit(p, 1) ? -1.0 : 1.0) * C[2] * inv * G.idx[1];
        if (DIM >= 3) cc -= (ax_bit(p, 2) ? -1.0 : 1.0) * C[1] * inv * G.idx[2];
        s += k2 * cc;
      }
    }
    if (Mt) {
      double m0 = 0.0;
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const int h = p + 8 * k;
        if (h >= HS::NH) break;
        const int o0 = HS::o[h][0], o1 = HS::o[h][1], o2 = HS::o[h][2];
        const int64_t gp = flat3(G, gx + o0, gy + o1, gz + o2);
#pragma unroll
        for (int j = 0; j < 3; ++j) m0 += (double)Mt[(int64_t)(h * 9 + j) * N + g] * x[j * N + gp];
        if (h == 0) continue;
        const int64_t gm = flat3(G, gx - o0, gy - o1, gz - o2);
#pragma unroll
        for (int j = 0; j < 3; ++j) m0 += (double)Mt[(int64_t)(h * 9 + j) * N + gm] * x[j * N + gm];
      }
      s += mcoef * m0;
    }
    if (kE && p < DIM) {
      const int d = p;
      const int64_t gp = flat3(G, gx + (d == 0), gy + (d == 1), gz + (d == 2));
      const int64_t gm = flat3(G, gx - (d == 0), gy - (d == 1), gz - (d == 2));
      const double kp = kE[(d * 3) * N + g], km = kE[(d * 3) * N + gm];
      s -= tdt * G.idx[d] * (kp * (x[gp] - x0) - km * (x0 - x[gm]));
    }
  }
  s += __shfl_xor(s, 1);
  s += __shfl_xor(s, 2);
  s += __shfl_xor(s, 4);
  if (live && p == 0) {
    y[g] = x0 + s;  // s = 0 on a held row
    y[N + g] = x[N + g];
    y[2 * N + g] = x[2 * N + g];
  }
}

// B^{n+1} = B^n - c dt curl_NC E^{n+theta} + dt D_B B^n  (C holds curl_NC E^{n+theta})
template <int DIM>
__global__ void k_update_B(DGrid G, const double* __restrict__ B, const double* __restrict__ C,
                           const double* __restrict__ kB, const double* __restrict__ psi, double cdt, double dt,
                           double* __restrict__ Bnew) {
  int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= G.N) return;
  if (walled(G)) {
    int cx, cy, cz;
    unflat3(G, c, cx, cy, cz);
    if (cx == G.nxp) {  // the ghost cell keeps its (upstream) value
      for (int q = 0; q < 3; ++q) Bnew[q * G.N + c] = B[q * G.N + c];
      return;
    }
  }
  for (int q = 0; q < 3; ++q) {
    double v = B[q * G.N + c] - cdt * C[q * G.N + c];
    if (kB) v += dt * diffusion_at<DIM>(G, kB, B, c, q);
    if (psi && q < DIM) {
      // - dt grad psi^{n+1} (central difference at the cell centre)
      const int64_t cp = nbr3(G, c, q == 0, q == 1, q == 2), cm = nbr3(G, c, -(q == 0), -(q == 1), -(q == 2));
      v -= dt * ((psi[cp] - psi[cm]) / (2.0 * G.dx[q]));
    }
    Bnew[q * G.N + c] = v;
  }
}

__global__ void k_update_E(int64_t n3, double theta, const double* __restrict__ Eth, double* __restrict__ E) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n3) return;
  E[i] = (Eth[i] - (1.0 - theta) * E[i]) / theta;
}

// ----------------------------------------------------------------- Jacobi (node 3x3 diagonal block)
template <typename T, int DIM>
__global__ void k_jacobi_setup(DGrid G, const T* __restrict__ Mt, const double* __restrict__ kE, double k2, double mcoef,
                               double tdt, double* __restrict__ jac) {
  int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= G.N) return;
  const int64_t N = G.N;
  double A[9];
  for (int e = 0; e < 9; ++e) A[e] = Mt ? mcoef * (double)Mt[(int64_t)e * N + g] : 0.0;
  const double avg = 1.0 / (double)(1 << (DIM - 1));
  for (int m = 0; m < 3; ++m) {
    double cc = 0;
    for (int d = 0; d < DIM; ++d)
      if (d != m) cc += 2.0 * G.idx[d] * G.idx[d] * avg;
    double dd = 0;
    if (kE)
      for (int d = 0; d < DIM; ++d) {
        int o[3] = {0, 0, 0};
        o[d] = 1;
        int64_t gm = nbr3(G, g, -o[0], -o[1], -o[2]);
        dd += (kE[(d * 3 + m) * N + g] + kE[(d * 3 + m) * N + gm]) * G.idx[d];
      }
    A[4 * m] += 1.0 + k2 * cc + tdt * dd;
  }
  if (walled(G)) {
    int gx, gy, gz;
    unflat3(G, g, gx, gy, gz);
    if (gx == 0 || gx == G.nxp)  // boundary planes: the identity block (a preconditioner need not be exact)
      for (int e = 0; e < 9; ++e) A[e] = (e % 4 == 0) ? 1.0 : 0.0;
  }
  double det = A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) + A[2] * (A[3] * A[7] - A[4] * A[6]);
  double id = det != 0.0 ? 1.0 / det : 0.0;
  double I[9];
  I[0] = (A[4] * A[8] - A[5] * A[7]) * id;
  I[1] = (A[2] * A[7] - A[1] * A[8]) * id;
  I[2] = (A[1] * A[5] - A[2] * A[4]) * id;
  I[3] = (A[5] * A[6] - A[3] * A[8]) * id;
  I[4] = (A[0] * A[8] - A[2] * A[6]) * id;
  I[5] = (A[2] * A[3] - A[0] * A[5]) * id;
  I[6] = (A[3] * A[7] - A[4] * A[6]) * id;
  I[7] = (A[1] * A[6] - A[0] * A[7]) * id;
  I[8] = (A[0] * A[4] - A[1] * A[3]) * id;
  for (int e = 0; e < 9; ++e) jac[(int64_t)e * N + g] = I[e];
}

__global__ void k_jacobi_apply(int64_t N, const double* __restrict__ jac, const double* __restrict__ x, double* __restrict__ y) {
  int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= N) return;
  double a = x[g], b = x[N + g], c = x[2 * N + g];
  for (int i = 0; i < 3; ++i)
    y[i * N + g] = jac[(3 * i) * N + g] * a + jac[(3 * i + 1) * N + g] * b + jac[(3 * i + 2) * N + g] * c;
}

// ----------------------------------------------------------------- conversions and diagnostics
template <typename S, typename D>
__global__ void k_convert(const S* __restrict__ src, D* __restrict__ dst, int64_t n) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (D)src[i];
}

// block partials of |E|^2 (nodes), |B|^2 (cells), |div E - 4 pi rho_c|^2 and |4 pi rho_c|^2
template <int DIM>
__global__ __launch_bounds__(256) void k_field_diag(DGrid G, const double* __restrict__ E, const double* __restrict__ B,
                                                    const double* __restrict__ rho, int nsp, double* __restrict__ part) {
  __shared__ double sh[4][256];
  constexpr int NC = Gd<DIM>::NC;
  const int64_t N = G.N;
  double a[4] = {0, 0, 0, 0};
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < N; c += (int64_t)gridDim.x * blockDim.x) {
    // walled x: half weight of the boundary node planes, ghost cells left out
    double wn = 1.0;
    if (walled(G)) {
      int cx, cy, cz;
      unflat3(G, c, cx, cy, cz);
      if (cx == 0 || cx == G.nxp) wn = 0.5;
      if (cx == G.nxp) {
        for (int q = 0; q < 3; ++q) a[0] += wn * E[q * N + c] * E[q * N + c];
        continue;
      }
    }
    for (int q = 0; q < 3; ++q) {
      a[0] += wn * E[q * N + c] * E[q * N + c];
      a[1] += B[q * N + c] * B[q * N + c];
    }
    double up[3] = {0, 0, 0}, lo[3] = {0, 0, 0}, rc = 0;
    for (int k = 0; k < NC; ++k) {
      int64_t g = nbr3(G, c, ax_bit(k, 0), DIM >= 2 ? ax_bit(k, 1) : 0, DIM >= 3 ? ax_bit(k, 2) : 0);
      for (int d = 0; d < DIM; ++d) {
        if (ax_bit(k, d)) up[d] += E[d * N + g];
        else lo[d] += E[d * N + g];
      }
      for (int s = 0; s < nsp; ++s) rc += rho[s * N + g];
    }
    double div = 0;
    for (int d = 0; d < DIM; ++d) div += (up[d] - lo[d]) * (2.0 / NC) * G.idx[d];
    double r4 = FOUR_PI * rc / NC;
    a[2] += (div - r4) * (div - r4);
    a[3] += r4 * r4;
  }
  for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] = a[k];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s)
      for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x < 4) part[threadIdx.x * gridDim.x + blockIdx.x] = sh[threadIdx.x][0];
}

inline dim3 grid1(int64_t n) { return dim3((unsigned)((n + 255) / 256)); }

}  // namespace

// ===================================================================== host
#define DISPATCH_DIM(c, KERNEL, ...)                                                                     \
  switch ((c)->G.dim) {                                                                                  \
    case 1: hipLaunchKernelGGL(KERNEL<1>, __VA_ARGS__); break;                                           \
    case 2: hipLaunchKernelGGL(KERNEL<2>, __VA_ARGS__); break;                                           \
    default: hipLaunchKernelGGL(KERNEL<3>, __VA_ARGS__); break;                                          \
  }

int ge_launch_node_avg(ge_ctx* c) {
  DISPATCH_DIM(c, k_node_avg, grid1(c->G.N), dim3(256), 0, c->stream, c->G, c->B, c->Bn);
  GE_HIP(c, hipGetLastError());
  return ge_launch_pack_node8(c, 1);
}

int ge_launch_pack_node8(ge_ctx* c, int half) {
  const double* src = half ? c->Bn : c->Eth;
  if (c->P.precision == GE_FP32)
    hipLaunchKernelGGL(k_pack_node8<float>, grid1(c->G.N), dim3(256), 0, c->stream, c->G.N, src, half, (float*)c->node8);
  else
    hipLaunchKernelGGL(k_pack_node8<double>, grid1(c->G.N), dim3(256), 0, c->stream, c->G.N, src, half,
                       (double*)c->node8);
  GE_HIP(c, hipGetLastError());
  return GE_OK;
}

template <typename T, int DIM>
static void assemble_t(ge_ctx* c) {
  hipLaunchKernelGGL((k_assemble<T, DIM>), grid1(c->G.N), dim3(256), 0, c->stream, c->G, (const T*)c->cellQ, c->Q,
                     c->nsp, (T*)c->Mt, (T*)c->M0, c->Jlab, c->mm, c->mass, c->rho);
}
// ns_j filter passes (stride 1, weight phi_u; x, then y, then z) on c->Jeff,
// ping-ponging with c->utmp (free once u is smoothed)
static void smooth_current(ge_ctx* c) {
  for (int k = 0; k < c->P.ns_j; ++k)
    for (int ax = 0; ax < c->G.dim; ++ax) {
      hipLaunchKernelGGL(k_filter, grid1(c->G.N), dim3(256), 0, c->stream, c->G, c->Jeff, c->utmp, ax, 1, c->P.phi_u);
      std::swap(c->Jeff, c->utmp);
    }
}

template <typename T, int DIM>
static void comoving_t(ge_ctx* c) {
  if (c->P.ns_j == 0) {
    hipLaunchKernelGGL((k_comoving<T, DIM, 0>), grid1(c->G.N), dim3(256), 0, c->stream, c->G, (const T*)c->Mt,
                       (const T*)c->M0, c->u, c->EM, c->Jlab, c->Jeff);
    return;
  }
  hipLaunchKernelGGL((k_comoving<T, DIM, 1>), grid1(c->G.N), dim3(256), 0, c->stream, c->G, (const T*)c->Mt,
                     (const T*)c->M0, c->u, c->EM, c->Jlab, c->Jeff);
  smooth_current(c);
  hipLaunchKernelGGL((k_comoving<T, DIM, 2>), grid1(c->G.N), dim3(256), 0, c->stream, c->G, (const T*)c->Mt,
                     (const T*)c->M0, c->u, c->EM, c->Jeff, c->utmp);
  std::swap(c->Jeff, c->utmp);
}
#define DISPATCH_TD(c, FN)                                          \
  switch ((c)->G.dim * 2 + ((c)->P.precision == GE_FP32 ? 1 : 0)) { \
    case 2: FN<double, 1>(c); break;                                \
    case 3: FN<float, 1>(c); break;                                 \
    case 4: FN<double, 2>(c); break;                                \
    case 5: FN<float, 2>(c); break;                                 \
    case 6: FN<double, 3>(c); break;                                \
    default: FN<float, 3>(c); break;                                \
  }

// Bulk velocity u = mm / mass, then the filter passes: strides 1, 2, 1, 2, ...;
// each pass sweeps x, then y, then z.
int ge_launch_bulk_velocity(ge_ctx* c) {
  const DGrid& G = c->G;
  const int64_t N = G.N;
  hipLaunchKernelGGL(k_bulk_u, grid1(N), dim3(256), 0, c->stream, N, c->mm, c->mass, c->u);
  for (int k = 0; k < c->P.n_smooth_u; ++k)
    for (int ax = 0; ax < G.dim; ++ax) {
      hipLaunchKernelGGL(k_filter, grid1(N), dim3(256), 0, c->stream, G, c->u, c->utmp, ax, (k % 2 == 0) ? 1 : 2,
                         c->P.phi_u);
      std::swap(c->u, c->utmp);
    }
  GE_HIP(c, hipGetLastError());
  return GE_OK;
}

// Leapfrog of the explicit step: B^{n+1/2} = B^n - (c dt/2) curl_NC E^n,
// E^{n+1} = E^n + c dt curl_CN B^{n+1/2} - 4 pi dt J (J in c->Jeff),
// B^{n+1} = B^{n+1/2} - (c dt/2) curl_NC E^{n+1}.  c->Eth and c->Bnew are
// scratch here.
int ge_launch_explicit_fields(ge_ctx* c) {
  const int64_t N = c->G.N;
  const double cdt = c->P.c * c->P.dt;
  DISPATCH_DIM(c, k_curl_nc, grid1(N), dim3(256), 0, c->stream, c->G, c->E, c->ccell);
  DISPATCH_DIM(c, k_update_B, grid1(N), dim3(256), 0, c->stream, c->G, c->B, c->ccell, nullptr, nullptr, 0.5 * cdt,
               c->P.dt, c->Bnew);
  DISPATCH_DIM(c, k_rhs, grid1(N), dim3(256), 0, c->stream, c->G, c->E, c->Bnew, c->Jeff, cdt,
               4.0 * M_PI * c->P.dt, c->Eth);
  std::swap(c->E, c->Eth);
  DISPATCH_DIM(c, k_curl_nc, grid1(N), dim3(256), 0, c->stream, c->G, c->E, c->ccell);
  DISPATCH_DIM(c, k_update_B, grid1(N), dim3(256), 0, c->stream, c->G, c->Bnew, c->ccell, nullptr, nullptr, 0.5 * cdt,
               c->P.dt, c->B);
  GE_HIP(c, hipGetLastError());
  return GE_OK;
}

int ge_launch_smooth_current(ge_ctx* c) {
  smooth_current(c);
  GE_HIP(c, hipGetLastError());
  return GE_OK;
}

// Everything between the particle deposit and the linear solve.
// LF coefficients of the E operator from the field E (E^n in the grid pass,
// the first E^{n+theta} for the Picard step of the limiter)
int ge_launch_kappa_E(ge_ctx* c, const double* E) {
  DISPATCH_DIM(c, k_kappa_E, grid1(c->G.N), dim3(256), 0, c->stream, c->G, E, c->anode, c->P.beta_lim, c->kE, c->kEf);
  GE_HIP(c, hipGetLastError());
  return GE_OK;
}

int ge_launch_grid_pass(ge_ctx* c) {
  const DGrid& G = c->G;
  const int64_t N = G.N;
  (void)hipEventRecord(c->ev[4], c->stream);
  DISPATCH_TD(c, assemble_t);
  GE_HIP(c, hipGetLastError());
  (void)hipEventRecord(c->ev[5], c->stream);
  (void)hipEventRecord(c->ev[6], c->stream);
  ge_launch_bulk_velocity(c);
  hipLaunchKernelGGL(k_motional, grid1(N), dim3(256), 0, c->stream, N, c->u, c->Bn, c->EM, c->anode, c->P.a_mode,
                     c->P.a_const);
  if (c->P.comoving) {
    DISPATCH_TD(c, comoving_t);
  } else {
    GE_HIP(c, hipMemcpyAsync(c->Jeff, c->Jlab, sizeof(double) * 3 * N, hipMemcpyDeviceToDevice, c->stream));
    smooth_current(c);
  }
  if (c->P.lf_E)
    DISPATCH_DIM(c, k_kappa_E, grid1(N), dim3(256), 0, c->stream, G, c->E, c->anode, c->P.beta_lim, c->kE, c->kEf);
  if (c->P.lf_B) DISPATCH_DIM(c, k_kappa_B, grid1(N), dim3(256), 0, c->stream, G, c->B, c->anode, c->P.beta_lim, c->kB);
  const double ctd = c->P.c * c->P.theta * c->P.dt, ftd = 4.0 * M_PI * c->P.theta * c->P.dt;
  DISPATCH_DIM(c, k_rhs, grid1(N), dim3(256), 0, c->stream, G, c->E, c->B, c->Jeff, ctd, ftd, c->rhs);
  GE_HIP(c, hipGetLastError());
  (void)hipEventRecord(c->ev[7], c->stream);
  return GE_OK;
}

// Stencil of curl_CN curl_NC: sum over d != m of D_CN,d D_NC,m (x_d) minus
// D_CN,d D_NC,d (x_m).  Each D_CN,a D_NC,b is a tensor product of 1D stencils:
// along a == b the second difference [1,-2,1]/dx^2; along a != b the centred
// difference [-1,0,1]/(2 dx) on both axes a and b; the average [1,2,1]/4
// along every other active axis.
static CurlCurl curl_curl_stencil(const DGrid& G) {
  CurlCurl K;
  std::memset(&K, 0, sizeof(K));
  const int dim = G.dim;
  auto s1 = [&](int axis, int a, int b, int o) -> double {  // 1D factor of D_CN,a D_NC,b along axis
    if (axis >= dim) return o == 0 ? 1.0 : 0.0;
    const double ih = G.idx[axis];
    if (axis == a && axis == b) return (o == 0 ? -2.0 : 1.0) * ih * ih;
    if (axis == a || axis == b) return o == 0 ? 0.0 : 0.5 * o * ih;
    return o == 0 ? 0.5 : 0.25;
  };
  auto prod = [&](int a, int b, int ox, int oy, int oz) {
    return s1(0, a, b, ox) * s1(1, a, b, oy) * s1(2, a, b, oz);
  };
  for (int oz = -1; oz <= 1; ++oz)
    for (int oy = -1; oy <= 1; ++oy)
      for (int ox = -1; ox <= 1; ++ox) {
        const int oi = (ox + 1) + 3 * (oy + 1) + 9 * (oz + 1);
        for (int m = 0; m < 3; ++m)
          for (int d = 0; d < dim; ++d) {
            if (d == m) continue;
            K.k[oi][3 * m + m] -= prod(d, d, ox, oy, oz);
            if (m < dim) K.k[oi][3 * m + d] += prod(d, m, ox, oy, oz);
          }
      }
  return K;
}

template <typename T, int DIM>
static void apply_t(ge_ctx* c, const double* x, double* y) {
  const double ctd = c->P.c * c->P.theta * c->P.dt;
  const double mcoef = 4.0 * M_PI * c->P.theta * c->P.dt / c->G.dV;
  const T* Mt = c->have_deposit ? (const T*)c->Mt : nullptr;
  const double* kE = c->P.lf_E ? c->kE : nullptr;
  // the interior operator reads the coefficients in the matrices' type
  const T* kEt = c->P.lf_E ? (sizeof(T) == 4 ? (const T*)(const void*)c->kEf : (const T*)(const void*)c->kE) : nullptr;
  const CurlCurl K = curl_curl_stencil(c->G);
  hipLaunchKernelGGL((k_apply_A<T, DIM>), grid1(c->G.N), dim3(256), 0, c->stream, c->G, x, Mt, kEt, K, ctd * ctd,
                     mcoef, c->P.theta * c->P.dt, y);
  if (walled(c->G))
    hipLaunchKernelGGL((k_apply_A_planes<T, DIM>), grid1(16 * (int64_t)c->G.n[1] * c->G.n[2]), dim3(256), 0,
                       c->stream, c->G, x, Mt, kE, ctd * ctd, mcoef, c->P.theta * c->P.dt, y);
}
int ge_launch_apply_A(ge_ctx* c, const double* x, double* y) {
  switch (c->G.dim * 2 + (c->P.precision == GE_FP32 ? 1 : 0)) {
    case 2: apply_t<double, 1>(c, x, y); break;
    case 3: apply_t<float, 1>(c, x, y); break;
    case 4: apply_t<double, 2>(c, x, y); break;
    case 5: apply_t<float, 2>(c, x, y); break;
    case 6: apply_t<double, 3>(c, x, y); break;
    default: apply_t<float, 3>(c, x, y); break;
  }
  GE_HIP(c, hipGetLastError());
  return GE_OK;
}

int ge_launch_update(ge_ctx* c) {
  const int64_t N = c->G.N;
  (void)hipEventRecord(c->ev[8], c->stream);
  DISPATCH_DIM(c, k_curl_nc, grid1(N), dim3(256), 0, c->stream, c->G, c->Eth, c->ccell);
  if (c->P.dedner) {
    double dxmin = c->G.dx[0];
    for (int d = 1; d < c->G.dim; ++d) dxmin = std::min(dxmin, c->G.dx[d]);
    const double ch = c->P.ch_frac * dxmin / c->P.dt;
    DISPATCH_DIM(c, k_dedner_psi, grid1(N), dim3(256), 0, c->stream, c->G, c->B, c->psi, c->P.dt * ch * ch,
                 std::exp(-c->P.dedner_damp));
  }
  DISPATCH_DIM(c, k_update_B, grid1(N), dim3(256), 0, c->stream, c->G, c->B, c->ccell, c->P.lf_B ? c->kB : nullptr,
               c->P.dedner ? c->psi : nullptr, c->P.c * c->P.dt, c->P.dt, c->Bnew);
  std::swap(c->B, c->Bnew);
  hipLaunchKernelGGL(k_update_E, grid1(3 * N), dim3(256), 0, c->stream, 3 * N, c->P.theta, c->Eth, c->E);
  // optional E smoothing: strides 1, 2, 1, ...; x, then y, then z per pass;
  // c->utmp is free between grid passes
  for (int k = 0; k < c->P.ns_e; ++k)
    for (int ax = 0; ax < c->G.dim; ++ax) {
      hipLaunchKernelGGL(k_filter, grid1(N), dim3(256), 0, c->stream, c->G, c->E, c->utmp, ax, (k % 2 == 0) ? 1 : 2,
                         c->P.phi_u);
      std::swap(c->E, c->utmp);
    }
  GE_HIP(c, hipGetLastError());
  (void)hipEventRecord(c->ev[9], c->stream);
  return GE_OK;
}

int ge_launch_widen_M(ge_ctx* c, const void* M, double* dst) {
  const int64_t n = (int64_t)c->nh * 9 * c->G.N;
  if (c->P.precision == GE_FP32)
    hipLaunchKernelGGL((k_convert<float, double>), grid1(n), dim3(256), 0, c->stream, (const float*)M, dst, n);
  else
    GE_HIP(c, hipMemcpyAsync(dst, M, sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream));
  GE_HIP(c, hipGetLastError());
  return GE_OK;
}

template <typename T, int DIM>
static void jac_t(ge_ctx* c) {
  const double ctd = c->P.c * c->P.theta * c->P.dt;
  const double mcoef = 4.0 * M_PI * c->P.theta * c->P.dt / c->G.dV;
  hipLaunchKernelGGL((k_jacobi_setup<T, DIM>), grid1(c->G.N), dim3(256), 0, c->stream, c->G,
                     c->have_deposit ? (const T*)c->Mt : nullptr, c->P.lf_E ? c->kE : nullptr, ctd * ctd, mcoef,
                     c->P.theta * c->P.dt, c->jac);
}
int ge_launch_jacobi_setup(ge_ctx* c) {
  DISPATCH_TD(c, jac_t);
  GE_HIP(c, hipGetLastError());
  return GE_OK;
}
int ge_launch_jacobi_apply(ge_ctx* c, const double* x, double* y) {
  hipLaunchKernelGGL(k_jacobi_apply, grid1(c->G.N), dim3(256), 0, c->stream, c->G.N, c->jac, x, y);
  GE_HIP(c, hipGetLastError());
  return GE_OK;
}

namespace {
__global__ void k_sub_vec(int64_t n, const double* __restrict__ a, const double* __restrict__ b, double* __restrict__ o) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) o[i] = a[i] - b[i];
}
}  // namespace
int ge_launch_sub(ge_ctx* c, const double* a, const double* b, double* out, int64_t n) {
  hipLaunchKernelGGL(k_sub_vec, grid1(n), dim3(256), 0, c->stream, n, a, b, out);
  GE_HIP(c, hipGetLastError());
  return GE_OK;
}

// k_field_diag into part[4][GE_DIAG_BLOCKS] (block partials of |E|^2, |B|^2 and
// the two Gauss-residual sums)
int ge_launch_field_diag_part(ge_ctx* c, double* part) {
  DISPATCH_DIM(c, k_field_diag, dim3(GE_DIAG_BLOCKS), dim3(256), 0, c->stream, c->G, c->E, c->B, c->rho, c->nsp, part);
  GE_HIP(c, hipGetLastError());
  return GE_OK;
}

int ge_launch_field_diag(ge_ctx* c, double* out) {
  const int nbk = GE_DIAG_BLOCKS;
  int rc = ge_launch_field_diag_part(c, c->partials);
  if (rc) return rc;
  double h[4 * 256];
  GE_HIP(c, hipMemcpyAsync(h, c->partials, sizeof(double) * 4 * nbk, hipMemcpyDeviceToHost, c->stream));
  GE_HIP(c, hipStreamSynchronize(c->stream));
  for (int k = 0; k < 4; ++k) {
    double a = 0;
    for (int b = 0; b < nbk; ++b) a += h[k * nbk + b];
    out[k] = a;
  }
  return GE_OK;
}
