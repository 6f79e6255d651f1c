/*
 * Seeded synthetic inputs for the GL-ECSIM particle pass.
 *
 * This file holds no arithmetic of the PIC method itself: it only turns
 * counters into particle positions, velocities and weights, and evaluates the
 * analytic initial conditions (density, drift, fields) of the workloads.
 * Both the CPU oracle and the GPU path take their inputs from here, so that
 * neither side ever feeds the other.
 *
 * Random numbers: Philox4x32-10, the counter-based generator of
 * Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as easy as 1, 2, 3"
 * (SC'11), written from its published definition.  Each particle is keyed by
 * (seed, stream) and counted by (cell, k, species, call), so any cell's
 * particles can be regenerated alone, in any order and on any thread.
 * Normal deviates: the Box-Muller transform; the thermal velocity vector is
 * truncated at |n| <= RCLIP (its length, so that gyration cannot rotate a
 * clipped tail into a faster component), which keeps every electron of the
 * workloads well below the speed of light of this non-relativistic mover.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u
#define RCLIP 4.5
#define TWO_PI 6.283185307179586476925286766559

void synth_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
  uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int r = 0; r < 10; ++r) {
    uint64_t p0 = (uint64_t)PHILOX_M0 * c0;
    uint64_t p1 = (uint64_t)PHILOX_M1 * c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    k0 += PHILOX_W0; k1 += PHILOX_W1;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* uniform in the open interval (0,1), 32-bit resolution, exact in FP64 */
static inline double u01(uint32_t u) { return ((double)u + 0.5) * 2.3283064365386962890625e-10; }
/* uniform in (0,1) on the grid (2k+1)/2^24, k < 2^23: exactly representable
 * in FP32 and FP64, never 0 or 1, so an FP32 copy of a cell offset is exact
 * and stays in [0,1) */
static inline double u01_24(uint32_t u) { return (double)(u >> 9) * 1.1920928955078125e-07 + 5.9604644775390625e-08; }

enum { PROF_UNIFORM = 0, PROF_SHOCK_TUBE = 1, PROF_HARRIS2 = 2 };

/* Description of one workload's initial state (all normalised units:
 * c = 1, e = 1, m_e = 1, n0 = 1/(4 pi) so that omega_pe = d_e = 1). */
typedef struct {
  int dim;
  int n[3];
  double dx[3];
  int ppc;            /* macro-particles per cell per species */
  int nsp;            /* number of species (<= 4) */
  double q[4], m[4], vth[4];
  int paired;         /* 1: all species share positions (zero net charge) */
  uint32_t seed;
  int profile;
  double n0;          /* reference density */
  double u0[3];       /* uniform drift added to every species */
  double ushock;      /* shock tube: +ushock for x < L/2, -ushock otherwise */
  double B0[3];       /* uniform magnetic field (UNIFORM, SHOCK_TUBE) */
  double lambda;      /* Harris half-width */
  double nb;          /* Harris background density (fraction of n0) */
  double Bh;          /* Harris asymptotic field */
  double psi;         /* perturbation amplitude (flux units) */
  double dsheet[4];   /* per-species drift speed along z inside sheet 1 */
  int ghost_x;        /* 1: x ends in walls; the last x cell (index n[0]-1) is a ghost cell */
  double dt_inj;      /* time step of the inflow injection (synth_inflow) */
} synth_cfg;

static void domain_len(const synth_cfg* c, double L[3]) {
  for (int d = 0; d < 3; ++d) L[d] = (d < c->dim) ? c->n[d] * c->dx[d] : 1.0;
}

/* Harris double sheet at y = Ly/4 and y = 3Ly/4.  Across sheet 1 B_x rises
 * (B_x ~ Bh tanh((y - y1)/lambda)), so (curl B)_z = -dB_x/dy < 0 there and the
 * current that Ampere's law asks for, sum_s q_s n u_s = (c/4 pi) curl B, points
 * along -z; sheet 2 carries the opposite current. */
static void harris_parts(const synth_cfg* c, double y, double* n1, double* n2, double* nbk) {
  double L[3]; domain_len(c, L);
  double y1 = 0.25 * L[1], y2 = 0.75 * L[1];
  double s1 = 1.0 / cosh((y - y1) / c->lambda), s2 = 1.0 / cosh((y - y2) / c->lambda);
  *n1 = c->n0 * s1 * s1;
  *n2 = c->n0 * s2 * s2;
  *nbk = c->n0 * c->nb;
}

double synth_density(const synth_cfg* c, const double x[3]) {
  if (c->profile == PROF_HARRIS2) {
    double n1, n2, nb; harris_parts(c, x[1], &n1, &n2, &nb);
    return n1 + n2 + nb;
  }
  return c->n0;
}

/* Drift of species s for a particle at x; 'pick' in (0,1) selects which
 * Harris population the particle belongs to (density-weighted). */
static void drift(const synth_cfg* c, int s, const double x[3], double pick, double u[3]) {
  double L[3]; domain_len(c, L);
  u[0] = c->u0[0]; u[1] = c->u0[1]; u[2] = c->u0[2];
  if (c->profile == PROF_SHOCK_TUBE) {
    u[0] += (x[0] < 0.5 * L[0]) ? c->ushock : -c->ushock;
  } else if (c->profile == PROF_HARRIS2) {
    double n1, n2, nb; harris_parts(c, x[1], &n1, &n2, &nb);
    double nt = n1 + n2 + nb;
    /* dsheet[s] is the drift of species s along +z that carries a current
     * along +z (ions positive, electrons negative); sheet 1 takes it reversed */
    if (pick * nt < n1) u[2] -= c->dsheet[s];
    else if (pick * nt < n1 + n2) u[2] += c->dsheet[s];
  }
}

static void normals4(const uint32_t r[4], double nout[4]) {
  for (int j = 0; j < 2; ++j) {
    double a = u01(r[2 * j]), b = u01(r[2 * j + 1]);
    double rad = sqrt(-2.0 * log(a));
    nout[2 * j] = rad * cos(TWO_PI * b);
    nout[2 * j + 1] = rad * sin(TWO_PI * b);
  }
}

int64_t synth_ncells(const synth_cfg* c) {
  int64_t nc = 1;
  for (int d = 0; d < c->dim; ++d) nc *= c->n[d];
  return nc;
}

/*
 * Particles of species s in cells [cb, ce) (linear index i + nx*(j + ny*k)),
 * ppc per cell, cell-major then k.  Outputs (stride = count):
 *   cell[p] (int32), off[d*stride + p] (offset in the cell, in (0,1)),
 *   v[d*stride + p], w[p].  Offsets of inactive axes are 0.
 * If f32 != 0 the float outputs are written as float, else double.
 * Returns the number of particles written.
 */
/* ghost cells (x index n[0]-1 of a walled grid) among the linear cells [0, a) */
static int64_t ghosts_before(const synth_cfg* c, int64_t a) {
  return c->ghost_x ? a / c->n[0] : 0;
}

int64_t synth_particles(const synth_cfg* c, int s, int64_t cb, int64_t ce, int32_t* cell,
                        void* off, void* v, void* w, int f32) {
  int64_t count = (ce - cb - (ghosts_before(c, ce) - ghosts_before(c, cb))) * (int64_t)c->ppc;
  double dV = 1.0;
  for (int d = 0; d < c->dim; ++d) dV *= c->dx[d];
  #pragma omp parallel for schedule(static)
  for (int64_t cc = cb; cc < ce; ++cc) {
    int64_t ic[3] = {0, 0, 0}, rem = cc;
    for (int d = 0; d < c->dim; ++d) { ic[d] = rem % c->n[d]; rem /= c->n[d]; }
    if (c->ghost_x && ic[0] == c->n[0] - 1) continue;  /* no particles in a ghost cell */
    const int64_t slot = cc - cb - (ghosts_before(c, cc) - ghosts_before(c, cb));
    for (int k = 0; k < c->ppc; ++k) {
      int64_t p = slot * c->ppc + k;
      uint32_t key[2] = {c->seed, 0x9A1Eu};
      uint32_t ca[4] = {(uint32_t)cc, (uint32_t)k, c->paired ? 0u : (uint32_t)(s + 1), 0x50u};
      uint32_t cv[4] = {(uint32_t)cc, (uint32_t)k, (uint32_t)(s + 1), 0x56u};
      uint32_t ra[4], rv[4];
      synth_philox4x32_10(ca, key, ra);
      synth_philox4x32_10(cv, key, rv);
      double f[3] = {0, 0, 0}, x[3] = {0, 0, 0};
      for (int d = 0; d < c->dim; ++d) {
        f[d] = u01_24(ra[d]);
        x[d] = ((double)ic[d] + f[d]) * c->dx[d];
      }
      double u[3]; drift(c, s, x, u01(ra[3]), u);
      double nn[4]; normals4(rv, nn);
      double r2 = nn[0] * nn[0] + nn[1] * nn[1] + nn[2] * nn[2];
      if (r2 > RCLIP * RCLIP) {
        double sc = RCLIP / sqrt(r2);
        nn[0] *= sc; nn[1] *= sc; nn[2] *= sc;
      }
      double vv[3];
      for (int d = 0; d < 3; ++d) vv[d] = u[d] + c->vth[s] * nn[d];
      double ww = synth_density(c, x) * dV / c->ppc;
      cell[p] = (int32_t)cc;
      if (f32) {
        float* fo = (float*)off; float* fv = (float*)v; float* fw = (float*)w;
        for (int d = 0; d < 3; ++d) { fo[d * count + p] = (float)f[d]; fv[d * count + p] = (float)vv[d]; }
        fw[p] = (float)ww;
      } else {
        double* fo = (double*)off; double* fv = (double*)v; double* fw = (double*)w;
        for (int d = 0; d < 3; ++d) { fo[d * count + p] = f[d]; fv[d * count + p] = vv[d]; }
        fw[p] = ww;
      }
    }
  }
  return count;
}

/* Magnetic field at a point (cell centres use this). */
static void bfield(const synth_cfg* c, const double x[3], double B[3]) {
  double L[3]; domain_len(c, L);
  B[0] = c->B0[0]; B[1] = c->B0[1]; B[2] = c->B0[2];
  if (c->profile == PROF_HARRIS2) {
    double y1 = 0.25 * L[1], y2 = 0.75 * L[1];
    B[0] += c->Bh * (tanh((x[1] - y1) / c->lambda) - tanh((x[1] - y2) / c->lambda) - 1.0);
    /* perturbation B = curl(psi z): (d psi/dy, -d psi/dx, 0),
       psi = amp cos(2 pi x / Lx) cos(2 pi (y - y1) / Ly) */
    double kx = TWO_PI / L[0], ky = TWO_PI / L[1];
    double cx = cos(kx * x[0]), sx = sin(kx * x[0]);
    double cy = cos(ky * (x[1] - y1)), sy = sin(ky * (x[1] - y1));
    B[0] += -c->psi * ky * cx * sy;
    B[1] += c->psi * kx * sx * cy;
  }
}

/* Initial fields: E at nodes (x_g = i dx), B at cell centres ((i+1/2) dx).
 * E = -u x B with the local mean drift of species 0 and 1 weighted by
 * mass (the motional field of the bulk flow), so a uniform flow starts in
 * equilibrium.  Layouts [3][N]. */
void synth_fields(const synth_cfg* c, double* E, double* B) {
  int64_t N = synth_ncells(c);
  double L[3]; domain_len(c, L);
  for (int64_t g = 0; g < N; ++g) {
    int64_t ic[3] = {0, 0, 0}, rem = g;
    for (int d = 0; d < c->dim; ++d) { ic[d] = rem % c->n[d]; rem /= c->n[d]; }
    double xn[3] = {0, 0, 0}, xc[3] = {0, 0, 0};
    for (int d = 0; d < c->dim; ++d) { xn[d] = ic[d] * c->dx[d]; xc[d] = (ic[d] + 0.5) * c->dx[d]; }
    double Bc[3]; bfield(c, xc, Bc);
    for (int d = 0; d < 3; ++d) B[d * N + g] = Bc[d];
    double Bn[3]; bfield(c, xn, Bn);
    double u[3] = {c->u0[0], c->u0[1], c->u0[2]};
    if (c->profile == PROF_SHOCK_TUBE) u[0] += (xn[0] < 0.5 * L[0]) ? c->ushock : -c->ushock;
    E[0 * N + g] = -(u[1] * Bn[2] - u[2] * Bn[1]);
    E[1 * N + g] = -(u[2] * Bn[0] - u[0] * Bn[2]);
    E[2 * N + g] = -(u[0] * Bn[1] - u[1] * Bn[0]);
    if (c->ghost_x && ic[0] == 0) E[1 * N + g] = E[2 * N + g] = 0.0;  /* the wall: no tangential E */
  }
}

/*
 * Particles of species s entering through the inflow plane x = L during
 * step `step` (0-based) of a walled grid: a slab of thickness |u_x| dt_inj
 * at the upper end of the last physical cell column, ppc |u_x| dt_inj / dx
 * particles per column and step on average, the count of step k being
 * floor((k+1) r) - floor(k r) so that the flux is exact over the run.  Drifting
 * Maxwellian velocities as in the bulk; keyed by (seed, 0x1F10), counted by
 * (cell, k, species, step).  Writes up to max particles (cell-major); returns
 * the number written (or the number needed if max is smaller).
 */
int64_t synth_inflow(const synth_cfg* c, int s, int64_t step, int64_t max, int32_t* cell, void* off, void* v,
                     void* w, int f32) {
  if (!c->ghost_x) return 0;
  const int nx = c->n[0] - 1;  /* physical cells along x */
  const double r = c->ppc * fabs(c->u0[0]) * c->dt_inj / c->dx[0];
  const int per = (int)(floor((step + 1) * r) - floor(step * r));
  const int64_t ncol = (int64_t)c->n[1] * c->n[2];
  const int64_t count = ncol * per;
  if (count > max) return count;
  double dV = 1.0;
  for (int d = 0; d < c->dim; ++d) dV *= c->dx[d];
  const double slab = fabs(c->u0[0]) * c->dt_inj / c->dx[0];
  for (int64_t col = 0; col < ncol; ++col) {
    const int64_t cc = (nx - 1) + (int64_t)c->n[0] * col;
    int64_t ic[3] = {nx - 1, col % c->n[1], col / c->n[1]};
    for (int k = 0; k < per; ++k) {
      const int64_t p = col * per + k;
      uint32_t key[2] = {c->seed, 0x1F10u};
      uint32_t ca[4] = {(uint32_t)cc, (uint32_t)k, (uint32_t)(s + 1), (uint32_t)(0x50000u + step)};
      uint32_t cv[4] = {(uint32_t)cc, (uint32_t)k, (uint32_t)(s + 1), (uint32_t)(0x560000u + step)};
      uint32_t ra[4], rv[4];
      synth_philox4x32_10(ca, key, ra);
      synth_philox4x32_10(cv, key, rv);
      double f[3] = {0, 0, 0}, x[3] = {0, 0, 0};
      for (int d = 0; d < c->dim; ++d) f[d] = u01_24(ra[d]);
      f[0] = 1.0 - slab * f[0];  /* in the slab next to x = L */
      if (f[0] >= 1.0) f[0] = 0.99999994039535522;
      for (int d = 0; d < c->dim; ++d) x[d] = ((double)ic[d] + f[d]) * c->dx[d];
      double u[3]; drift(c, s, x, u01(ra[3]), u);
      double nn[4]; normals4(rv, nn);
      double r2 = nn[0] * nn[0] + nn[1] * nn[1] + nn[2] * nn[2];
      if (r2 > RCLIP * RCLIP) {
        double sc = RCLIP / sqrt(r2);
        nn[0] *= sc; nn[1] *= sc; nn[2] *= sc;
      }
      double vv[3];
      for (int d = 0; d < 3; ++d) vv[d] = u[d] + c->vth[s] * nn[d];
      double ww = synth_density(c, x) * dV / c->ppc;
      cell[p] = (int32_t)cc;
      if (f32) {
        float* fo = (float*)off; float* fv = (float*)v; float* fw = (float*)w;
        for (int d = 0; d < 3; ++d) { fo[d * count + p] = (float)f[d]; fv[d * count + p] = (float)vv[d]; }
        fw[p] = (float)ww;
      } else {
        double* fo = (double*)off; double* fv = (double*)v; double* fw = (double*)w;
        for (int d = 0; d < 3; ++d) { fo[d * count + p] = f[d]; fv[d * count + p] = vv[d]; }
        fw[p] = ww;
      }
    }
  }
  return count;
}

int synth_cfg_size(void) { return (int)sizeof(synth_cfg); }
