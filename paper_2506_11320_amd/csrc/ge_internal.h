// Internal declarations of the gfx950 GL-ECSIM library (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "glecsim.h"

#define GE_MAX_SPECIES 4
#define GE_WAVE 64

// Device view of the periodic mesh.  Inactive axes have n = 1 and are never
// offset, so 3D index arithmetic serves every dimension.
struct DGrid {
  int dim;
  int n[3];
  int64_t N;
  double dx[3], idx[3];
  double dV;
  // division by n[0] and n[1] as a multiply-shift (set by grid_div_magic):
  // q = (x * dm[a]) >> ds[a] for every 0 <= x < 2^31
  uint32_t dm[2];
  int ds[2];
  // visiting order of the stencil kernels (visit_order); < 0: storage order
  int colsh;
  // x boundaries: bcl = GE_BC_PERIODIC (both periodic) or GE_BC_WALL, with
  // bch = GE_BC_WALL or GE_BC_INFLOW; a walled grid stores n[0] = nxp + 1
  // points along x (nodes 0..nxp, cells 0..nxp-1 and the ghost cell nxp)
  int bcl, bch, nxp;
};

// Walled x axis: the wall is the mirror plane of the domain (tangential E and
// normal B odd, normal E and tangential B even); the inflow plane holds E at
// its upstream value and its ghost cell the upstream B.
__host__ __device__ inline bool walled(const DGrid& G) { return G.bcl != GE_BC_PERIODIC; }
// storage x index of cell i (i = -1 or nxp beyond a wall) and the sign of an
// odd component there
__device__ inline int cell_mirror(const DGrid& G, int i, double& sg, bool odd) {
  sg = 1.0;
  if (i < 0) { sg = odd ? -1.0 : 1.0; return -1 - i; }
  if (i >= G.nxp && G.bch == GE_BC_WALL) { sg = odd ? -1.0 : 1.0; return 2 * G.nxp - 1 - i; }
  return i;
}
// storage x index of node i mirrored about the wall planes (i in [-nxp, 2 nxp])
__device__ inline int node_mirror(const DGrid& G, int i, double& sg, bool odd) {
  sg = 1.0;
  if (i < 0) { sg = odd ? -1.0 : 1.0; return -i; }
  if (i > G.nxp) { sg = odd ? -1.0 : 1.0; return 2 * G.nxp - i; }
  return i;
}
// E^{n+theta} components held at node plane i: tangential ones on a wall,
// all three on the inflow plane
__device__ inline bool held(const DGrid& G, int i, int comp) {
  if (i == 0) return comp != 0;
  if (i == G.nxp) return G.bch == GE_BC_INFLOW ? true : comp != 0;
  return false;
}

// Multiplier m = ceil(2^(31+s) / n), s = ceil(log2 n): for x < 2^31 the error
// of x m / 2^(31+s) against x / n is below 2^-s <= 1/n, so the floor is exact
// (division by invariant integers, Granlund and Montgomery 1994); m < 2^32.
inline void grid_div_magic(DGrid& G) {
  for (int a = 0; a < 2; ++a) {
    const uint64_t n = (uint64_t)G.n[a];
    int s = 0;
    while (((uint64_t)1 << s) < n) ++s;
    G.dm[a] = (uint32_t)((((uint64_t)1 << (31 + s)) + n - 1) / n);
    G.ds[a] = 31 + s;
  }
}
__device__ inline unsigned grid_div(const DGrid& G, unsigned x, int a) {
  return (unsigned)(((uint64_t)x * G.dm[a]) >> G.ds[a]);
}

__host__ __device__ inline int wrapi(int i, int n) {
  return i < 0 ? i + n : (i >= n ? i - n : i);
}
// Linear index <-> (i, j, k).  N < 2^31, so 32-bit arithmetic is exact.
__device__ inline void unflat3(const DGrid& G, int64_t g, int& i, int& j, int& k) {
  const unsigned gg = (unsigned)g, nx = (unsigned)G.n[0], ny = (unsigned)G.n[1];
  const unsigned r = grid_div(G, gg, 0);
  i = (int)(gg - r * nx);
  k = (int)grid_div(G, r, 1);
  j = (int)(r - (unsigned)k * ny);
}
__device__ inline int64_t flat3(const DGrid& G, int i, int j, int k) {
  return (int64_t)(wrapi(i, G.n[0]) + G.n[0] * (wrapi(j, G.n[1]) + G.n[1] * wrapi(k, G.n[2])));
}
// Visiting order of the node- and cell-wise stencil kernels in 3D: rows of
// n[0] points taken in columns of 2^colsh y-rows that march in z, so the row
// one step down in z was visited 2^colsh rows earlier and its data is still in
// the L2 (in storage order it lies a whole plane back).  t is the logical
// thread index (< N); returns the point and its (i, j, k).
constexpr int GE_COLSH = 4;
__device__ inline int64_t visit_order(const DGrid& G, unsigned t, int& i, int& j, int& k) {
  const unsigned nx = (unsigned)G.n[0], R = grid_div(G, t, 0);
  i = (int)(t - R * nx);
  if (G.colsh < 0) {
    k = (int)grid_div(G, R, 1);
    j = (int)(R - (unsigned)k * (unsigned)G.n[1]);
  } else {
    const unsigned cz = (unsigned)G.n[2] << G.colsh, c = R / cz, rem = R - c * cz;
    k = (int)(rem >> G.colsh);
    j = (int)((c << G.colsh) + (rem & ((1u << G.colsh) - 1u)));
  }
  return (int64_t)i + (int64_t)G.n[0] * ((int64_t)j + (int64_t)G.n[1] * k);
}
// colsh for a grid: the widest column up to 2^GE_COLSH rows that divides n[1]
inline int visit_colsh(const DGrid& G) {
  if (G.dim < 3) return -1;
  int s = GE_COLSH;
  while (s > 0 && G.n[1] % (1 << s) != 0) --s;
  return s;
}
__device__ inline int64_t nbr3(const DGrid& G, int64_t g, int ox, int oy, int oz) {
  int i, j, k;
  unflat3(G, g, i, j, k);
  return flat3(G, i + ox, j + oy, k + oz);
}

// Per-cell partial sums: value k of cell c at cq_index(c, k, Q), laid out as
// [cell/8][Q/4][8 cells][4 values] (Q a multiple of 4).  The 8 cells of a
// group fill whole 128-byte lines (their deposit waves run side by side, and
// a node-assembly wave reads 64 consecutive cells' vectors as 8 full lines),
// and 4 consecutive values of one cell form one 16-byte vector, which the node
// assembly reads with a single load.
constexpr int GE_CQG = 8;  // cells per group
__host__ __device__ inline int cq_off(int k) { return (k >> 2) * (4 * GE_CQG) + (k & 3); }
__host__ __device__ inline int64_t cq_index(int64_t c, int k, int Q) {
  return ((c / GE_CQG) * (Q >> 2) * GE_CQG + (c % GE_CQG)) * 4 + cq_off(k);
}

// Workgroups are dispatched round-robin over the 8 XCDs; remap so that each
// XCD (and its L2) receives one contiguous range of logical blocks.
__device__ inline int64_t xcd_block(int64_t b, int64_t nb) {
  int64_t q = nb / 8, r = nb % 8, x = b % 8, i = b / 8;
  return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// Half-stencil offsets (see glecsim.h), h -> (ox, oy, oz): o = 0 first, then
// every o != 0 whose last nonzero component is +1, enumerated z-major.
__host__ __device__ inline int half_count(int dim) { return dim == 3 ? 14 : (dim == 2 ? 5 : 2); }
template <int DIM>
struct HalfStencil;
template <>
struct HalfStencil<1> {
  static constexpr int NH = 2;
  static constexpr int o[2][3] = {{0, 0, 0}, {1, 0, 0}};
};
template <>
struct HalfStencil<2> {
  static constexpr int NH = 5;
  static constexpr int o[5][3] = {{0, 0, 0}, {1, 0, 0}, {-1, 1, 0}, {0, 1, 0}, {1, 1, 0}};
};
template <>
struct HalfStencil<3> {
  static constexpr int NH = 14;
  static constexpr int o[14][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 1, 0}, {0, 1, 0},  {1, 1, 0},
                                   {-1, -1, 1}, {0, -1, 1}, {1, -1, 1}, {-1, 0, 1}, {0, 0, 1},
                                   {1, 0, 1},  {-1, 1, 1}, {0, 1, 1},  {1, 1, 1}};
};

// values per particle record: offset in the cell (3), weight, velocity (3)
constexpr int GE_REC = 7;

// Direction code of a particle that moved more than one cell along some axis
// in one push (the 27 codes below it are the moves d in {-1,0,1}^3).
constexpr int GE_DIR_FAR = 27;
// Direction code of a particle that left through an inflow plane.
constexpr int GE_DIR_GONE = 28;

struct SpeciesBuf {
  double q, m, beta;     // beta = q dt / (2 m)
  int64_t n;
  void* rec[2];          // T[max(n,1)][GE_REC]: offset in the cell (3), w, velocity (3)
  int32_t* runs[2];      // [Ncell][ND][2]: (start, count) of the run entering cell c by move d
  int32_t* far;          // [Ncell][4]: (start, count) of the far movers of home cell h (last push),
                         // the largest move in the cell (float bits), particles gone through an inflow plane
  int cur;
  int64_t nbuf;          // records held by rec[cur] (n, or the count before a push's losses are compacted)
  int64_t cap;           // records each of rec[0], rec[1] can hold
  int32_t* inj_cell;     // cells of the injected particles waiting for the next re-sort [inj_cap]
  int64_t inj_n, inj_cap;
};

// Device flag block (int32): the errors, then per species the push statistics
// that the host reads back after a push.
enum {
  GE_FL_CFL = 0,       // a particle moved the whole domain length or more (kept in place)
  GE_FL_RUNS = 1,      // internal run bookkeeping mismatch
  GE_FL_LOAD = 2,      // unsorted or out-of-range cell index at load
  GE_FL_NONFINITE = 3, // a non-finite position after the push (kept in place)
  GE_FL_SPECIES = 4,   // + 4 s: [0] far movers, [1] largest move in cells (float bits), [2] particles kept
                       // in place, [3] particles gone through an inflow plane
  GE_FL_COUNT = 4 + 4 * GE_MAX_SPECIES
};

// Host-side record of the moves since the last ge_moves() call.
struct MoveStats {
  int64_t far[GE_MAX_SPECIES], gone[GE_MAX_SPECIES], injected[GE_MAX_SPECIES];
  double maxmove[GE_MAX_SPECIES];
  int resorts, pushes;
};

// Scratch of the re-sort of far movers (allocated on first use).
struct FarScratch {
  int64_t cap;                  // entries of the far lists
  int32_t *dest, *pos, *sorted; // [cap]: far list (destination, buffer position), positions sorted by destination
  int32_t *pos_h, *cnt_in, *start_in, *fill, *newstart;  // [N] each
};

struct ge_ctx {
  ge_grid grid;
  ge_params P;
  DGrid G;
  hipStream_t stream;
  std::string err;
  int nsp, nh, ND, NC, NR, Q;
  SpeciesBuf sp[GE_MAX_SPECIES];
  // fields (double)
  double *E, *B, *Eth, *Bn, *Jlab, *Jeff, *rho, *mm, *mass, *u, *utmp, *EM, *anode, *kE, *kB, *rhs, *Bnew, *ccell;
  double* psi;  // divergence-cleaning scalar at cells [N]
  // FP32 copies for particle gathers
  void* node8;
  // FP32 path: the E diffusion coefficients rounded to float, read by the
  // interior field operator (kE stays the FP64 value of record)
  float* kEf;  // T[N][8] in the particle precision: E^{n+theta} (3), 0, node-averaged B^n (3), 0
  // mass matrices (T) and per-cell partial sums (T)
  void *Mt, *M0, *cellQ;
  // Jacobi blocks (double [9][N], inverted 3x3 per node)
  double* jac;
  // sort scratch
  int32_t *seg_next, *scan_blocks;  // seg_next: [GE_MAX_SPECIES][N]
  int64_t scan_nblocks;
  // Krylov workspace
  int kr_m;
  int n_cu;     // compute units of the device (persistent launches)
  int kr_last;  // Arnoldi vectors built in the last GMRES cycle
  double *V, *Zp, *kw, *kr, *kx, *hdev, *partials, *scal;
  double* Ub;     // GMRES candidate basis (delayed CGS2), allocated by the first solve
  double* hhost;  // pinned host copy of hdev (per-iteration read-backs of the solve)
  int64_t nred_blocks;
  int* flags;            // GE_FL_COUNT ints (see GE_FL_*)
  int have_deposit, have_solve;
  int push_pending;      // a push ran whose statistics (and far movers) are not settled yet
  int inject_pending;    // injected particles wait for their re-sort
  int device;            // HIP device the context was created on
  int64_t steps;         // completed steps (field updates)
  MoveStats moves;
  FarScratch fx;
  void* cnn;           // learned preconditioner state (ge_cnn.hip), lazily created
  double* Zb;          // flexible-GMRES basis of preconditioned vectors (lazily allocated)
  hipEvent_t ev[11];   // pairs: push, deposit, assemble, grid rest, update; [10] end of the push's scans
  double tsum[8];      // accumulated per-phase seconds (see ge_timings)
  int tcnt;
};

// error helpers
int ge_fail(ge_ctx* c, int code, const std::string& msg);
#define GE_HIP(ctx, call)                                                                   \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess) return ge_fail((ctx), GE_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// launchers (host side), each returns GE_OK or an error via ge_fail
int ge_launch_load_species(ge_ctx* c, int s, const int32_t* cell, const void* off, const void* v, const void* w);
int ge_launch_scan_counts(ge_ctx* c, int s);  // into seg_next + s*N
int ge_launch_push(ge_ctx* c, int s);          // needs ge_launch_scan_counts(c, s) first
// stable re-sort of species s: nfar far movers of the last push, its gone
// particles dropped, the pending injected particles merged in
int ge_launch_far_resort(ge_ctx* c, int s, int64_t nfar);
int ge_launch_inject_pack(ge_ctx* c, int s, int64_t m, const int32_t* cell, const void* off, const void* v,
                          const void* w);  // records at rec[cur][nbuf + inj_n ..], cells into inj_cell
int ge_launch_move_max(ge_ctx* c, int s);  // largest move of the last push into the flag block
void ge_far_free(ge_ctx* c);
int ge_launch_deposit(ge_ctx* c);
int ge_launch_get_particles(ge_ctx* c, int s, int32_t* cell, void* off, void* v, void* w);
int ge_launch_particle_moments(ge_ctx* c, int s, double* out4);  // K, P[3] (sync)

int ge_launch_grid_pass(ge_ctx* c);          // assemble .. rhs
int ge_launch_bulk_velocity(ge_ctx* c);      // u from mm / mass, then the n_smooth_u filter passes
int ge_launch_smooth_current(ge_ctx* c);     // ns_j filter passes on c->Jeff
int ge_launch_explicit_linear(ge_ctx* c, int mode);  // explicit-PIC passes (ge_explicit.hip)
int ge_launch_explicit_fields(ge_ctx* c);    // leapfrog E and B update with c->Jeff
int ge_launch_node_avg(ge_ctx* c);
int ge_launch_apply_A(ge_ctx* c, const double* x, double* y);
int ge_launch_kappa_E(ge_ctx* c, const double* E);  // E limiter coefficients from E
int ge_launch_update(ge_ctx* c);
int ge_launch_widen_M(ge_ctx* c, const void* M, double* dst);
int ge_launch_pack_node8(ge_ctx* c, int half);  // half 0: E^{n+theta} from Eth, 1: B from Bn
int ge_launch_jacobi_setup(ge_ctx* c);
int ge_launch_jacobi_apply(ge_ctx* c, const double* x, double* y);
// blocks of the FP64 diagnostic reductions (each writes 4 partial sums)
constexpr int GE_DIAG_BLOCKS = 256;
int ge_launch_field_diag(ge_ctx* c, double* out);  // W_E, W_B, gauss (sync)
int ge_launch_field_diag_part(ge_ctx* c, double* part);             // partials only, asynchronous
int ge_launch_particle_moments_part(ge_ctx* c, int s, double* part);  // partials only, asynchronous
int ge_noalloc_setup(ge_ctx* c);  // per-device address of the static diagnostics scratch
int ge_launch_sub(ge_ctx* c, const double* a, const double* b, double* out, int64_t n);  // out = a - b

int ge_gmres(ge_ctx* c, double tol, int maxit, int restart, int precond, ge_solve_report* rep);
int ge_cnn_apply_grid(ge_ctx* c, const double* v, double* z, double scale);  // z = N(v) with input scale
void ge_cnn_free(ge_ctx* c);
extern "C" int ge_cnn_add_pair(ge_ctx* c, const double* r, const double* e);
int ge_cnn_harvesting(const ge_ctx* c);
#include <vector>
int ge_cnn_export(ge_ctx* c, std::vector<float>& w, std::vector<float>& m, std::vector<float>& v, int& t, int& cap);
int ge_cnn_import(ge_ctx* c, const float* w, const float* m, const float* v, int t, int cap);
