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
};

__host__ __device__ inline int wrapi(int i, int n) {
  return i < 0 ? i + n : (i >= n ? i - n : i);
}
__device__ inline void unflat3(const DGrid& G, int64_t g, int& i, int& j, int& k) {
  i = (int)(g % G.n[0]);
  int64_t r = g / G.n[0];
  j = (int)(r % G.n[1]);
  k = (int)(r / G.n[1]);
}
__device__ inline int64_t flat3(const DGrid& G, int i, int j, int k) {
  return (int64_t)wrapi(i, G.n[0]) + (int64_t)G.n[0] * ((int64_t)wrapi(j, G.n[1]) + (int64_t)G.n[1] * wrapi(k, G.n[2]));
}
__device__ inline int64_t nbr3(const DGrid& G, int64_t g, int ox, int oy, int oz) {
  int i, j, k;
  unflat3(G, g, i, j, k);
  return flat3(G, i + ox, j + oy, k + oz);
}

// Workgroups are dispatched round-robin over the 8 XCDs; remap so that each
// XCD (and its L2) receives one contiguous range of logical blocks.
__device__ inline int64_t xcd_block(int64_t b, int64_t nb) {
  int64_t q = nb / 8, r = nb % 8, x = b % 8, i = b / 8;
  return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// Half-stencil offsets (see glecsim.h): index h -> (ox, oy, oz).
__host__ __device__ inline int half_count(int dim) { return dim == 3 ? 14 : (dim == 2 ? 5 : 2); }
__host__ __device__ inline void half_offset(int dim, int h, int o[3]) {
  // o = 0 first, then o != 0 with last nonzero component +1, z-major.
  o[0] = o[1] = o[2] = 0;
  if (h == 0) return;
  int k = 0;
  int rz = dim >= 3 ? 1 : 0, ry = dim >= 2 ? 1 : 0;
  for (int oz = -rz; oz <= rz; ++oz)
    for (int oy = -ry; oy <= ry; ++oy)
      for (int ox = -1; ox <= 1; ++ox) {
        int last = oz != 0 ? oz : (oy != 0 ? oy : ox);
        if (last <= 0) continue;
        if (++k == h) { o[0] = ox; o[1] = oy; o[2] = oz; return; }
      }
}

struct SpeciesBuf {
  double q, m, beta;     // beta = q dt / (2 m)
  int64_t n;
  void* off[2];          // T[3][n]
  void* v[2];            // T[3][n]
  void* w[2];            // T[n]
  int32_t* sub_start[2]; // [ND][Ncell]: start of the run (home cell, direction)
  int32_t* sub_cnt[2];   // [ND][Ncell]
  int cur;
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
  // FP32 copies for particle gathers
  float *Eth32, *Bn32;
  // mass matrices (T) and per-cell partial sums (T)
  void *Mt, *M0, *cellQ;
  // Jacobi blocks (double [9][N], inverted 3x3 per node)
  double* jac;
  // sort scratch
  int32_t *seg_next, *scan_blocks;  // seg_next: [GE_MAX_SPECIES][N]
  int64_t scan_nblocks;
  // Krylov workspace
  int kr_m;
  double *V, *Zp, *kw, *kr, *kx, *hdev, *partials, *scal;
  int64_t nred_blocks;
  int* flags;            // [0] CFL clamp, [1] run overflow, [2] load error
  int have_deposit, have_solve;
  hipEvent_t ev[10];   // pairs: push, deposit, assemble, grid rest, update
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
int ge_launch_deposit(ge_ctx* c);
int ge_launch_get_particles(ge_ctx* c, int s, int32_t* cell, void* off, void* v, void* w);
int ge_launch_particle_moments(ge_ctx* c, int s, double* out4);  // K, P[3] (sync)

int ge_launch_grid_pass(ge_ctx* c);          // assemble .. rhs
int ge_launch_node_avg(ge_ctx* c);
int ge_launch_apply_A(ge_ctx* c, const double* x, double* y);
int ge_launch_update(ge_ctx* c);
int ge_launch_widen_M(ge_ctx* c, const void* M, double* dst);
int ge_launch_to_f32(ge_ctx* c, const double* src, float* dst, int64_t n);
int ge_launch_jacobi_setup(ge_ctx* c);
int ge_launch_jacobi_apply(ge_ctx* c, const double* x, double* y);
int ge_launch_field_diag(ge_ctx* c, double* out);  // W_E, W_B, gauss (sync)

int ge_gmres(ge_ctx* c, double tol, int maxit, int restart, int precond, ge_solve_report* rep);
