// Current of an explicit PIC step (Sec. 3.1, explicit form) without mass
// matrices: two passes over the particles of each cell.
//   pass 1: moments per corner, m w W_a and m w v W_a, summed into nodes ->
//           mass-weighted bulk velocity u (then the filter passes of the grid
//           pass);
//   pass 2: comoving frame: q w (v - u(x_p)) W_a with u(x_p) = sum_b W_b u_b
//           over the cell's corners; lab frame: q w v W_a; summed into nodes
//           and divided by the cell volume.
// One wavefront per cell; each lane sums its particles in registers, the wave
// reduces through LDS in a fixed order, and the nodes add their 2^DIM cells in
// a fixed order, so the result is deterministic.
#include <cstring>

#include "ge_internal.h"

namespace {

typedef int i2v __attribute__((ext_vector_type(2)));

template <int DIM>
struct Ex {
  static constexpr int NC = 1 << DIM;                               // corners of a cell
  static constexpr int ND = DIM == 3 ? 27 : (DIM == 2 ? 9 : 3);     // run directions
};
constexpr int EX_NV = 32;  // per-cell values stored (corners x {1 or 3 or 4})

// Inclusive scans over the 64 lanes (DPP row shifts, then the row broadcasts).
template <bool MAX>
__device__ inline int wave_scan(int x) {
#define EX_STEP(CTRL, RMASK)                                                \
  {                                                                         \
    const int y = __builtin_amdgcn_update_dpp(0, x, CTRL, RMASK, 0xf, true); \
    x = MAX ? max(x, y) : x + y;                                            \
  }
  EX_STEP(0x111, 0xf)  // row_shr:1
  EX_STEP(0x112, 0xf)  // row_shr:2
  EX_STEP(0x114, 0xf)  // row_shr:4
  EX_STEP(0x118, 0xf)  // row_shr:8
  EX_STEP(0x142, 0xa)  // row_bcast:15
  EX_STEP(0x143, 0xc)  // row_bcast:31
#undef EX_STEP
  return x;
}
// the value of lane - 1 within each row of 16 (0 in the row's first lane)
__device__ inline float dpp_shr1(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0x111, 0xf, 0xf, true));
}
__device__ inline double dpp_shr1(double x) {
  const long long b = __builtin_bit_cast(long long, x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), 0x111, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x111, 0xf, 0xf, true);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ inline void wsync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T>
struct ExSpecies {
  const T* rec;          // records [n][GE_REC]: offset (3), w, v (3)
  const int32_t* runs;   // [N][ND] (start, count) at the destination cell
  T qs, ms;
};
template <typename T>
struct ExArgs {
  ExSpecies<T> sp[GE_MAX_SPECIES];
  int nsp;
  const double* u;  // [3][N] bulk velocity at nodes (pass 2, comoving)
  T* cells;         // [N][EX_NV] per-cell corner sums
};

// A particle record in registers: offset (3), w, v (3).  No load reaches past
// the record (the last record of a buffer ends where the allocation may end):
// FP32 reads one 4-vector and three values that the compiler merges into one
// 12-byte load; FP64 reads the 4-vectors (x, y, z, w) and (w, vx, vy, vz), the
// second ending at the record's last byte (three separate values there would
// be merged into a wider load reading 8 bytes of the next record).
template <typename T>
struct ExRec {
  T r[GE_REC];
};
template <typename T>
using ex4 = T __attribute__((ext_vector_type(4), aligned(sizeof(T))));
template <typename T>
__device__ inline ExRec<T> load_rec(const T* __restrict__ p) {
  ExRec<T> q;
  const ex4<T> a = *reinterpret_cast<const ex4<T>*>(p);
  q.r[0] = a[0]; q.r[1] = a[1]; q.r[2] = a[2]; q.r[3] = a[3];
  if constexpr (sizeof(T) == 8) {
    const ex4<T> b = *reinterpret_cast<const ex4<T>*>(p + 3);
    q.r[4] = b[1]; q.r[5] = b[2]; q.r[6] = b[3];
  } else {
    q.r[4] = p[4]; q.r[5] = p[5]; q.r[6] = p[6];
  }
  return q;
}

// One particle's contribution to the lane's corner sums.
template <typename T, int DIM, int MODE>
__device__ inline void add_particle(const ExRec<T>& q, T qs, T ms, const T* s_u, T* acc) {
  constexpr int NC = Ex<DIM>::NC;
  const T* r = q.r;
  const T f0 = r[0], f1 = DIM >= 2 ? r[1] : (T)0, f2 = DIM >= 3 ? r[2] : (T)0, w = r[3];
  const T v[3] = {r[4], r[5], r[6]};
  T W[NC];
#pragma unroll
  for (int a = 0; a < NC; ++a) {
    T x = (a & 1) ? f0 : (T)1 - f0;
    if (DIM >= 2) x *= ((a >> 1) & 1) ? f1 : (T)1 - f1;
    if (DIM >= 3) x *= ((a >> 2) & 1) ? f2 : (T)1 - f2;
    W[a] = x;
  }
  if constexpr (MODE == 0) {
    const T mw = ms * w;
#pragma unroll
    for (int a = 0; a < NC; ++a) {
      const T mwa = mw * W[a];
      acc[4 * a] += mwa;
#pragma unroll
      for (int q = 0; q < 3; ++q) acc[4 * a + 1 + q] += mwa * v[q];
    }
  } else {
    T d[3] = {v[0], v[1], v[2]};
    if constexpr (MODE == 1) {
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        T up = 0;
#pragma unroll
        for (int b = 0; b < NC; ++b) up += W[b] * s_u[q * NC + b];
        d[q] -= up;
      }
    }
    const T qw = qs * w;
#pragma unroll
    for (int a = 0; a < NC; ++a)
#pragma unroll
      for (int q = 0; q < 3; ++q) acc[3 * a + q] += qw * W[a] * d[q];
  }
}

// MODE 0: moments (m w, m w v) per corner; 1: comoving current q w (v - u_p);
// 2: lab current q w v.  Species go in pairs: lanes 0..26 read the runs of
// the first, lanes 32..58 those of the second, the particles of both are
// numbered one after the other, and each lane takes two per round (t and
// t + 64), with both records in flight before either is used.
template <typename T, int DIM, int MODE>
__global__ __launch_bounds__(64) void k_cell_linear(DGrid G, ExArgs<T> A) {
  constexpr int NC = Ex<DIM>::NC, ND = Ex<DIM>::ND, NQ = MODE == 0 ? 4 : 3, NV = NC * NQ;
  constexpr int RS = 33;  // reduction table: value k of lane pair l / 2 at k * RS + l / 2
  static_assert(NV <= EX_NV, "per-cell values");
  __shared__ int s_st[64], s_pre[64], s_mk[128];
  __shared__ T s_u[3 * 8];
  __shared__ T s_red[EX_NV * RS];  // 32 lane pairs (+1 pad) per value
  const int lane = threadIdx.x, hl = lane >> 5, rl = lane & 31;
  const int64_t c = __builtin_amdgcn_readfirstlane((int)xcd_block(blockIdx.x, gridDim.x));
  if (c >= G.N) return;
  if (MODE == 1 && lane < NC) {
    const int64_t g = nbr3(G, c, lane & 1, DIM >= 2 ? (lane >> 1) & 1 : 0, DIM >= 3 ? (lane >> 2) & 1 : 0);
#pragma unroll
    for (int q = 0; q < 3; ++q) s_u[q * NC + lane] = (T)A.u[q * G.N + g];
  }
  T acc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = (T)0;
  for (int s0 = 0; s0 < A.nsp; s0 += 2) {
    const ExSpecies<T>& Sa = A.sp[s0];
    const ExSpecies<T>& Sb = A.sp[s0 + 1 < A.nsp ? s0 + 1 : s0];
    const bool has_b = s0 + 1 < A.nsp;
    // the pair's pointers and constants as wave-uniform values (a per-lane
    // choice between the two structures would become a per-lane memory load)
    const T* const reca = Sa.rec;
    const T* const recb = Sb.rec;
    const int32_t* const runa = Sa.runs;
    const int32_t* const runb = Sb.runs;
    const T qsa = Sa.qs, msa = Sa.ms, qsb = Sb.qs, msb = Sb.ms;
    int st = 0, cnt = 0;
    if (rl < ND && (hl == 0 || has_b)) {
      const i2v rv = reinterpret_cast<const i2v*>(hl ? runb : runa)[c * ND + rl];
      st = rv.x;
      cnt = rv.y;
    }
    const int incl = wave_scan<false>(cnt);
    const int total = __builtin_amdgcn_readlane(incl, 63);
    const uint64_t m = __ballot(cnt > 0);
    const int nseg = __popcll(m), nseg0 = __popcll(m & 0xffffffffull);
    wsync();  // the previous pair's readers of s_st / s_pre are done
    if (cnt > 0) {
      const int pos = __popcll(m & (lane == 0 ? 0ull : (~0ull >> (64 - lane))));
      s_st[pos] = st;
      s_pre[pos] = incl - cnt;
    }
    int carry = 0;
    for (int t0 = 0; t0 < total; t0 += 128) {
      // particles t0 + lane and t0 + 64 + lane: run index from a max-scan of
      // run-start markers (k + 1 at the run's first position)
      s_mk[lane] = 0;
      s_mk[64 + lane] = 0;
      wsync();
      if (lane < nseg) {
        const int p = s_pre[lane] - t0;
        if (p >= 0 && p < 128) s_mk[p] = lane + 1;
      }
      wsync();
      const int m0 = max(wave_scan<true>(s_mk[lane]), carry);
      const int m1 = max(wave_scan<true>(s_mk[64 + lane]), __builtin_amdgcn_readlane(m0, 63));
      carry = __builtin_amdgcn_readlane(m1, 63);
      const int ta = t0 + lane, tb = t0 + 64 + lane;
      const bool aa = ta < total, ab = tb < total;
      const int ka = aa ? m0 - 1 : 0, kb = ab ? m1 - 1 : 0;
      const bool sba = ka >= nseg0, sbb = kb >= nseg0;
      // both records are loaded unconditionally before either is used (idle
      // lanes read record 0 of the first species, which every buffer holds):
      // a load under a branch would wait for the first particle's sums
      const int64_t ia = aa ? (int64_t)s_st[ka] + (ta - s_pre[ka]) : 0;
      const int64_t ib = ab ? (int64_t)s_st[kb] + (tb - s_pre[kb]) : 0;
      const ExRec<T> qa = load_rec((aa && sba ? recb : reca) + GE_REC * ia);
      const ExRec<T> qb = load_rec((ab && sbb ? recb : reca) + GE_REC * ib);
      __builtin_amdgcn_s_waitcnt(0xF70);  // vmcnt(0): both records are in
      if (aa) add_particle<T, DIM, MODE>(qa, sba ? qsb : qsa, sba ? msb : msa, s_u, acc);
      if (ab) add_particle<T, DIM, MODE>(qb, sbb ? qsb : qsa, sbb ? msb : msa, s_u, acc);
      wsync();  // s_mk is reset by the next round
    }
  }
  // wave reduction in a fixed order: odd lanes add their even neighbour's
  // values (DPP), value k of lane pair p = lane / 2 goes to k * RS + p; lane k
  // (< NV) of each half sums 16 pairs' values of k, the halves are added
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] += dpp_shr1(acc[k]);
  wsync();
  if (lane & 1)
#pragma unroll
    for (int k = 0; k < NV; ++k) s_red[k * RS + (lane >> 1)] = acc[k];
  wsync();
  const int col = lane & 31, h = lane >> 5;
  T part = 0;
  if (col < NV)
#pragma unroll 8
    for (int r = 0; r < 16; ++r) part += s_red[col * RS + 16 * h + r];
  const T other = __shfl(part, lane + 32, 64);
  if (lane < NV) A.cells[c * EX_NV + lane] = part + other;
}

// Node g is corner a of cell g - a: sum the 2^DIM cells' values in corner
// order.  MODE 0 -> mass[N], mm[3][N]; otherwise out[3][N] = sum / dV.
template <typename T, int DIM, int MODE>
__global__ __launch_bounds__(256) void k_node_linear(DGrid G, const T* __restrict__ cells, double* __restrict__ mass,
                                                     double* __restrict__ out) {
  constexpr int NC = Ex<DIM>::NC, NQ = MODE == 0 ? 4 : 3;
  const int64_t g = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (g >= G.N) return;
  int i, j, k;
  unflat3(G, g, i, j, k);
  double s[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) s[q] = 0;
#pragma unroll
  for (int a = 0; a < NC; ++a) {
    const int64_t cc = flat3(G, i - (a & 1), DIM >= 2 ? j - ((a >> 1) & 1) : j, DIM >= 3 ? k - ((a >> 2) & 1) : k);
#pragma unroll
    for (int q = 0; q < NQ; ++q) s[q] += (double)cells[cc * EX_NV + NQ * a + q];
  }
  if (MODE == 0) {
    mass[g] = s[0];
#pragma unroll
    for (int q = 0; q < 3; ++q) out[q * G.N + g] = s[1 + q];
  } else {
#pragma unroll
    for (int q = 0; q < 3; ++q) out[q * G.N + g] = s[q] / G.dV;
  }
}

inline dim3 cells_grid(int64_t N) { return dim3((unsigned)N); }
inline dim3 nodes_grid(int64_t N) { return dim3((unsigned)((N + 255) / 256)); }

template <typename T, int DIM>
static void explicit_t(ge_ctx* c, int mode) {
  ExArgs<T> A;
  std::memset(&A, 0, sizeof(A));
  A.nsp = c->nsp;
  for (int s = 0; s < c->nsp; ++s) {
    const SpeciesBuf& S = c->sp[s];
    A.sp[s].rec = (const T*)S.rec[S.cur];
    A.sp[s].runs = S.runs[S.cur];
    A.sp[s].qs = (T)S.q;
    A.sp[s].ms = (T)S.m;
  }
  A.u = c->u;
  A.cells = (T*)c->cellQ;
  const int64_t N = c->G.N;
  if (mode == 0) {
    hipLaunchKernelGGL((k_cell_linear<T, DIM, 0>), cells_grid(N), dim3(64), 0, c->stream, c->G, A);
    hipLaunchKernelGGL((k_node_linear<T, DIM, 0>), nodes_grid(N), dim3(256), 0, c->stream, c->G, (const T*)c->cellQ,
                       c->mass, c->mm);
  } else {
    if (mode == 1)
      hipLaunchKernelGGL((k_cell_linear<T, DIM, 1>), cells_grid(N), dim3(64), 0, c->stream, c->G, A);
    else
      hipLaunchKernelGGL((k_cell_linear<T, DIM, 2>), cells_grid(N), dim3(64), 0, c->stream, c->G, A);
    hipLaunchKernelGGL((k_node_linear<T, DIM, 1>), nodes_grid(N), dim3(256), 0, c->stream, c->G, (const T*)c->cellQ,
                       nullptr, c->Jeff);
  }
}

}  // namespace

// mode 0: moments into c->mass, c->mm; mode 1: comoving current (needs c->u);
// mode 2: lab current; modes 1 and 2 write c->Jeff.
int ge_launch_explicit_linear(ge_ctx* c, int mode) {
  switch (c->G.dim * 2 + (c->P.precision == GE_FP32 ? 1 : 0)) {
    case 2: explicit_t<double, 1>(c, mode); break;
    case 3: explicit_t<float, 1>(c, mode); break;
    case 4: explicit_t<double, 2>(c, mode); break;
    case 5: explicit_t<float, 2>(c, mode); break;
    case 6: explicit_t<double, 3>(c, mode); break;
    default: explicit_t<float, 3>(c, mode); break;
  }
  GE_HIP(c, hipGetLastError());
  return GE_OK;
}
