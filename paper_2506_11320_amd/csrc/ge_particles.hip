// Particle-side kernels of the GL-ECSIM pass on gfx950: loading, the
// implicit mover with stable re-binning, and the mass-matrix/current deposit.
//
// Particle storage.  Each species keeps two buffers (ping-pong) of particle
// records, two 4-vectors per particle: (offset in the cell x, y, z, weight)
// and (velocity x, y, z, 0).  A buffer is ordered by "home" cell h (the cell a
// particle occupied before the last push) and, inside a home segment,
// partitioned by the direction d in {-1,0,1}^dim to the particle's present
// cell h + d.  The run of (h, d) is recorded at its destination: runs[c][d] =
// (start, count) for c = h + d, so the ND runs a cell receives sit together.
// The particles now in cell c are the runs (c - d, d) taken in ascending
// linear order of the home cell: that concatenation is exactly the order a
// stable sort by present cell gives, so the re-binning is an integer,
// deterministic, bit-exact stable sort that moves each particle once, inside
// the push.
#include <algorithm>
#include <cstring>

#include "ge_internal.h"

namespace {

typedef int i2 __attribute__((ext_vector_type(2)));  // (start, count) of a run

template <int DIM>
struct Dm {
  static constexpr int ND = DIM == 3 ? 27 : (DIM == 2 ? 9 : 3);  // directions = quad rows
  static constexpr int NC = 1 << DIM;                             // corners
  static constexpr int NRB = DIM == 3 ? 2 : 1;                    // 16-row MFMA blocks
};

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
__device__ inline int rl_i(int x, int l) { return __builtin_amdgcn_readlane(x, l); }
__device__ inline float rl(float x, int l) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l)); }
__device__ inline double rl(double x, int l) {
  int64_t b = __double_as_longlong(x);
  int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), l);
  int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((int64_t)hi << 32) | (uint32_t)lo);
}
// 1/x: the hardware reciprocal (1 ulp) in FP32, a true division in FP64
__device__ inline float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline double recip(double x) { return 1.0 / x; }
__device__ inline uint64_t lanemask_lt(int lane) { return lane == 0 ? 0ull : ((~0ull) >> (64 - lane)); }

// Wavefront scans on DPP lane moves (no LDS round trips): row_shr:1,2,4,8
// within each row of 16 lanes (sources outside the row read 0), then
// row_bcast:15 / row_bcast:31 carry the row totals forward.  0 must be the
// identity of the operation (sums, or maxima of non-negative values).
template <bool MAX, bool HALVES>
__device__ inline int dpp_scan(int x) {
#define GE_DPP_STEP(CTRL, RMASK)                                              \
  {                                                                         \
    const int y = __builtin_amdgcn_update_dpp(0, x, CTRL, RMASK, 0xf, true); \
    x = MAX ? max(x, y) : x + y;                                            \
  }
  GE_DPP_STEP(0x111, 0xf)  // row_shr:1
  GE_DPP_STEP(0x112, 0xf)  // row_shr:2
  GE_DPP_STEP(0x114, 0xf)  // row_shr:4
  GE_DPP_STEP(0x118, 0xf)  // row_shr:8
  GE_DPP_STEP(0x142, 0xa)  // row_bcast:15 into rows 1 and 3
  if (!HALVES) GE_DPP_STEP(0x143, 0xc)  // row_bcast:31 into rows 2 and 3
#undef GE_DPP_STEP
  return x;
}


// Offset e (neighbour h = c + e along one axis) of rank j in ascending order
// of the neighbour's coordinate, on a periodic axis of n >= 3 cells.
__device__ inline int axis_order(int ci, int n, int j) {
  if (ci == 0) return j == 0 ? 0 : (j == 1 ? 1 : -1);
  if (ci == n - 1) return j == 0 ? 1 : (j == 1 ? -1 : 0);
  return j - 1;
}

// Collect the runs of particles present in cell c, ascending by home cell.
// Lane j < ND loads run j; the non-empty runs are compacted into s_start /
// s_pre (exclusive prefix of counts).  Returns the total; nseg the run count.
// Move direction of the run that lane r (< ND) of cell c reads: lanes take the
// runs in ascending order of their home cell c + e, whose move is -e.
template <int DIM>
__device__ inline int run_dir(const DGrid& G, int cx, int cy, int cz, int r) {
  const int ex = axis_order(cx, G.n[0], r % 3);
  const int ey = DIM >= 2 ? axis_order(cy, G.n[1], (r / 3) % 3) : 0;
  const int ez = DIM >= 3 ? axis_order(cz, G.n[2], r / 9) : 0;
  return (1 - ex) + (DIM >= 2 ? 3 * (1 - ey) : 0) + (DIM >= 3 ? 9 * (1 - ez) : 0);
}

template <int DIM>
__device__ int runs_setup(const DGrid& G, int64_t c, const int32_t* __restrict__ runs, int* s_start, int* s_pre,
                          int lane, int& nseg) {
  int cx, cy, cz;
  unflat3(G, c, cx, cy, cz);
  int cnt = 0, st = 0;
  if (lane < Dm<DIM>::ND) {
    const i2 rv = reinterpret_cast<const i2*>(runs)[c * Dm<DIM>::ND + run_dir<DIM>(G, cx, cy, cz, lane)];
    st = rv.x;
    cnt = rv.y;
  }
  const int incl = dpp_scan<false, false>(cnt);
  const int total = rl_i(incl, 31);
  uint64_t m = __ballot(cnt > 0);
  if (cnt > 0) {
    int pos = __popcll(m & lanemask_lt(lane));
    s_start[pos] = st;
    s_pre[pos] = incl - cnt;
  }
  nseg = __popcll(m);
  wave_sync();
  return total;
}

__device__ inline int run_index(int t, const int* s_start, const int* s_pre, int nseg) {
  int k = 0;
  for (int i = 1; i < nseg; ++i)
    if (s_pre[i] <= t) k = i;
  return s_start[k] + (t - s_pre[k]);
}

// E and B at the 2^DIM corner nodes of cell c, from the node records ([N][8]:
// E (3), 0, B (3), 0), into the wavefront's LDS slot, component-major:
// fc[q NC + a] = E_q and fc[(3 + q) NC + a] = B_q at corner a.  Lane 2a + h
// loads half h of corner a as one vector.
template <typename T, int DIM>
__device__ inline void corners_to_lds(const DGrid& G, int64_t c, const T* __restrict__ NF, T* fc, int lane) {
  constexpr int NC = Dm<DIM>::NC;
  typedef T t4 __attribute__((ext_vector_type(4)));
  if (lane < 2 * NC) {
    const int a = lane >> 1, h = lane & 1;
    const int64_t g = nbr3(G, c, a & 1, DIM >= 2 ? (a >> 1) & 1 : 0, DIM >= 3 ? (a >> 2) & 1 : 0);
    const t4 x = reinterpret_cast<const t4*>(NF)[2 * g + h];
    T* dst = fc + 3 * h * NC + a;
    dst[0] = x[0];
    dst[NC] = x[1];
    dst[2 * NC] = x[2];
  }
}

// The same corner values with wave-uniform scalar loads into registers (the
// node records are read-only in the particle kernels): fc[q NC + a] as above,
// E then B (WITH_E), or B alone from fc[0].
template <typename T, int DIM, bool WITH_E>
__device__ inline void corners_scalar(const DGrid& G, int64_t c, const T* NF, T* fc) {
  constexpr int NC = Dm<DIM>::NC;
  typedef T t4 __attribute__((ext_vector_type(4)));
  typedef const __attribute__((address_space(4))) t4* cptr;  // constant address space: scalar loads
  const cptr nf = reinterpret_cast<cptr>(reinterpret_cast<uintptr_t>(NF));
#pragma unroll
  for (int a = 0; a < NC; ++a) {
    const int64_t g = nbr3(G, c, a & 1, DIM >= 2 ? (a >> 1) & 1 : 0, DIM >= 3 ? (a >> 2) & 1 : 0);
    const t4 b = nf[2 * g + 1];
    if constexpr (WITH_E) {
      const t4 e = nf[2 * g];
#pragma unroll
      for (int q = 0; q < 3; ++q) fc[q * NC + a] = e[q];
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) fc[((WITH_E ? 3 : 0) + q) * NC + a] = b[q];
  }
}

template <typename T, int DIM>
__device__ inline void lin_weights(const T f[3], T W[8]) {
  constexpr int NC = Dm<DIM>::NC;
#pragma unroll
  for (int a = 0; a < NC; ++a) {
    T w = (a & 1) ? f[0] : (T)1 - f[0];
    if (DIM >= 2) w *= ((a >> 1) & 1) ? f[1] : (T)1 - f[1];
    if (DIM >= 3) w *= ((a >> 2) & 1) ? f[2] : (T)1 - f[2];
    W[a] = w;
  }
}

// out[q] = sum_a W_a F_q(corner a), corner values read from LDS (broadcast)
template <typename T, int DIM>
__device__ inline void gather_lds(const T W[8], const T* fc, T out[3]) {
  constexpr int NC = Dm<DIM>::NC;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    T s = 0;
#pragma unroll
    for (int a = 0; a < NC; ++a) s += W[a] * fc[q * NC + a];
    out[q] = s;
  }
}

// The implicit mover (Sec. 3.1): vbar = alpha (v + beta E_p),
// v^{n+1} = 2 vbar - v^n, x^{n+3/2} = x^{n+1/2} + dt v^{n+1}.  alpha applied
// as (t + beta t x B + beta^2 (t.B) B) / (1 + beta^2 |B|^2).  fc holds the
// corner values of E^{n+theta} then of B^n.  Returns the direction code of the
// cell move (offsets renormalised to the new cell), or GE_DIR_FAR for a move
// of more than one cell along some axis, with f then holding the new position
// relative to the home cell (renormalised by the far re-sort).  Along an axis
// of n cells a move is accepted while the new position relative to the home
// cell stays in [-(n - 2), n - 1): beyond that the periodic wrap could land it
// on a neighbour of its home cell, where it would share the destination of a
// direction run and the stable order could no longer be rebuilt.  A refused
// or non-finite move keeps the particle where it was and sets 'stuck' (1: too
// far, 2: non-finite).  mv: running maximum of the accepted moves in cells
// along any axis.
template <typename T, int DIM>
__device__ inline int push_one(T f[3], T v[3], const T* fc, T beta, const T dtx[3],
                               int& stuck, T& mv, const DGrid& G, int hx) {
  constexpr int NC = Dm<DIM>::NC;
  T W[8];
  lin_weights<T, DIM>(f, W);
  T Ep[3], Bp[3];
  gather_lds<T, DIM>(W, fc, Ep);
  gather_lds<T, DIM>(W, fc + 3 * NC, Bp);
  const T t0 = v[0] + beta * Ep[0], t1 = v[1] + beta * Ep[1], t2 = v[2] + beta * Ep[2];
  const T b2 = Bp[0] * Bp[0] + Bp[1] * Bp[1] + Bp[2] * Bp[2];
  const T den = recip((T)1 + beta * beta * b2);
  const T tb = beta * beta * (t0 * Bp[0] + t1 * Bp[1] + t2 * Bp[2]);
  const T vb0 = (t0 + beta * (t1 * Bp[2] - t2 * Bp[1]) + tb * Bp[0]) * den;
  const T vb1 = (t1 + beta * (t2 * Bp[0] - t0 * Bp[2]) + tb * Bp[1]) * den;
  const T vb2 = (t2 + beta * (t0 * Bp[1] - t1 * Bp[0]) + tb * Bp[2]) * den;
  v[0] = (T)2 * vb0 - v[0];
  v[1] = (T)2 * vb1 - v[1];
  v[2] = (T)2 * vb2 - v[2];
  T sn[3];
  bool far = false, keep = false;
  T mloc = 0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const T m = v[d] * dtx[d];
    sn[d] = f[d] + m;
    // accepted new positions relative to the home cell: [-(n - 2), n - 1)
    // (derived here rather than passed: fewer live scalar registers)
    T lo_d = (T)(2 - G.n[d]), hi_d = (T)(G.n[d] - 1);
    if (d == 0 && walled(G)) {
      // walled x: specular reflection on a wall (about x = 0: hx + s -> -(hx + s);
      // about x = L: -> 2 nxp - (hx + s)), or leaving through an inflow plane;
      // positions relative to the home cell, so no large numbers cancel
      if (sn[0] < (T)(-hx)) {
        sn[0] = (T)(-2 * hx) - sn[0];
        v[0] = -v[0];
      } else if (sn[0] >= (T)(G.nxp - hx)) {
        if (G.bch == GE_BC_INFLOW) {
          if (sn[0] - sn[0] == (T)0) {
            const T am = fabs(m);
            mv = am > mv ? am : mv;
            return GE_DIR_GONE;
          }
        } else {
          sn[0] = (T)(2 * (G.nxp - hx)) - sn[0];
          v[0] = -v[0];
        }
      }
      lo_d = (T)(-hx);
      hi_d = (T)(G.nxp - hx);
    }
    if (!(sn[d] >= lo_d && sn[d] < hi_d)) {  // also catches NaN and Inf
      keep = true;
      stuck |= (sn[d] - sn[d] == (T)0) ? 1 : 2;  // finite: too far; NaN or Inf: non-finite
    }
    const T am = fabs(m);
    mloc = am > mloc ? am : mloc;
    far = far || !(sn[d] >= (T)-1 && sn[d] < (T)2);
  }
  if (keep) return DIM == 3 ? 13 : (DIM == 2 ? 4 : 1);  // stays in its cell, offsets unchanged
  mv = mloc > mv ? mloc : mv;
  if (far) {
#pragma unroll
    for (int d = 0; d < DIM; ++d) f[d] = sn[d];
    return GE_DIR_FAR;
  }
  int dir = 0, mul = 1;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    T e = floor(sn[d]);
    T fn = sn[d] - e;
    if (fn >= (T)1) { fn = 0; e += (T)1; }
    f[d] = fn;
    dir += ((int)e + 1) * mul;
    mul *= 3;
  }
  return dir;
}

// ------------------------------------------------------------------ push
template <typename T>
struct PushArgs {
  const T* rec;  // particle records [n][GE_REC], read
  T* rec_o;      // written
  const int32_t *runs, *seg_next;
  int32_t* runs_o;
  const T* NF;   // node fields [N][8]: E^{n+theta}, node-averaged B^n
  int32_t* far_o;  // [N][4]: far movers of each home cell (start, count), largest move (float bits), 0
  T beta;
  T dtx[3];
  int64_t n;
  int* flags;      // error flags, then this species' statistics at flags + GE_FL_SPECIES + 4 s
  int* stats;
};

// Direction statistics of one chunk from five bit-ballots of the direction
// code (<= GE_DIR_FAR): 'same' is the mask of active lanes sharing this lane's
// direction; lane k <= GE_DIR_FAR receives the chunk's count of direction k.
struct DirStats {
  uint64_t same;
  int count_k;
};
__device__ inline DirStats dir_stats(bool act, int dir, int lane) {
  const int d = act ? dir : 31;
  uint64_t bm[5];
#pragma unroll
  for (int b = 0; b < 5; ++b) bm[b] = __ballot(act && ((d >> b) & 1));
  const uint64_t am = __ballot(act);
  uint64_t same = am, kk = am;
#pragma unroll
  for (int b = 0; b < 5; ++b) {
    same &= ((d >> b) & 1) ? bm[b] : ~bm[b];
    kk &= ((lane >> b) & 1) ? bm[b] : ~bm[b];
  }
  DirStats r;
  r.same = same;
  r.count_k = lane <= GE_DIR_GONE ? __popcll(kk) : 0;
  return r;
}
__device__ inline int excl_scan(int x) { return dpp_scan<false, false>(x) - x; }

// Particle record i: GE_REC = 7 consecutive values, offset x, y, z, w, then
// velocity x, y, z (28 bytes in FP32, 56 in FP64).  Consecutive records are
// contiguous, so a wave's records are read and written as whole cache lines
// without padding.  No access may reach past the record: the last record of
// a buffer ends where the allocation may end.
//   FP32: read as one 4-vector and three values that the compiler merges into
//   one 12-byte load.
//   FP64: read as the 4-vectors (x, y, z, w) and (w, vx, vy, vz), the second
//   ending at the record's last byte: three separate values at the end would
//   be merged into a wider load that reads 8 bytes of the next record, past
//   the buffer at its last record.
// Written as one 4-vector and three values (a vec3 type is avoided: its FP64
// store writes a fourth, padding element over the next record).
template <typename T>
using rec4 = T __attribute__((ext_vector_type(4), aligned(sizeof(T))));
template <typename T, int DIM>
__device__ inline void read_rec(const T* __restrict__ rec, int64_t i, T f[3], T v[3], T& w) {
  const T* p = rec + GE_REC * i;
  const rec4<T> a = *reinterpret_cast<const rec4<T>*>(p);
#pragma unroll
  for (int d = 0; d < 3; ++d) f[d] = d < DIM ? a[d] : (T)0;
  if constexpr (sizeof(T) == 8) {
    const rec4<T> b = *reinterpret_cast<const rec4<T>*>(p + 3);
    v[0] = b[1]; v[1] = b[2]; v[2] = b[3];
  } else {
    v[0] = p[4]; v[1] = p[5]; v[2] = p[6];
  }
  w = a[3];
}
template <typename T>
__device__ inline void write_rec(T* __restrict__ rec, int64_t o, const T f[3], const T v[3], T w) {
  *reinterpret_cast<rec4<T>*>(rec + GE_REC * o) = rec4<T>{f[0], f[1], f[2], w};
  T* b = rec + GE_REC * o + 4;
  b[0] = v[0]; b[1] = v[1]; b[2] = v[2];
}
template <typename T, int DIM>
__device__ inline void load_particle(const PushArgs<T>& A, int i, T f[3], T v[3], T& w) {
  read_rec<T, DIM>(A.rec, i, f, v, w);
}
template <typename T>
__device__ inline void store_particle(const PushArgs<T>& A, int64_t o, const T f[3], const T v[3], T w) {
  write_rec<T>(A.rec_o, o, f, v, w);
}

// One wavefront per cell: push every particle present in the cell and write
// it into the cell's new segment, partitioned by the direction of its move.
// Cells with up to 128 particles keep the pushed state in registers; larger
// cells count in a first pass and push again in a second (same arithmetic).
template <typename T, int DIM>
__global__ __launch_bounds__(64) void k_push(DGrid G, PushArgs<T> A) {
  constexpr int ND = Dm<DIM>::ND, NC = Dm<DIM>::NC;
  __shared__ int s_start[32], s_pre[32];
  __shared__ int s_mark[128];
  __shared__ T s_fc[48];
  __shared__ uint64_t s_dm[64];  // lane masks per direction, two slots
  const int lane = threadIdx.x;
  // one wavefront (one workgroup) per cell; the cell is uniform over the
  // wave: keep its index (and coordinates) scalar
  const int64_t c = __builtin_amdgcn_readfirstlane((int)xcd_block(blockIdx.x, gridDim.x));
  if (c >= G.N) return;
  // corner E and B: FP32 in scalar registers, FP64 (twice the registers) in LDS
  T fcr[6 * 8];
  const T* fc;
  if constexpr (sizeof(T) == 4) {
    corners_scalar<T, DIM, true>(G, c, A.NF, fcr);
    fc = fcr;
  } else {
    corners_to_lds<T, DIM>(G, c, A.NF, s_fc, lane);
    fc = s_fc;
  }
  int nseg;
  int* sst = s_start;
  int* spr = s_pre;
  const int total = runs_setup<DIM>(G, c, A.runs, sst, spr, lane, nseg);
  int hx, hy, hz;
  unflat3(G, c, hx, hy, hz);
  const int64_t base = A.seg_next[c];
  int cnt = 0, dir_off = 0, stuck = 0, bad = 0;
  T mv = 0;
  if (total <= 128) {
    // particle t = lane and t = 64 + lane: run k from a max-scan of run-start
    // markers (k + 1 at position s_pre[k], 0 elsewhere)
    int* mk = s_mark;
    mk[lane] = 0;
    mk[64 + lane] = 0;
    wave_sync();
    if (lane < nseg) {
      const int p0 = spr[lane];
      if (p0 < 128) mk[p0] = lane + 1;
    }
    wave_sync();
    const int m0 = dpp_scan<true, false>(mk[lane]);
    const int m1 = max(dpp_scan<true, false>(mk[64 + lane]), rl_i(m0, 63));
    T f0[3], v0[3], w0, f1[3], v1[3], w1;
    const bool a0 = lane < total, a1 = 64 + lane < total;
    const int k0 = a0 ? m0 - 1 : 0, k1 = a1 ? m1 - 1 : 0;
    const int i0 = sst[k0] + lane - spr[k0], i1 = sst[k1] + 64 + lane - spr[k1];
    // both records are loaded before either push, unconditionally (idle
    // lanes read record 0, which every buffer holds, and drop it): a load
    // under a branch would wait for the first push before the second load
    load_particle<T, DIM>(A, a0 ? i0 : 0, f0, v0, w0);
    load_particle<T, DIM>(A, a1 ? i1 : 0, f1, v1, w1);
    // wait for both here (vmcnt(0); expcnt and lgkmcnt left at their
    // maxima): the compiler then knows no load is pending on any path below
    // and does not hold the second store for the first one's completion
    __builtin_amdgcn_s_waitcnt(0xF70);
    int d0 = 31, d1 = 31;
    if (a0) d0 = push_one<T, DIM>(f0, v0, fc, A.beta, A.dtx, stuck, mv, G, hx);
    if (a1) d1 = push_one<T, DIM>(f1, v1, fc, A.beta, A.dtx, stuck, mv, G, hx);
    // lanes sharing a direction: each lane ORs its bit into the 64-bit mask of
    // its direction, one mask per direction and slot (s_dm[slot][dir]).  OR
    // does not depend on the order in which the lanes' updates land, so the
    // masks are exactly the sets of lanes; direction 31 (no particle) is
    // never set and reads as empty.
    s_dm[lane] = 0;
    wave_sync();
    const uint64_t bit = 1ull << lane;
    if (a0) __hip_atomic_fetch_or(&s_dm[d0], bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    if (a1) __hip_atomic_fetch_or(&s_dm[32 + d1], bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    wave_sync();
    const uint64_t same0 = s_dm[d0 & 31], same1 = s_dm[32 + (d1 & 31)];
    // lane k <= GE_DIR_GONE: the count of direction k in each slot
    const int c0k = lane <= GE_DIR_GONE ? __popcll(s_dm[lane & 31]) : 0;
    const int c1k = lane <= GE_DIR_GONE ? __popcll(s_dm[32 + (lane & 31)]) : 0;
    cnt = c0k + c1k;
    dir_off = excl_scan(cnt);
    const int b0 = __shfl(dir_off, d0 & 31, 64);
    const int b1 = __shfl(dir_off + c0k, d1 & 31, 64);
    const uint64_t lt = lanemask_lt(lane);
    if (a0) store_particle(A, base + b0 + __popcll(same0 & lt), f0, v0, w0);
    if (a1) store_particle(A, base + b1 + __popcll(same1 & lt), f1, v1, w1);
  } else {
    int running = 0;
#pragma clang loop unroll(disable)
    for (int pass = 0; pass < 2; ++pass) {
      for (int t0 = 0; t0 < total; t0 += 64) {
        const int t = t0 + lane;
        const bool act = t < total;
        T f[3] = {0, 0, 0}, v[3] = {0, 0, 0}, w = 0;
        int dir = 31;
        if (act) {
          load_particle<T, DIM>(A, run_index(t, sst, spr, nseg), f, v, w);
          dir = push_one<T, DIM>(f, v, fc, A.beta, A.dtx, stuck, mv, G, hx);
        }
        const DirStats q = dir_stats(act, dir, lane);
        if (pass == 0) {
          cnt += q.count_k;
        } else {
          const int b = __shfl(dir_off + running, dir & 31, 64);
          const int pos = b + __popcll(q.same & lanemask_lt(lane));
          running += q.count_k;
          if (act) {
            if (pos >= 0 && pos < total) store_particle(A, base + pos, f, v, w);
            else bad = 1;
          }
        }
      }
      if (pass == 0) dir_off = excl_scan(cnt);
    }
    if (lane <= GE_DIR_GONE && running != cnt) bad = 1;
  }
  if (lane < ND) {
    // run (c, lane) is recorded at its destination cell; away from the faces
    // of the grid (a wave-uniform test) no coordinate wraps and the
    // destination is c plus the direction's offset
    const int ox = lane % 3 - 1, oy = DIM >= 2 ? (lane / 3) % 3 - 1 : 0, oz = DIM >= 3 ? lane / 9 - 1 : 0;
    const bool inner = hx > 0 && hx < G.n[0] - 1 && (DIM < 2 || (hy > 0 && hy < G.n[1] - 1)) &&
                       (DIM < 3 || (hz > 0 && hz < G.n[2] - 1));
    const i2 run = i2{(int)(base + dir_off), cnt};
    if (inner)
      reinterpret_cast<i2*>(A.runs_o)[(int64_t)((int)c + ox + G.n[0] * (oy + G.n[1] * oz)) * ND + lane] = run;
    else
      reinterpret_cast<i2*>(A.runs_o)[flat3(G, hx + ox, hy + oy, hz + oz) * ND + lane] = run;
  }
  // the far movers close the home segment; their run is kept at the home
  // cell, with the cell's largest move (reduced over the cells afterwards:
  // one atomic per wave on a single address would serialise the push)
  const int mvb = dpp_scan<true, false>(__float_as_int((float)mv));  // non-negative floats order as integers
  const int mvmax = __builtin_amdgcn_readlane(mvb, 63);
  const int ngone = __builtin_amdgcn_readlane(cnt, GE_DIR_GONE);  // the segment's last group: dropped later
  if (lane == GE_DIR_FAR) {
    typedef int i4 __attribute__((ext_vector_type(4)));
    reinterpret_cast<i4*>(A.far_o)[c] = i4{(int)(base + dir_off), cnt, mvmax, ngone};
    if (cnt > 0) atomicAdd(&A.stats[0], cnt);  // rare: far movers only
    if (ngone > 0) atomicAdd(&A.stats[3], ngone);  // boundary cells of an inflow plane only
  }
  // refusals are rare too: one atomic per quantity from lane 0
  const uint64_t sflags = __ballot((stuck & 1) != 0), nflags = __ballot((stuck & 2) != 0);
  if (lane == 0 && (sflags | nflags)) {
    atomicAdd(&A.stats[2], __popcll(sflags | nflags));
    if (sflags) atomicOr(&A.flags[GE_FL_CFL], 1);
    if (nflags) atomicOr(&A.flags[GE_FL_NONFINITE], 1);
  }
  if (bad) atomicOr(&A.flags[GE_FL_RUNS], 1);
}

// Largest move of a push over the cells (the per-cell maxima the push left
// with the far runs), into the species' statistics: a block maximum, then
// one atomic per block.
__global__ __launch_bounds__(256) void k_move_max(int64_t N, const int32_t* __restrict__ far, int* __restrict__ out) {
  __shared__ int sh[256];
  int m = 0;
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < N; c += (int64_t)gridDim.x * blockDim.x)
    m = max(m, far[4 * c + 2]);
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] = max(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0 && sh[0] > 0) atomicMax(out, sh[0]);
}

// ------------------------------------------------------------------ scan
// cnt[c] = particles now in cell c; seg[c] = exclusive prefix over cells.
template <int DIM>
__global__ __launch_bounds__(256) void k_count(DGrid G, const int32_t* __restrict__ runs, int32_t* __restrict__ cnt) {
  int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= G.N) return;
  int s = 0;
  for (int j = 0; j < Dm<DIM>::ND; ++j) s += runs[2 * (c * Dm<DIM>::ND + j) + 1];
  cnt[c] = s;
}

constexpr int SCAN_ITEMS = 4;
constexpr int SCAN_BLOCK = 256;

__device__ int block_excl_scan(int x, int* sh, int& total) {
  // 256 threads, 4 waves
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int incl = x;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    int t = __shfl_up(incl, d, 64);
    if (lane >= d) incl += t;
  }
  if (lane == 63) sh[wid] = incl;
  __syncthreads();
  int off = 0;
  for (int k = 0; k < wid; ++k) off += sh[k];
  total = sh[0] + sh[1] + sh[2] + sh[3];
  __syncthreads();
  return off + incl - x;
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_reduce(const int32_t* __restrict__ a, int64_t n, int32_t* __restrict__ bsum) {
  __shared__ int sh[4];
  int64_t b0 = (int64_t)blockIdx.x * SCAN_BLOCK * SCAN_ITEMS;
  int s = 0;
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    int64_t i = b0 + (int64_t)threadIdx.x * SCAN_ITEMS + k;
    if (i < n) s += a[i];
  }
  int total;
  block_excl_scan(s, sh, total);
  if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_blocks(int32_t* __restrict__ bsum, int64_t nb) {
  __shared__ int sh[4];
  int carry = 0;
  for (int64_t b0 = 0; b0 < nb; b0 += SCAN_BLOCK) {
    int64_t i = b0 + threadIdx.x;
    int x = i < nb ? bsum[i] : 0;
    int total;
    int e = block_excl_scan(x, sh, total);
    if (i < nb) bsum[i] = carry + e;
    carry += total;
  }
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_final(const int32_t* __restrict__ a, int64_t n,
                                                           const int32_t* __restrict__ boff, int32_t* __restrict__ out) {
  __shared__ int sh[4];
  int64_t b0 = (int64_t)blockIdx.x * SCAN_BLOCK * SCAN_ITEMS;
  int vals[SCAN_ITEMS];
  int s = 0;
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    int64_t i = b0 + (int64_t)threadIdx.x * SCAN_ITEMS + k;
    vals[k] = i < n ? a[i] : 0;
    s += vals[k];
  }
  int total;
  int e = block_excl_scan(s, sh, total) + boff[blockIdx.x];
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    int64_t i = b0 + (int64_t)threadIdx.x * SCAN_ITEMS + k;
    if (i < n) out[i] = e;
    e += vals[k];
  }
}

// ------------------------------------------------------------------ deposit
// For every cell, one wavefront reduces over the cell's particles, species by
// species, with FP32 (or FP64) MFMA 16x16x4: A[row][p] = quadratic weight
// product of row r = (ix, iy, iz) (per axis (1-f)^2, f(1-f), f^2), B[p][col]
// = (w alpha (9), w alpha v (3), w v (3), w).  Every node-pair product
// W_a W_b of the cell is one of these rows, and every linear weight W_a is a
// sum of them, so S = A B holds the whole cell's contribution to the mass
// matrices, current and moments.  Each lane computes one particle's operands
// and writes them to an LDS row laid out for the MFMA reads: the per-axis
// weight factors, whose products give the A rows as the operands are read,
// and the B columns.  Each
// species' S is scaled (beta_s q_s, q_s, m_s) into per-wave LDS accumulators
// and the cell's sums are written once at the end.
template <typename T>
struct DepSpecies {
  const T* rec;  // particle records [n][GE_REC]
  const int32_t* runs;  // [N][ND][2]
  T q, m, beta;
  int64_t n;
};
template <typename T>
struct DepArgs {
  DepSpecies<T> sp[GE_MAX_SPECIES];
  int nsp;
  const T* NF;  // node records [N][8] (the B half is used)
  T* cellQ;     // per-cell sums (cq_index)
  int Qn;
};

template <typename T>
struct Mfma;
template <>
struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  __device__ static v4 op(float a, float b, v4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static int row(int lane, int i) { return 4 * (lane >> 4) + i; }
};
template <>
struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  __device__ static v4 op(double a, double b, v4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  __device__ static int row(int lane, int i) { return (lane >> 4) + 4 * i; }
};

template <typename T, int DIM>
struct DepCfg {
  static constexpr int NR = Dm<DIM>::ND;
  static constexpr int NRB = Dm<DIM>::NRB;
  // staged values of a particle: the quadratic weight factors of x (3
  // values) and the products of those of the other axes (NB = 3^(DIM-1)
  // values), whose products are the NR A values (row r = factor r % 3 times
  // product r / 3, formed when the MFMA operands are read); then the 16 B
  // columns.  Stored value-major, value k of particle p at k SP + p: the 16
  // MFMA steps of one operand read lie within 64 elements of one base address,
  // in reach of the paired LDS reads' offsets (no address arithmetic per
  // step), and the stride SP = 66 puts the lanes of each half-wave read on
  // distinct banks (or on one address).
  static constexpr int NB = DIM == 3 ? 9 : (DIM == 2 ? 3 : 1);
  static constexpr int AW = 3 + NB;
  static constexpr int NV = AW + 16;
  static constexpr int SP = 66;
  // linear sums only (quadratic ones stay in registers): [NR][LW], the 7
  // species-summed columns then the charge of each species (odd stride)
  static constexpr int LW = 7 + GE_MAX_SPECIES;
  static constexpr int NACC = NR * LW;
};

// Run table of one cell for two species at once: lanes 0..26 hold the runs
// of species 0 (and 2), lanes 32..58 those of species 1 (and 3).
struct RunRegs {
  int cnt[2], st[2];
};
// All loads below are issued unconditionally (out-of-range lanes read a valid
// dummy address and drop the value): a load under a branch makes the
// compiler's wait-count analysis fall back to "wait for everything" at the
// join, which would stall on the prefetched data of the next cell.
template <typename T, int DIM>
__device__ inline RunRegs load_runs(const DGrid& G, int64_t c, const DepArgs<T>& A, int lane) {
  RunRegs R;
  const int r0 = lane & 31, half = lane >> 5;
  const int r = r0 < Dm<DIM>::ND ? r0 : 0;
  int cx, cy, cz;
  unflat3(G, c, cx, cy, cz);
  const int64_t ob = (c * Dm<DIM>::ND + run_dir<DIM>(G, cx, cy, cz, r)) * (int64_t)sizeof(i2);
  // species (half) and (half + 2): base pointer of the even species plus a
  // uniform byte distance to the odd one, so the address is base + select
  const int nsp = A.nsp;
  const uintptr_t p0 = (uintptr_t)A.sp[0].runs;
  const uintptr_t p1 = nsp > 1 ? (uintptr_t)A.sp[1].runs : p0;
  const uintptr_t p2 = nsp > 2 ? (uintptr_t)A.sp[2].runs : p0;
  const uintptr_t p3 = nsp > 3 ? (uintptr_t)A.sp[3].runs : p2;
  typedef const __attribute__((address_space(1))) i2* gptr;  // global, not flat
  const i2 a = *(gptr)(p0 + (half ? p1 - p0 : 0) + ob);
  const i2 b = *(gptr)(p2 + (half ? p3 - p2 : 0) + ob);
  // raw values: lanes without a run are masked where the values are used, so
  // that nothing touches the loaded registers before the data are needed
  R.st[0] = a.x;
  R.cnt[0] = a.y;
  R.st[1] = b.x;
  R.cnt[1] = b.y;
  return R;
}

// Per-wave LDS of the deposit: MFMA staging (first, at offset 0, so that a
// lane's read addresses are its own offsets and the steps' particle offsets
// fit the LDS reads' immediates), accumulators, compacted run tables of the
// cell, the run-start markers, corner values.
template <typename T, int DIM>
struct DepLds {
  union {  // the run-start markers are dead before the staging starts
    int mark[2][128];
    __attribute__((aligned(16))) T stage[DepCfg<T, DIM>::NV * DepCfg<T, DIM>::SP];
  };
  T acc[DepCfg<T, DIM>::NACC];
  int runs[GE_MAX_SPECIES][2][32];  // [species][start, pre][run]
  int nseg[GE_MAX_SPECIES];
  int total[GE_MAX_SPECIES];
  T fc[24];
};

// Compact the run tables R (of one cell) and find the source index of the
// particles t = lane and t = 64 + lane of species 0 and 1 (-1 where t is past
// the species' count).
template <typename T, int DIM>
__device__ inline void runs_locate(RunRegs R, DepLds<T, DIM>& L, int nsp, int lane, int idx[2][2]) {
  const int half = lane >> 5, r = lane & 31;
  {
    const bool ok = r < Dm<DIM>::ND;
    if (!(ok && half < nsp)) { R.cnt[0] = 0; R.st[0] = 0; }
    if (!(ok && half + 2 < nsp)) { R.cnt[1] = 0; R.st[1] = 0; }
  }
  int pre[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    if (k == 1 && nsp <= 2) {  // no species 2 and 3 (wave-uniform)
      pre[1] = 0;
      break;
    }
    const int incl = dpp_scan<false, true>(R.cnt[k]);  // within each half
    pre[k] = incl - R.cnt[k];
    const int t0 = __builtin_amdgcn_readlane(incl, 31), t1 = __builtin_amdgcn_readlane(incl, 63);
    const int tot = half ? t1 : t0;
    const uint64_t m = __ballot(R.cnt[k] > 0);
    const uint32_t mh = (uint32_t)(m >> (32 * half));
    const int sp = half + 2 * k;
    if (R.cnt[k] > 0) {
      const int pos = __popc(mh & ((1u << r) - 1u));
      L.runs[sp][0][pos] = R.st[k];
      L.runs[sp][1][pos] = pre[k];
    }
    if (r == 0) {
      L.nseg[sp] = __popc(mh);
      L.total[sp] = sp < nsp ? tot : 0;
    }
  }
  // run-start markers hold lane + 1 (0 = no run starts here)
  L.mark[0][lane] = 0; L.mark[0][64 + lane] = 0;
  L.mark[1][lane] = 0; L.mark[1][64 + lane] = 0;
  wave_sync();
  if (R.cnt[0] > 0 && pre[0] < 128) L.mark[half][pre[0]] = lane + 1;
  wave_sync();
  const int basev = R.st[0] - pre[0];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int tot = L.total[s];
    const int s0 = dpp_scan<true, false>(L.mark[s][lane]);
    const int m0 = s0 - 1;
    const int m1 = max(dpp_scan<true, false>(L.mark[s][64 + lane]), __builtin_amdgcn_readlane(s0, 63)) - 1;
    const int b0 = __shfl(basev, m0 & 63, 64), b1 = __shfl(basev, m1 & 63, 64);
    idx[s][0] = lane < tot ? b0 + lane : -1;
    idx[s][1] = 64 + lane < tot ? b1 + 64 + lane : -1;
  }
}

template <typename T>
struct PState {
  T f[3], v[3], w;
};
template <typename T, int DIM>
__device__ inline void load_p(const DepSpecies<T>& S, int i, PState<T>& P) {
  i = i < 0 ? 0 : i;  // every buffer holds at least one record
  read_rec<T, DIM>(S.rec, i, P.f, P.v, P.w);
}

// One wavefront per cell (the cell index is wave-uniform and lives in scalar
// registers).  The corner fields and the run table are loaded first; the run
// table gives the particle indices, whose loads are then all in flight
// together before the first chunk is staged.
// In FP32 the registers fit four waves per SIMD, which the staging memory
// also allows; latency hiding sets this kernel's speed.
template <typename T, int DIM>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 1))) void k_deposit(DGrid G, DepArgs<T> A) {
  using M = Mfma<T>;
  typedef typename M::v4 v4;
  using C = DepCfg<T, DIM>;
  constexpr int NC = Dm<DIM>::NC, NRB = C::NRB, NR = C::NR, AW = C::AW, NV = C::NV, SP = C::SP;
  static_assert(NV * SP >= 18 * NR + NC * (7 + GE_MAX_SPECIES) + 3, "the staging memory holds a cell's values");
  __shared__ DepLds<T, DIM> L;
  const int lane = threadIdx.x;
  const int64_t c = __builtin_amdgcn_readfirstlane((int)xcd_block(blockIdx.x, gridDim.x));
  if (c >= G.N) return;
  constexpr int LW = C::LW;
  T* lin = L.acc;  // [NR][LW]: q alpha v (3), m v (3), m w, then q_s w of each species
  const int col = lane & 15;
  // MFMA operand reads of a step: particle 4 stp + lane/16; A row col (and
  // 16 + col) as the product of its two staged factors, B column col.  A rows
  // past NR read other (finite) staged values: their products land in
  // accumulator rows that are never used.
  const int prt = lane >> 4, r1 = 16 + col;
  const int rofsXa0 = (col % 3) * SP + prt, rofsXb0 = (3 + col / 3) * SP + prt;
  const int rofsXa1 = (r1 % 3) * SP + prt, rofsXb1 = (3 + r1 / 3) * SP + prt;
  const int rofsB = (AW + col) * SP + prt;

  // B at the corners: FP32 in scalar registers (wave-uniform loads); FP64 (twice
  // the registers) one corner per lane (lanes past the corners reload corner 0)
  // into LDS
  typedef T t3 __attribute__((ext_vector_type(3)));
  T fbr[3 * 8];
  const T* fb;
  t3 cv;
  if constexpr (sizeof(T) == 4) {
    corners_scalar<T, DIM, false>(G, c, A.NF, fbr);
    fb = fbr;
  } else {
    const int a = lane < NC ? lane : 0;
    const int64_t g = nbr3(G, c, a & 1, DIM >= 2 ? (a >> 1) & 1 : 0, DIM >= 3 ? (a >> 2) & 1 : 0);
    cv = *reinterpret_cast<const t3*>(A.NF + 8 * g + 4);
    fb = L.fc;
  }
  const DepSpecies<T>& S1 = A.nsp > 1 ? A.sp[1] : A.sp[0];  // a valid buffer even without species 1
  PState<T> P[2][2];
  {
    int idx[2][2];
    RunRegs R = load_runs<T, DIM>(G, c, A, lane);
    runs_locate(R, L, A.nsp, lane, idx);
#pragma unroll
    for (int j = 0; j < 2; ++j) load_p<T, DIM>(A.sp[0], idx[0][j], P[0][j]);
#pragma unroll
    for (int j = 0; j < 2; ++j) load_p<T, DIM>(S1, idx[1][j], P[1][j]);
  }
  if constexpr (sizeof(T) != 4) {
    if (lane < NC) {
      L.fc[lane] = cv[0];
      L.fc[NC + lane] = cv[1];
      L.fc[2 * NC + lane] = cv[2];
    }
  }
  wave_sync();
  {
    // Mtilde rows (B columns 0..8; the linear sums, columns 9..15, in the
    // same registers of the other lanes) and M0 rows accumulate over species
    // in registers; the charge density of each species goes to LDS as it is
    // completed
    v4 aX[NRB], aM0[NRB];
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb) aX[rb] = aM0[rb] = v4{0, 0, 0, 0};
    // one species: p0, p1 hold its particles 0..127 when 'fast' (species 0
    // and 1, passed as compile-time register operands at each call)
    auto species = [&](const int s, const PState<T>& p0, const PState<T>& p1, const bool fast) {
      const DepSpecies<T>& S = A.sp[s];
      const int total = L.total[s];
      // the MFMA sums each chunk of up to 64 particles from zero; the chunk
      // sums of a species are added with a compensated (Neumaier) sum, so
      // that many chunks (hundreds of particles per cell) do not accumulate
      // FP32 rounding in the matrix core
      v4 acc[NRB], cmp[NRB];
#pragma unroll
      for (int rb = 0; rb < NRB; ++rb) acc[rb] = cmp[rb] = v4{0, 0, 0, 0};
      int nchunk = 0;
      // one chunk of up to 64 particles: operands to LDS, then the MFMA sweep
      auto chunk = [&](const PState<T>& q, int t0) {
        // lanes past the count take a zero weight (all B columns vanish) at
        // the corner-0 position with zero velocity, so every staged value is
        // finite and the MFMA adds exact zeros for them
        const bool ok = t0 + lane < total;
        T vals[NV];  // the A factors, then the 16 B columns
        {
          T f[3], v[3];
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            f[d] = ok ? q.f[d] : (T)0;
            v[d] = ok ? q.v[d] : (T)0;
          }
          const T w = ok ? q.w : (T)0;
          T W[8];
          lin_weights<T, DIM>(f, W);
          T Bp[3];
          gather_lds<T, DIM>(W, fb, Bp);
          const T be = S.beta, bb = be * be;
          const T den = recip((T)1 + bb * (Bp[0] * Bp[0] + Bp[1] * Bp[1] + Bp[2] * Bp[2]));
          const T wd = w * den;
          T al[9];  // w alpha (Sec. 3.1), row-major
          al[0] = (1 + bb * Bp[0] * Bp[0]) * wd;
          al[1] = (be * Bp[2] + bb * Bp[0] * Bp[1]) * wd;
          al[2] = (-be * Bp[1] + bb * Bp[0] * Bp[2]) * wd;
          al[3] = (-be * Bp[2] + bb * Bp[1] * Bp[0]) * wd;
          al[4] = (1 + bb * Bp[1] * Bp[1]) * wd;
          al[5] = (be * Bp[0] + bb * Bp[1] * Bp[2]) * wd;
          al[6] = (be * Bp[1] + bb * Bp[2] * Bp[0]) * wd;
          al[7] = (-be * Bp[0] + bb * Bp[2] * Bp[1]) * wd;
          al[8] = (1 + bb * Bp[2] * Bp[2]) * wd;
          T* bcol = vals + AW;
#pragma unroll
          for (int k = 0; k < 9; ++k) bcol[k] = al[k];
#pragma unroll
          for (int r = 0; r < 3; ++r) bcol[9 + r] = al[3 * r] * v[0] + al[3 * r + 1] * v[1] + al[3 * r + 2] * v[2];
#pragma unroll
          for (int r = 0; r < 3; ++r) bcol[12 + r] = w * v[r];
          bcol[15] = w;
          T X[3][3];
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            if (d < DIM) {
              const T g0 = (T)1 - f[d];
              X[d][0] = g0 * g0;
              X[d][1] = f[d] * g0;
              X[d][2] = f[d] * f[d];
            } else {
              X[d][0] = 1; X[d][1] = 0; X[d][2] = 0;
            }
          }
#pragma unroll
          for (int k = 0; k < 3; ++k) vals[k] = X[0][k];
#pragma unroll
          for (int k = 0; k < C::NB; ++k) vals[3 + k] = X[1][k % 3] * X[2][k / 3];
        }
        {
          // this lane's particle, value-major; single stores (volatile keeps
          // them from being paired), whose 16-bit offsets reach every value
          // from one address, where paired stores would need a new base
          // address every two values
          typedef volatile __attribute__((address_space(3))) T* lds_ptr;
          const lds_ptr own = (lds_ptr)(L.stage + lane);
#pragma unroll
          for (int k = 0; k < NV; ++k) own[k * SP] = vals[k];
        }
        wave_sync();
        // groups of 4 MFMA steps (16 particles; particles past the count are
        // zero); the group count is wave-uniform, and the operands of group
        // g + 1 are read from LDS while the MFMAs of group g run.  Particle
        // offsets are immediates of the LDS reads, the lane's value offsets are
        // precomputed (rofs*).
        const int ngrp = __builtin_amdgcn_readfirstlane((min(64, total - t0) + 15) >> 4);
        T ca[2][4], cb[4];
        auto rd = [&](int g, T (&a)[2][4], T (&b)[4]) {
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const T* rows = L.stage + (16 * g + 4 * i);
            b[i] = rows[rofsB];
            a[0][i] = rows[rofsXa0] * rows[rofsXb0];
            a[1][i] = NRB == 2 ? rows[rofsXa1] * rows[rofsXb1] : (T)0;
          }
        };
        v4 cacc[NRB];
#pragma unroll
        for (int rb = 0; rb < NRB; ++rb) cacc[rb] = v4{0, 0, 0, 0};
        rd(0, ca, cb);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          if (g >= ngrp) break;
          T na[2][4], nb[4];
          if (g < 3) rd(g + 1, na, nb);
          // keep the scheduler from sinking the reads next to their MFMAs
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            cacc[0] = M::op(ca[0][i], cb[i], cacc[0]);
            if (NRB == 2) cacc[NRB - 1] = M::op(ca[1][i], cb[i], cacc[NRB - 1]);
          }
          __builtin_amdgcn_sched_barrier(0);
          if (g < 3) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              ca[0][i] = na[0][i];
              ca[1][i] = na[1][i];
              cb[i] = nb[i];
            }
          }
        }
        wave_sync();
        if (nchunk == 0) {
#pragma unroll
          for (int rb = 0; rb < NRB; ++rb) acc[rb] = cacc[rb];
        } else if (total <= 128) {
          // the second and last chunk: the compensated sum of two terms
          // rounds to the plain sum, so add directly (same bits)
#pragma unroll
          for (int rb = 0; rb < NRB; ++rb) acc[rb] += cacc[rb];
        } else {
#pragma unroll
          for (int rb = 0; rb < NRB; ++rb)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const T a = acc[rb][i], x = cacc[rb][i], t = a + x;
              cmp[rb][i] += fabs(a) >= fabs(x) ? (a - t) + x : (x - t) + a;
              acc[rb][i] = t;
            }
        }
        ++nchunk;
      };
      // particles 0..127 of species 0 and 1 come from the prefetched registers;
      // the rest are loaded here
      const int nfast = fast ? min(total, 128) : 0;
      if (nfast > 0) chunk(p0, 0);
      if (nfast > 64) chunk(p1, 64);
      for (int t0 = nfast; t0 < total; t0 += 64) {
        PState<T> q;
        const int t = t0 + lane;
        load_p<T, DIM>(S, t < total ? run_index(t, L.runs[s][0], L.runs[s][1], L.nseg[s]) : -1, q);
        chunk(q, t0);
      }
      // scale this species' sums into the cell accumulators (each (row, col)
      // belongs to one lane)
      const T qs = S.q, ms = S.m, bq = S.beta * S.q, sx = col < 9 ? bq : (col < 12 ? qs : ms);
      // the compensation terms are exactly zero unless a third chunk was added
      if (nchunk > 2) {
#pragma unroll
        for (int rb = 0; rb < NRB; ++rb) acc[rb] += cmp[rb];
      }
#pragma unroll
      for (int rb = 0; rb < NRB; ++rb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const T val = acc[rb][i];
          aX[rb][i] += sx * val;
          aM0[rb][i] += qs * val;
          const int r = 16 * rb + M::row(lane, i);
          if (col == 15 && r < NR) lin[r * LW + 7 + s] = qs * val;
        }
    };
    // species 0 and 1 with their prefetched particles as fixed registers (a
    // run-time choice between the two would copy them into common registers,
    // and a dynamic index would send the arrays to scratch memory)
    species(0, P[0][0], P[0][1], true);
    if (A.nsp > 1) species(1, P[1][0], P[1][1], true);
    for (int s = 2; s < A.nsp; ++s) species(s, P[0][0], P[0][0], false);
    // The cell's values k < QW are gathered in LDS (the staging rows are free
    // now) and written as 4-value vectors: values 4j..4j+3 of the cell are
    // contiguous at Qc + cq_off(4j).  First the quadratic rows of Mtilde and
    // M0, and the linear sums (rows < NR, columns 9..15) for the corner sums.
    T* V = L.stage;
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = 16 * rb + M::row(lane, i);
        if (r < NR) {
          if (col < 9) {
            V[r * 9 + col] = aX[rb][i];
            V[9 * NR + r * 9 + col] = aM0[rb][i];
          } else {
            lin[r * LW + col - 9] = aX[rb][i];
          }
        }
      }
    wave_sync();
    // corner sums of the linear quantities, W_a = prod_d (X_{a_d} + X_{a_d + 1})
    const int NK = 7 + A.nsp, QW = 18 * NR + NK * NC, QV = (QW + 3) >> 2;
    for (int t = lane; t < NC * NK; t += 64) {
      const int a = t % NC, k = t / NC;
      T sum = 0;
#pragma unroll
      for (int b = 0; b < NC; ++b) {
        int r = (a & 1) + (b & 1);
        if (DIM >= 2) r += 3 * (((a >> 1) & 1) + ((b >> 1) & 1));
        if (DIM >= 3) r += 9 * (((a >> 2) & 1) + ((b >> 2) & 1));
        sum += lin[r * LW + k];
      }
      V[18 * NR + k * NC + a] = sum;
    }
    if (lane < 4 * QV - QW) V[QW + lane] = 0;  // the rest of the last vector
    wave_sync();
    typedef T t4 __attribute__((ext_vector_type(4)));
    T* Qc = A.cellQ + cq_index(c, 0, A.Qn);
    for (int j = lane; j < QV; j += 64)
      *reinterpret_cast<t4*>(Qc + cq_off(4 * j)) = reinterpret_cast<const t4*>(V)[j];
  }
}

// ------------------------------------------------------------------ load / read back
// Initial run table: the particles of cell c, sorted by cell, form the run
// "no move" of cell c: r[c stride] = start, r[c stride + 1] = end, then count.
template <int DIM>
__global__ void k_load_bounds(DGrid G, const int32_t* __restrict__ cell, int64_t n, int32_t* __restrict__ r,
                              int64_t stride, int* flags) {
  int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= n) return;
  int32_t c = cell[p];
  if (c < 0 || c >= G.N) { atomicOr(&flags[GE_FL_LOAD], 1); return; }
  if (p > 0 && cell[p - 1] > c) atomicOr(&flags[GE_FL_LOAD], 1);
  if (p == 0 || cell[p - 1] != c) r[c * stride] = (int32_t)p;
  if (p == n - 1 || cell[p + 1] != c) r[c * stride + 1] = (int32_t)(p + 1);
}
__global__ void k_load_fix(int64_t N, int32_t* __restrict__ r, int64_t stride) {
  int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= N) return;
  int32_t e = r[c * stride + 1];
  r[c * stride + 1] = e > 0 ? e - r[c * stride] : 0;
}

template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_get_particles(DGrid G, const T* __restrict__ rec,
                                                       const int32_t* __restrict__ runs, const int32_t* __restrict__ seg,
                                                       int64_t n, int32_t* __restrict__ cell_o, T* __restrict__ off_o,
                                                       T* __restrict__ v_o, T* __restrict__ w_o) {
  __shared__ int s_start[4][32], s_pre[4][32];
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t c = blockIdx.x * 4 + wid;
  if (c >= G.N) return;
  int nseg;
  const int total = runs_setup<DIM>(G, c, runs, s_start[wid], s_pre[wid], lane, nseg);
  const int64_t base = seg[c];
  for (int t = lane; t < total; t += 64) {
    const int i = run_index(t, s_start[wid], s_pre[wid], nseg);
    const int64_t o = base + t;
    T f[3], v[3], w;
    read_rec<T, 3>(rec, i, f, v, w);
    cell_o[o] = (int32_t)c;
    for (int d = 0; d < 3; ++d) off_o[d * n + o] = f[d];
    for (int d = 0; d < 3; ++d) v_o[d * n + o] = v[d];
    w_o[o] = w;
  }
}

// Particle records from the caller's structure-of-arrays input.
template <typename T>
__global__ void k_pack_particles(int64_t n, const T* __restrict__ off, const T* __restrict__ v, const T* __restrict__ w,
                                 T* __restrict__ rec) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= n) return;
  const T f[3] = {off[p], off[n + p], off[2 * n + p]};
  const T u[3] = {v[p], v[n + p], v[2 * n + p]};
  write_rec<T>(rec, p, f, u, w[p]);
}

// Kinetic energy and momentum of one species, deterministic block partials.
template <typename T>
__global__ __launch_bounds__(256) void k_particle_moments(const T* __restrict__ rec, int64_t n, double* __restrict__ part) {
  __shared__ double sh[4][256];
  double a[4] = {0, 0, 0, 0};
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
    T f[3], v[3], w;
    read_rec<T, 3>(rec, p, f, v, w);
    const double vx = v[0], vy = v[1], vz = v[2], ww = w;
    a[0] += ww * (vx * vx + vy * vy + vz * vz);
    a[1] += ww * vx; a[2] += ww * vy; a[3] += ww * vz;
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

// ------------------------------------------------------------------ far movers
// A particle that moved more than one cell along some axis has no run of its
// own: the push leaves it at the end of its home segment (the far run of the
// home cell, far[h]) with its position relative to the home cell.  The
// re-sort below then rebuilds the canonical layout -- every cell's particles
// contiguous, in the order of a stable sort by cell of the previous order --
// as one run per cell: the buffer order after the push is (home cell,
// direction group, previous order), and a destination cell's contributions
// (its 27 direction runs and its far movers) are ordered by buffer position.

__global__ void k_far_counts(int64_t N, const int32_t* __restrict__ far, int32_t* __restrict__ cnt) {
  const int64_t h = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (h < N) cnt[h] = far[4 * h + 1];
}

// One wavefront per home cell: the far movers' destinations (wrapped on the
// periodic axes), their list entries in buffer order, the per-destination
// counts (integer atomics), and the offsets renormalised in place to the
// destination cell with the arithmetic of the mover.
template <typename T, int DIM>
__global__ __launch_bounds__(64) void k_far_list(DGrid G, T* __restrict__ rec, const int32_t* __restrict__ far,
                                                 const int32_t* __restrict__ pos_h, int32_t* __restrict__ ldest,
                                                 int32_t* __restrict__ lpos, int32_t* __restrict__ cnt_in) {
  const int64_t h = blockIdx.x;
  if (h >= G.N) return;
  const int start = far[4 * h], cnt = far[4 * h + 1];
  if (cnt == 0) return;
  int hc[3];
  unflat3(G, h, hc[0], hc[1], hc[2]);
  for (int t = threadIdx.x; t < cnt; t += 64) {
    const int64_t i = (int64_t)start + t;
    T f[3], v[3], w;
    read_rec<T, DIM>(rec, i, f, v, w);
    int dc[3] = {hc[0], hc[1], hc[2]};
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      T e = floor(f[d]);
      T fn = f[d] - e;
      if (fn >= (T)1) { fn = 0; e += (T)1; }
      f[d] = fn;
      const int64_t n = G.n[d];
      dc[d] = (int)((((int64_t)hc[d] + (int64_t)e) % n + n) % n);
    }
    write_rec<T>(rec, i, f, v, w);
    const int64_t dst = (int64_t)dc[0] + (int64_t)G.n[0] * ((int64_t)dc[1] + (int64_t)G.n[1] * dc[2]);
    const int64_t j = (int64_t)pos_h[h] + t;
    ldest[j] = (int32_t)dst;
    lpos[j] = (int32_t)i;
    atomicAdd(&cnt_in[dst], 1);
  }
}

// Injected particles as far-list entries after the nfar far movers: their
// cells, buffer positions base + j, and the per-destination counts.
__global__ void k_inj_list(int64_t m, const int32_t* __restrict__ cell, int64_t base, int64_t nfar,
                           int32_t* __restrict__ ldest, int32_t* __restrict__ lpos, int32_t* __restrict__ cnt_in) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= m) return;
  const int32_t c = cell[j];
  ldest[nfar + j] = c;
  lpos[nfar + j] = (int32_t)(base + j);
  atomicAdd(&cnt_in[c], 1);
}

// Cells of injected particles: in range and not a ghost cell (flag otherwise).
__global__ void k_inj_check(DGrid G, int64_t m, const int32_t* __restrict__ cell, int* __restrict__ flags) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= m) return;
  const int32_t c = cell[j];
  bool ok = c >= 0 && c < G.N;
  if (ok && walled(G)) ok = (c % G.n[0]) < G.nxp;
  if (!ok) atomicOr(&flags[GE_FL_LOAD], 1);
}

// Bucket of every list entry (far movers in home-cell order, then the
// injected particles in their order): its list index j into the entries of
// its destination, in any slot order (integer atomics).
__global__ void k_far_scatter(int64_t F, const int32_t* __restrict__ ldest, const int32_t* __restrict__ start_in,
                              int32_t* __restrict__ fill, int32_t* __restrict__ sorted) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= F) return;
  const int32_t d = ldest[j];
  const int32_t k = atomicAdd(&fill[d], 1);
  sorted[start_in[d] + k] = (int32_t)j;
}

// One thread per destination: its entries put back in list order (the list
// order is the stable order), then replaced by the particles' buffer
// positions.  Insertion sort for the few entries a cell gets in practice,
// heap sort (O(n log n)) for large buckets.
__device__ inline void sift_down(int32_t* a, int i, int n) {
  for (;;) {
    int m = i, l = 2 * i + 1, r = l + 1;
    if (l < n && a[l] > a[m]) m = l;
    if (r < n && a[r] > a[m]) m = r;
    if (m == i) return;
    const int32_t t = a[i]; a[i] = a[m]; a[m] = t;
    i = m;
  }
}
__global__ void k_far_order(int64_t N, const int32_t* __restrict__ cnt_in, const int32_t* __restrict__ start_in,
                            const int32_t* __restrict__ lpos, int32_t* __restrict__ sorted) {
  const int64_t d = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (d >= N) return;
  const int n = cnt_in[d];
  if (n == 0) return;
  int32_t* b = sorted + start_in[d];
  if (n <= 32) {
    for (int i = 1; i < n; ++i) {
      const int32_t v = b[i];
      int k = i - 1;
      while (k >= 0 && b[k] > v) { b[k + 1] = b[k]; --k; }
      b[k + 1] = v;
    }
  } else {
    for (int i = n / 2 - 1; i >= 0; --i) sift_down(b, i, n);
    for (int e = n - 1; e > 0; --e) {
      const int32_t t = b[0]; b[0] = b[e]; b[e] = t;
      sift_down(b, 0, e);
    }
  }
  for (int i = 0; i < n; ++i) b[i] = lpos[b[i]];
}

// Particles of cell c after the re-sort: its direction runs plus its far
// movers (scan -> new segment starts).
template <int DIM>
__global__ __launch_bounds__(256) void k_far_newcount(DGrid G, const int32_t* __restrict__ runs,
                                                      const int32_t* __restrict__ cnt_in, int32_t* __restrict__ out) {
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= G.N) return;
  int s = cnt_in[c];
  for (int j = 0; j < Dm<DIM>::ND; ++j) s += runs[2 * (c * Dm<DIM>::ND + j) + 1];
  out[c] = s;
}

// number of entries of the ascending list a[0..n) below x
__device__ inline int count_below(const int32_t* a, int n, int x) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (a[mid] < x) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// Two destination cells per wavefront, one per 32-lane half (a cell holds a
// few tens of particles; a whole wavefront per cell would leave most lanes
// idle): merge the cell's direction runs and its far movers by buffer position
// into one contiguous segment of the other buffer; the cell's run table then
// holds the single run "no move".  The runs are collected as in runs_setup,
// within each half.
template <typename T, int DIM>
__global__ __launch_bounds__(64) void k_far_merge(DGrid G, const T* __restrict__ rec, const int32_t* __restrict__ runs,
                                                  const int32_t* __restrict__ sorted,
                                                  const int32_t* __restrict__ cnt_in,
                                                  const int32_t* __restrict__ start_in,
                                                  const int32_t* __restrict__ newstart, T* __restrict__ rec_o,
                                                  int32_t* __restrict__ runs_o) {
  constexpr int ND = Dm<DIM>::ND;
  static_assert(ND <= 32, "the runs of a cell fit in half a wavefront");
  __shared__ int s_start[2][32], s_pre[2][32];
  const int lane = threadIdx.x, half = lane >> 5, hl = lane & 31;
  const int64_t c = 2 * (int64_t)blockIdx.x + half;
  const bool live = c < G.N;  // both halves take part in the wave-wide steps
  const int64_t cc = live ? c : 0;
  int cx, cy, cz;
  unflat3(G, cc, cx, cy, cz);
  int cnt = 0, st = 0;
  if (live && hl < ND) {
    const i2 rv = reinterpret_cast<const i2*>(runs)[cc * ND + run_dir<DIM>(G, cx, cy, cz, hl)];
    st = rv.x;
    cnt = rv.y;
  }
  const int incl = dpp_scan<false, true>(cnt);  // within each half
  const int tot0 = rl_i(incl, 31), tot1 = rl_i(incl, 63);
  const int total = half ? tot1 : tot0;
  const uint64_t m = __ballot(cnt > 0);
  const uint32_t mh = (uint32_t)(m >> (32 * half));
  if (cnt > 0) {
    const int pos = __popc(mh & ((1u << hl) - 1u));
    s_start[half][pos] = st;
    s_pre[half][pos] = incl - cnt;
  }
  const int nseg = __popc(mh);
  wave_sync();
  const int* sst = s_start[half];
  const int* spr = s_pre[half];
  const int nf = live ? cnt_in[cc] : 0;
  const int32_t* fl = sorted + (live ? start_in[cc] : 0);  // ascending buffer positions
  const int64_t o = live ? newstart[cc] : 0;
  for (int t = hl; t < total; t += 32) {
    int k = 0;
    for (int i = 1; i < nseg; ++i)
      if (spr[i] <= t) k = i;
    const int src = sst[k] + (t - spr[k]);
    const int nb = nf > 0 ? count_below(fl, nf, sst[k]) : 0;
    T f[3], v[3], w;
    read_rec<T, DIM>(rec, src, f, v, w);
    write_rec<T>(rec_o, o + t + nb, f, v, w);
  }
  for (int j = hl; j < nf; j += 32) {
    const int p = fl[j];
    int nn = 0;
    for (int k = 0; k < nseg; ++k) {
      const int ck = (k + 1 < nseg ? spr[k + 1] : total) - spr[k];
      if (sst[k] < p) nn += ck;
    }
    T f[3], v[3], w;
    read_rec<T, DIM>(rec, p, f, v, w);
    write_rec<T>(rec_o, o + j + nn, f, v, w);
  }
  if (live && hl < ND) {
    const bool centre = hl == (ND - 1) / 2;
    reinterpret_cast<i2*>(runs_o)[cc * ND + hl] = centre ? i2{(int)o, total + nf} : i2{0, 0};
  }
}

}  // namespace

// ===================================================================== host
static int scan_into(ge_ctx* c, const int32_t* in, int32_t* out) {
  const int64_t N = c->G.N;
  const int64_t per = SCAN_BLOCK * SCAN_ITEMS;
  const int64_t nb = (N + per - 1) / per;
  hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(SCAN_BLOCK), 0, c->stream, in, N, c->scan_blocks);
  hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(SCAN_BLOCK), 0, c->stream, c->scan_blocks, nb);
  hipLaunchKernelGGL(k_scan_final, dim3(nb), dim3(SCAN_BLOCK), 0, c->stream, in, N, c->scan_blocks, out);
  GE_HIP(c, hipGetLastError());
  return GE_OK;
}

// seg_next <- exclusive scan of the per-cell counts of species s
int ge_launch_scan_counts(ge_ctx* c, int s) {
  SpeciesBuf& S = c->sp[s];
  const int64_t N = c->G.N;
  dim3 gb((N + 255) / 256);
  int32_t* cnt = c->seg_next + (int64_t)s * N;  // counts, then scanned in place
  switch (c->G.dim) {
    case 1: hipLaunchKernelGGL(k_count<1>, gb, dim3(256), 0, c->stream, c->G, S.runs[S.cur], cnt); break;
    case 2: hipLaunchKernelGGL(k_count<2>, gb, dim3(256), 0, c->stream, c->G, S.runs[S.cur], cnt); break;
    default: hipLaunchKernelGGL(k_count<3>, gb, dim3(256), 0, c->stream, c->G, S.runs[S.cur], cnt); break;
  }
  GE_HIP(c, hipGetLastError());
  return scan_into(c, cnt, cnt);
}

template <typename T, int DIM>
static void launch_push_t(ge_ctx* c, int s) {
  SpeciesBuf& S = c->sp[s];
  PushArgs<T> A;
  const int cur = S.cur, nxt = 1 - S.cur;
  A.rec = (const T*)S.rec[cur];
  A.rec_o = (T*)S.rec[nxt];
  A.runs = S.runs[cur]; A.seg_next = c->seg_next + (int64_t)s * c->G.N;
  A.runs_o = S.runs[nxt];
  A.NF = (const T*)c->node8;
  A.far_o = S.far;
  A.beta = (T)S.beta;
  for (int d = 0; d < 3; ++d) {
    A.dtx[d] = (T)(c->P.dt * c->G.idx[d]);
  }
  A.n = S.n;
  A.flags = c->flags;
  A.stats = c->flags + GE_FL_SPECIES + 4 * s;
  hipLaunchKernelGGL((k_push<T, DIM>), dim3((unsigned)c->G.N), dim3(64), 0, c->stream, c->G, A);
}

// Push species s; needs ge_launch_scan_counts(c, s) first.
int ge_launch_push(ge_ctx* c, int s) {
  const bool f32 = c->P.precision == GE_FP32;
  switch (c->G.dim * 2 + (f32 ? 1 : 0)) {
    case 2: launch_push_t<double, 1>(c, s); break;
    case 3: launch_push_t<float, 1>(c, s); break;
    case 4: launch_push_t<double, 2>(c, s); break;
    case 5: launch_push_t<float, 2>(c, s); break;
    case 6: launch_push_t<double, 3>(c, s); break;
    default: launch_push_t<float, 3>(c, s); break;
  }
  GE_HIP(c, hipGetLastError());
  c->sp[s].cur = 1 - c->sp[s].cur;
  return GE_OK;
}


// ------------------------------------------------------------------ far re-sort (host)
template <typename P>
static int far_alloc(ge_ctx* c, P** p, size_t bytes) {
  hipError_t e = hipMalloc((void**)p, bytes ? bytes : 8);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return ge_fail(c, GE_ERR_OOM, "hipMalloc of the far-mover scratch failed: " + std::string(hipGetErrorString(e)));
  }
  return GE_OK;
}

void ge_far_free(ge_ctx* c) {
  FarScratch& X = c->fx;
  int32_t** all[] = {&X.dest, &X.pos, &X.sorted, &X.pos_h, &X.cnt_in, &X.start_in, &X.fill, &X.newstart};
  for (auto p : all) {
    if (*p) (void)hipFree(*p);
    *p = nullptr;
  }
  X.cap = 0;
}

template <typename T, int DIM>
static void far_kernels_t(ge_ctx* c, SpeciesBuf& S, int64_t F, int64_t nfar) {
  FarScratch& X = c->fx;
  const int64_t N = c->G.N;
  const int cur = S.cur;
  // (the far runs of a species that has not been pushed since its last
  // re-sort are zero: the re-sort clears them; with no far mover at all, as
  // when only injected particles join, there is nothing to list)
  if (nfar > 0)
    hipLaunchKernelGGL((k_far_list<T, DIM>), dim3((unsigned)N), dim3(64), 0, c->stream, c->G, (T*)S.rec[cur], S.far,
                       X.pos_h, X.dest, X.pos, X.cnt_in);
  scan_into(c, X.cnt_in, X.start_in);
  if (F > 0)
    hipLaunchKernelGGL(k_far_scatter, dim3((unsigned)((F + 255) / 256)), dim3(256), 0, c->stream, F, X.dest,
                       X.start_in, X.fill, X.sorted);
  hipLaunchKernelGGL(k_far_order, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, c->stream, N, X.cnt_in, X.start_in,
                     X.pos, X.sorted);
  hipLaunchKernelGGL((k_far_newcount<DIM>), dim3((N + 255) / 256), dim3(256), 0, c->stream, c->G, S.runs[cur],
                     X.cnt_in, X.newstart);
  scan_into(c, X.newstart, X.newstart);
  hipLaunchKernelGGL((k_far_merge<T, DIM>), dim3((unsigned)((N + 1) / 2)), dim3(64), 0, c->stream, c->G, (const T*)S.rec[cur],
                     S.runs[cur], X.sorted, X.cnt_in, X.start_in, X.newstart, (T*)S.rec[1 - cur], S.runs[1 - cur]);
}

// Largest move of the last push of species s into the flag block.
int ge_launch_move_max(ge_ctx* c, int s) {
  hipLaunchKernelGGL(k_move_max, dim3(256), dim3(256), 0, c->stream, c->G.N, c->sp[s].far,
                     c->flags + GE_FL_SPECIES + 4 * s + 1);
  GE_HIP(c, hipGetLastError());
  return GE_OK;
}

// Stable re-sort of species s: the far movers of the last push (nfar), its
// gone particles dropped, the pending injected particles merged in.
int ge_launch_far_resort(ge_ctx* c, int s, int64_t nfar) {
  FarScratch& X = c->fx;
  SpeciesBuf& S = c->sp[s];
  const int64_t N = c->G.N;
  const int64_t F = nfar + S.inj_n;
  int rc = GE_OK;
  if (!X.pos_h) {
    int32_t** per_cell[] = {&X.pos_h, &X.cnt_in, &X.start_in, &X.fill, &X.newstart};
    for (auto p : per_cell)
      if (!rc) rc = far_alloc(c, p, sizeof(int32_t) * N);
    if (rc) { ge_far_free(c); return rc; }
  }
  if (X.cap < F || F == 0) {
    int32_t** lists[] = {&X.dest, &X.pos, &X.sorted};
    for (auto p : lists) {
      if (*p) (void)hipFree(*p);
      *p = nullptr;
    }
    X.cap = 0;
    const int64_t cap = F > 0 ? F : 1;
    for (auto p : lists)
      if (!rc) rc = far_alloc(c, p, sizeof(int32_t) * cap);
    if (rc) { ge_far_free(c); return rc; }
    X.cap = cap;
  }
  GE_HIP(c, hipMemsetAsync(X.cnt_in, 0, sizeof(int32_t) * N, c->stream));
  GE_HIP(c, hipMemsetAsync(X.fill, 0, sizeof(int32_t) * N, c->stream));
  if (nfar > 0) {  // each home cell's first entry in the far list
    hipLaunchKernelGGL(k_far_counts, dim3((N + 255) / 256), dim3(256), 0, c->stream, N, S.far, X.pos_h);
    scan_into(c, X.pos_h, X.pos_h);
  }
  if (S.inj_n > 0)
    hipLaunchKernelGGL(k_inj_list, dim3((S.inj_n + 255) / 256), dim3(256), 0, c->stream, S.inj_n, S.inj_cell, S.nbuf,
                       nfar, X.dest, X.pos, X.cnt_in);
  const bool f32 = c->P.precision == GE_FP32;
  switch (c->G.dim * 2 + (f32 ? 1 : 0)) {
    case 2: far_kernels_t<double, 1>(c, S, F, nfar); break;
    case 3: far_kernels_t<float, 1>(c, S, F, nfar); break;
    case 4: far_kernels_t<double, 2>(c, S, F, nfar); break;
    case 5: far_kernels_t<float, 2>(c, S, F, nfar); break;
    case 6: far_kernels_t<double, 3>(c, S, F, nfar); break;
    default: far_kernels_t<float, 3>(c, S, F, nfar); break;
  }
  GE_HIP(c, hipGetLastError());
  // the far runs are consumed: a later re-sort without a push (injection
  // only) must not see them again
  GE_HIP(c, hipMemsetAsync(S.far, 0, sizeof(int32_t) * 4 * N, c->stream));
  S.cur = 1 - S.cur;
  return GE_OK;
}

// Injected particles: records appended to rec[cur] after the held ones (the
// buffers grow when needed), cells kept for the next re-sort.
int ge_launch_inject_pack(ge_ctx* c, int s, int64_t m, const int32_t* cell, const void* off, const void* v,
                          const void* w) {
  SpeciesBuf& S = c->sp[s];
  const size_t es = c->P.precision == GE_FP32 ? 4 : 8;
  const int64_t at = S.nbuf + S.inj_n, need = at + m;
  if (need > S.cap) {
    const int64_t cap = std::max(need, S.cap + S.cap / 2);
    void* nb[2] = {nullptr, nullptr};
    for (int b = 0; b < 2; ++b) {
      if (hipMalloc(&nb[b], es * GE_REC * cap) != hipSuccess) {
        (void)hipGetLastError();
        if (nb[0]) (void)hipFree(nb[0]);
        return ge_fail(c, GE_ERR_OOM, "particle buffer growth failed");
      }
    }
    GE_HIP(c, hipMemcpyAsync(nb[S.cur], S.rec[S.cur], es * GE_REC * at, hipMemcpyDeviceToDevice, c->stream));
    GE_HIP(c, hipStreamSynchronize(c->stream));
    for (int b = 0; b < 2; ++b) {
      (void)hipFree(S.rec[b]);
      S.rec[b] = nb[b];
    }
    S.cap = cap;
  }
  if (S.inj_n + m > S.inj_cap) {
    const int64_t cap = std::max(S.inj_n + m, 2 * S.inj_cap);
    int32_t* nc = nullptr;
    if (hipMalloc((void**)&nc, sizeof(int32_t) * cap) != hipSuccess) {
      (void)hipGetLastError();
      return ge_fail(c, GE_ERR_OOM, "injection list allocation failed");
    }
    if (S.inj_n) GE_HIP(c, hipMemcpyAsync(nc, S.inj_cell, sizeof(int32_t) * S.inj_n, hipMemcpyDeviceToDevice, c->stream));
    GE_HIP(c, hipStreamSynchronize(c->stream));
    if (S.inj_cell) (void)hipFree(S.inj_cell);
    S.inj_cell = nc;
    S.inj_cap = cap;
  }
  hipLaunchKernelGGL(k_inj_check, dim3((m + 255) / 256), dim3(256), 0, c->stream, c->G, m, cell, c->flags);
  GE_HIP(c, hipMemcpyAsync(S.inj_cell + S.inj_n, cell, sizeof(int32_t) * m, hipMemcpyDeviceToDevice, c->stream));
  if (es == 4)
    hipLaunchKernelGGL(k_pack_particles<float>, dim3((m + 255) / 256), dim3(256), 0, c->stream, m, (const float*)off,
                       (const float*)v, (const float*)w, (float*)S.rec[S.cur] + GE_REC * at);
  else
    hipLaunchKernelGGL(k_pack_particles<double>, dim3((m + 255) / 256), dim3(256), 0, c->stream, m, (const double*)off,
                       (const double*)v, (const double*)w, (double*)S.rec[S.cur] + GE_REC * at);
  GE_HIP(c, hipGetLastError());
  S.inj_n += m;
  return GE_OK;
}

template <typename T, int DIM>
static void launch_deposit_t(ge_ctx* c) {
  DepArgs<T> A;
  std::memset(&A, 0, sizeof(A));
  A.nsp = c->nsp;
  for (int s = 0; s < c->nsp; ++s) {
    SpeciesBuf& S = c->sp[s];
    A.sp[s].rec = (const T*)S.rec[S.cur];
    A.sp[s].runs = S.runs[S.cur];
    A.sp[s].q = (T)S.q; A.sp[s].m = (T)S.m; A.sp[s].beta = (T)S.beta; A.sp[s].n = S.n;
  }
  A.NF = (const T*)c->node8;
  A.cellQ = (T*)c->cellQ;
  A.Qn = c->Q;
  // one wavefront (one workgroup) per cell
  hipLaunchKernelGGL((k_deposit<T, DIM>), dim3((unsigned)c->G.N), dim3(64), 0, c->stream, c->G, A);
}

int ge_launch_deposit(ge_ctx* c) {
  const bool f32 = c->P.precision == GE_FP32;
  switch (c->G.dim * 2 + (f32 ? 1 : 0)) {
    case 2: launch_deposit_t<double, 1>(c); break;
    case 3: launch_deposit_t<float, 1>(c); break;
    case 4: launch_deposit_t<double, 2>(c); break;
    case 5: launch_deposit_t<float, 2>(c); break;
    case 6: launch_deposit_t<double, 3>(c); break;
    default: launch_deposit_t<float, 3>(c); break;
  }
  GE_HIP(c, hipGetLastError());
  return GE_OK;
}

int ge_launch_load_species(ge_ctx* c, int s, const int32_t* cell, const void* off, const void* v, const void* w) {
  SpeciesBuf& S = c->sp[s];
  const int64_t N = c->G.N, n = S.n;
  const size_t es = c->P.precision == GE_FP32 ? 4 : 8;
  if (n > 0) {
    if (es == 4)
      hipLaunchKernelGGL(k_pack_particles<float>, dim3((n + 255) / 256), dim3(256), 0, c->stream, n, (const float*)off,
                         (const float*)v, (const float*)w, (float*)S.rec[0]);
    else
      hipLaunchKernelGGL(k_pack_particles<double>, dim3((n + 255) / 256), dim3(256), 0, c->stream, n, (const double*)off,
                         (const double*)v, (const double*)w, (double*)S.rec[0]);
  }
  for (int b = 0; b < 2; ++b) {
    GE_HIP(c, hipMemsetAsync(S.runs[b], 0, sizeof(int32_t) * 2 * c->ND * N, c->stream));
  }
  S.cur = 0;
  const int center = (c->ND - 1) / 2;
  int32_t* r0 = S.runs[0] + 2 * center;
  const int64_t stride = 2 * c->ND;
  if (n > 0) {
    dim3 gp((n + 255) / 256);
    switch (c->G.dim) {
      case 1: hipLaunchKernelGGL(k_load_bounds<1>, gp, dim3(256), 0, c->stream, c->G, cell, n, r0, stride, c->flags); break;
      case 2: hipLaunchKernelGGL(k_load_bounds<2>, gp, dim3(256), 0, c->stream, c->G, cell, n, r0, stride, c->flags); break;
      default: hipLaunchKernelGGL(k_load_bounds<3>, gp, dim3(256), 0, c->stream, c->G, cell, n, r0, stride, c->flags); break;
    }
  }
  hipLaunchKernelGGL(k_load_fix, dim3((N + 255) / 256), dim3(256), 0, c->stream, N, r0, stride);
  GE_HIP(c, hipGetLastError());
  return GE_OK;
}

template <typename T, int DIM>
static void launch_get_t(ge_ctx* c, int s, int32_t* cell, void* off, void* v, void* w) {
  SpeciesBuf& S = c->sp[s];
  hipLaunchKernelGGL((k_get_particles<T, DIM>), dim3((c->G.N + 3) / 4), dim3(256), 0, c->stream, c->G,
                     (const T*)S.rec[S.cur], S.runs[S.cur], c->seg_next + (int64_t)s * c->G.N, S.n, cell, (T*)off, (T*)v, (T*)w);
}

int ge_launch_get_particles(ge_ctx* c, int s, int32_t* cell, void* off, void* v, void* w) {
  int rc = ge_launch_scan_counts(c, s);
  if (rc) return rc;
  const bool f32 = c->P.precision == GE_FP32;
  switch (c->G.dim * 2 + (f32 ? 1 : 0)) {
    case 2: launch_get_t<double, 1>(c, s, cell, off, v, w); break;
    case 3: launch_get_t<float, 1>(c, s, cell, off, v, w); break;
    case 4: launch_get_t<double, 2>(c, s, cell, off, v, w); break;
    case 5: launch_get_t<float, 2>(c, s, cell, off, v, w); break;
    case 6: launch_get_t<double, 3>(c, s, cell, off, v, w); break;
    default: launch_get_t<float, 3>(c, s, cell, off, v, w); break;
  }
  GE_HIP(c, hipGetLastError());
  return GE_OK;
}

// k_particle_moments of species s into part[4][GE_DIAG_BLOCKS]
int ge_launch_particle_moments_part(ge_ctx* c, int s, double* part) {
  SpeciesBuf& S = c->sp[s];
  if (c->P.precision == GE_FP32)
    hipLaunchKernelGGL(k_particle_moments<float>, dim3(GE_DIAG_BLOCKS), dim3(256), 0, c->stream,
                       (const float*)S.rec[S.cur], S.n, part);
  else
    hipLaunchKernelGGL(k_particle_moments<double>, dim3(GE_DIAG_BLOCKS), dim3(256), 0, c->stream,
                       (const double*)S.rec[S.cur], S.n, part);
  GE_HIP(c, hipGetLastError());
  return GE_OK;
}

int ge_launch_particle_moments(ge_ctx* c, int s, double* out4) {
  const int nbk = GE_DIAG_BLOCKS;
  double* part = c->partials;  // needs 4 * nbk
  int rc = ge_launch_particle_moments_part(c, s, part);
  if (rc) return rc;
  double h[4 * GE_DIAG_BLOCKS];
  GE_HIP(c, hipMemcpyAsync(h, part, sizeof(double) * 4 * nbk, hipMemcpyDeviceToHost, c->stream));
  GE_HIP(c, hipStreamSynchronize(c->stream));
  for (int k = 0; k < 4; ++k) {
    double a = 0;
    for (int b = 0; b < nbk; ++b) a += h[k * nbk + b];
    out4[k] = a;
  }
  return GE_OK;
}
