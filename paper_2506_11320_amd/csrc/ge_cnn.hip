// Learned preconditioner for the implicit E solve: a 3-layer 3x3x3
// convolutional network z = N(r) (3 -> 32 -> 32 -> 3 channels, ReLU after the
// first two layers, no bias, so N(s r) = s N(r) for s > 0), run and trained on
// gfx950 with BF16 MFMA (v_mfma_f32_16x16x32_bf16) and FP32 accumulation.
//
// Activations are channels-last BF16 ([box nodes][C]).  A convolution is an
// implicit GEMM with K running over (tap, input channel) in chunks of 32, each
// lane holding 8 consecutive channels (16 B) of one tapped node.  The
// whole-grid periodic layers (inference inside the solver) use an LDS-tiled
// kernel; the training crops use a simpler kernel with two geometries: valid
// (output = input - 2) and full (backward pass of the data gradient, output =
// input + 2, zero padding).
// Weight gradients are a GEMM over nodes per tap, also on MFMA, reduced over
// node chunks in a fixed order.  Training data are (residual, correction)
// pairs harvested from converged solves, normalised by the residual's RMS;
// random unit-norm combinations of two pairs are valid pairs too (the target
// map is linear), which multiplies the data.
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "ge_internal.h"

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

namespace {

enum { CONV_VALID = 1, CONV_FULL = 2 };

struct ConvArgs {
  const __bf16* in;    // [B][in box][CIN]
  const __bf16* w;     // [27][COUT][CIN]
  __bf16* out_bf;      // [B][out box][COUT] (optional)
  float* out_f32;      // [B][out box][COUT] (optional)
  const __bf16* mask;  // [B][out box][COUT]: zero the output where mask <= 0 (optional)
  int B;
  int ix, iy, iz;
  int ox, oy, oz;
  int relu;
};

__device__ inline bf8 zero8() {
  bf8 z;
#pragma unroll
  for (int j = 0; j < 8; ++j) z[j] = (__bf16)0.0f;
  return z;
}

// Output node -> input node of tap t = (tx, ty, tz) in {0,1,2}^3, or -1 outside.
template <int MODE>
__device__ inline int64_t tap_src(const ConvArgs& A, int b, int x, int y, int z, int tx, int ty, int tz) {
  int xi, yi, zi;
  if (MODE == CONV_VALID) {
    xi = x + tx; yi = y + ty; zi = z + tz;
  } else {
    xi = x + tx - 2; yi = y + ty - 2; zi = z + tz - 2;
    if (xi < 0 || yi < 0 || zi < 0 || xi >= A.ix || yi >= A.iy || zi >= A.iz) return -1;
  }
  return (((int64_t)b * A.iz + zi) * A.iy + yi) * A.ix + xi;
}

template <int CIN, int COUT, int MODE>
__global__ __launch_bounds__(256) void k_conv(ConvArgs A) {
  constexpr int NB = COUT / 16;          // output-channel blocks
  constexpr int TPK = 32 / CIN;          // taps per K chunk
  constexpr int NK = (27 + TPK - 1) / TPK;
  __shared__ __attribute__((aligned(16))) __bf16 sw[27 * COUT * CIN];
  for (int i = threadIdx.x; i < 27 * COUT * CIN / 8; i += blockDim.x)
    reinterpret_cast<bf8*>(sw)[i] = reinterpret_cast<const bf8*>(A.w)[i];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int64_t ovol = (int64_t)A.ox * A.oy * A.oz, total = ovol * A.B;
  const int64_t ntiles = (total + 15) / 16;
  const int row = lane & 15, kq = lane >> 4;  // MFMA row (node in tile) and K quarter
  for (int64_t tile = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); tile < ntiles; tile += (int64_t)gridDim.x * 4) {
    const int64_t o = tile * 16 + row;
    const bool valid = o < total;
    int b = 0, x = 0, y = 0, z = 0;
    if (valid) {
      b = (int)(o / ovol);
      int64_t r = o - (int64_t)b * ovol;
      x = (int)(r % A.ox); r /= A.ox;
      y = (int)(r % A.oy);
      z = (int)(r / A.oy);
    }
    f4 acc[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[nb] = f4{0, 0, 0, 0};
#pragma unroll 3
    for (int q = 0; q < NK; ++q) {
      const int t = q * TPK + (8 * kq) / CIN;  // this lane's tap
      const int c0 = (8 * kq) % CIN;          // and first channel
      bf8 a = zero8();
      if (valid && t < 27) {
        const int64_t src = tap_src<MODE>(A, b, x, y, z, t % 3, (t / 3) % 3, t / 9);
        if (src >= 0) a = *reinterpret_cast<const bf8*>(A.in + src * CIN + c0);
      }
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        bf8 wv = zero8();
        if (t < 27) wv = *reinterpret_cast<const bf8*>(sw + ((t * COUT) + 16 * nb + row) * CIN + c0);
        acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, wv, acc[nb], 0, 0, 0);
      }
    }
    // C[node 4 kq + i][channel 16 nb + row]
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t on = tile * 16 + 4 * kq + i;
        if (on >= total) continue;
        const int co = 16 * nb + row;
        float val = acc[nb][i];
        if (A.relu) val = val <= 0.0f ? 0.0f : val;  // ReLU that keeps NaN (fmaxf would drop it)
        if (A.mask && !((float)A.mask[on * COUT + co] > 0.0f)) val = 0.0f;
        if (A.out_bf) A.out_bf[on * COUT + co] = (__bf16)val;
        if (A.out_f32) A.out_f32[on * COUT + co] = val;
      }
  }
}

// x extent of the network's periodic domain: the stored node planes, less an
// inflow plane (all of whose components are held, so the preconditioned
// vector there is the input itself)
inline int cnn_nx(const DGrid& G) { return walled(G) && G.bch == GE_BC_INFLOW ? G.nxp : G.n[0]; }

// z = v on the held components of a walled grid's boundary node planes
// (x = 0 and x = nxp): their operator rows are the identity, so the exact
// preconditioner keeps the input there.  One thread per node of the two
// planes (t < 2 n[1] n[2]).
__global__ void k_hold_rows(DGrid G, const double* __restrict__ v, double* __restrict__ z) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t np = (int64_t)G.n[1] * G.n[2];
  if (t >= 2 * np) return;
  const int gx = t < np ? 0 : G.nxp;
  const int64_t g = gx + (int64_t)G.n[0] * (t < np ? t : t - np);
  for (int q = 0; q < 3; ++q)
    if (held(G, gx, q)) z[q * G.N + g] = v[q * G.N + g];
}

// Whole-grid (periodic) layer, the one that runs inside every FGMRES
// iteration.  A workgroup of 8 waves owns an output tile of 16 x 8 x 4 nodes;
// its input halo (18 x 10 x 6 nodes) and the layer's weights sit in LDS, so
// each input node is fetched from memory about twice instead of 27 times.
// MFMA operands: A = weights (rows = 16 output channels), B = activations
// (columns = 16 x-consecutive nodes), K = 32 (taps x input channels), so an
// accumulator lane holds 4 consecutive channels of one node and stores them
// as one 8-byte write.  Rows of 64 bytes (32 channels) are XOR-swizzled in
// 16-byte chunks so that the 16 lanes of an LDS phase hit distinct banks.
// With 32 input channels (one tap per K step) a wave's 4 output rows are
// consecutive in y, so for each (tx, tz) its 6 input rows are read once and
// serve the 3 taps along y (6 activation reads for 12 products instead of 12).
// Blocks are persistent; each prefetches its next tile's halo into registers
// while it computes the current one, and the block -> tile order keeps
// neighbouring tiles (shared halos) on one XCD.
// IN_F64: the layer reads the FP64 grid vector v[3][N] times s (first layer);
// OUT_F64: the layer writes z[c][N] = out[c] / s for c < 3 (last layer).
constexpr int TLX = 16, TLY = 8, TLZ = 4, THX = TLX + 2, THY = TLY + 2, THZ = TLZ + 2, THN = THX * THY * THZ;
constexpr int TNT = 512;

struct TileArgs {
  const __bf16* in;  // [N][CIN] (unless IN_F64)
  const double* v;   // [3][N] (IN_F64)
  double s;
  const __bf16* w;   // [27][COUT][CIN]
  __bf16* out;       // [N][COUT] (unless OUT_F64)
  double* z;         // [3][N] (OUT_F64)
  int nx, ny, nz, ntx, nty, ntiles;  // nx: the network's periodic x extent (<= sx)
  int sx;                            // x row length of the grid storage
  int64_t N;
};

__device__ inline int pmod(int a, int n) {
  const int r = a % n;
  return r < 0 ? r + n : r;
}
// 16-byte chunk c of LDS row r (CH chunks per row)
template <int CH>
__device__ inline int swz(int r, int c) {
  return CH == 4 ? r * 4 + (c ^ ((r >> 2) & 3)) : r * CH + c;
}

template <int CIN, int COUT, bool IN_F64, bool OUT_F64>
__global__ __launch_bounds__(TNT) void k_conv_tile(TileArgs A) {
  constexpr int NB = COUT / 16, TPK = 32 / CIN, NK = (27 + TPK - 1) / TPK, CH = CIN / 8;
  constexpr int NLD = (THN * CH + TNT - 1) / TNT;
  static_assert(!IN_F64 || CIN == 8, "FP64 input feeds the 8-channel first layer");
  static_assert(!OUT_F64 || COUT == 16, "FP64 output comes from the 16-channel last layer");
  __shared__ __attribute__((aligned(16))) bf8 sw[27 * COUT * CH];
  __shared__ __attribute__((aligned(16))) bf8 sh[THN * CH];
  for (int i = threadIdx.x; i < 27 * COUT * CH; i += TNT)
    sw[swz<CH>(i / CH, i % CH)] = reinterpret_cast<const bf8*>(A.w)[i];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, row = lane & 15, kq = lane >> 4;
  const int nblk = (int)gridDim.x;
  int tile = (int)xcd_block(blockIdx.x, nblk);

  bf8 pre[NLD];
  double pd[IN_F64 ? NLD : 1][3];
  auto fetch = [&](int tl) {
    const int tx = tl % A.ntx, ty = (tl / A.ntx) % A.nty, tz = tl / (A.ntx * A.nty);
    const int x0 = tx * TLX - 1, y0 = ty * TLY - 1, z0 = tz * TLZ - 1;
#pragma unroll
    for (int i = 0; i < NLD; ++i) {
      const int c = threadIdx.x + i * TNT;
      if (c < THN * CH) {
        const int h = c / CH, part = c % CH;
        const int hx = h % THX, hy = (h / THX) % THY, hz = h / (THX * THY);
        const int64_t g = pmod(x0 + hx, A.nx) + (int64_t)A.sx * (pmod(y0 + hy, A.ny) + (int64_t)A.ny * pmod(z0 + hz, A.nz));
        if constexpr (IN_F64) {
          pd[i][0] = A.v[g];
          pd[i][1] = A.v[A.N + g];
          pd[i][2] = A.v[2 * A.N + g];
        } else {
          pre[i] = reinterpret_cast<const bf8*>(A.in)[g * CH + part];
        }
      }
    }
  };
  auto stage = [&]() {
#pragma unroll
    for (int i = 0; i < NLD; ++i) {
      const int c = threadIdx.x + i * TNT;
      if (c < THN * CH) {
        const int h = c / CH, part = c % CH;
        bf8 x;
        if constexpr (IN_F64) {
          x = zero8();
          x[0] = (__bf16)(float)(A.s * pd[i][0]);
          x[1] = (__bf16)(float)(A.s * pd[i][1]);
          x[2] = (__bf16)(float)(A.s * pd[i][2]);
        } else {
          x = pre[i];
        }
        sh[swz<CH>(h, part)] = x;
      }
    }
  };

  if (tile < A.ntiles) fetch(tile);
  for (; tile < A.ntiles; tile += nblk) {
    __syncthreads();  // the previous tile's readers are done (and the weights are in)
    stage();
    __syncthreads();
    if (tile + nblk < A.ntiles) fetch(tile + nblk);  // in flight during the MFMA work
    f4 acc[4][NB];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[m][nb] = f4{0, 0, 0, 0};
    if constexpr (CIN == 32) {
      // one tap per K step: for each (tx, tz) the wave's 4 output rows
      // (consecutive y at one z) read 6 input rows, each used by up to 3 taps
      const int r0 = 4 * wv, yb = r0 % TLY, zb = r0 / TLY;
#pragma unroll 1
      for (int tz = 0; tz < 3; ++tz)
#pragma unroll
        for (int tx = 0; tx < 3; ++tx) {
          bf8 bv[6];
#pragma unroll
          for (int j = 0; j < 6; ++j) bv[j] = sh[swz<CH>(((zb + tz) * THY + yb + j) * THX + row + tx, kq)];
#pragma unroll
          for (int ty = 0; ty < 3; ++ty) {
            const int t = tx + 3 * ty + 9 * tz;
            bf8 a[NB];
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) a[nb] = sw[swz<CH>(t * COUT + 16 * nb + row, kq)];
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
              for (int nb = 0; nb < NB; ++nb)
                acc[m][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[nb], bv[m + ty], acc[m][nb], 0, 0, 0);
          }
        }
    } else
#pragma unroll 3
    for (int q = 0; q < NK; ++q) {
      const int traw = q * TPK + (8 * kq) / CIN;
      const int c = ((8 * kq) % CIN) / 8;  // this lane's 16-byte chunk of the input channels
      const bool tv = traw < 27;
      const int t = tv ? traw : 26;
      const int tx = t % 3, ty = (t / 3) % 3, tz = t / 9;
      bf8 a[NB];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) a[nb] = tv ? sw[swz<CH>(t * COUT + 16 * nb + row, c)] : zero8();
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int r = 4 * wv + m, yy = r % TLY, zz = r / TLY;
        const bf8 b = sh[swz<CH>(((zz + tz) * THY + yy + ty) * THX + row + tx, c)];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[m][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[nb], b, acc[m][nb], 0, 0, 0);
      }
    }
    // C[channel 16 nb + 4 kq + i][node row]
    const int tx = tile % A.ntx, ty = (tile / A.ntx) % A.nty, tz = tile / (A.ntx * A.nty);
    const int gx = tx * TLX + row;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int r = 4 * wv + m;
      const int gy = ty * TLY + r % TLY, gz = tz * TLZ + r / TLY;
      if (gx >= A.nx || gy >= A.ny || gz >= A.nz) continue;
      const int64_t g = gx + (int64_t)A.sx * (gy + (int64_t)A.ny * gz);
      if constexpr (OUT_F64) {
        if (kq == 0) {
          const double inv = 1.0 / A.s;
          A.z[g] = (double)acc[m][0][0] * inv;
          A.z[A.N + g] = (double)acc[m][0][1] * inv;
          A.z[2 * A.N + g] = (double)acc[m][0][2] * inv;
        }
      } else {
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          typedef __bf16 bf4 __attribute__((ext_vector_type(4)));
          bf4 o;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const float val = acc[m][nb][i];
            o[i] = (__bf16)(val <= 0.0f ? 0.0f : val);  // ReLU that keeps NaN
          }
          *reinterpret_cast<bf4*>(A.out + g * COUT + 16 * nb + 4 * kq) = o;
        }
      }
    }
  }
}

// Weight gradient of one layer in the valid geometry (in box = out box + 2):
// part[chunk][t][co][ci] = sum over the chunk's output nodes o of
// dout[o][co] * in[o + t][ci].  MFMA rows = co, columns = ci, K = nodes.
struct WgradArgs {
  const __bf16* in;    // [B][out+2 box][CIN]
  const __bf16* dout;  // [B][out box][COUT]
  float* part;         // [nchunk][27][COUT][CIN_PAD]
  int B, ox, oy, oz;
  int64_t chunk;       // output nodes per chunk (multiple of 32)
};
template <int CIN, int COUT>
__global__ __launch_bounds__(64) void k_wgrad(WgradArgs A) {
  constexpr int CP = CIN < 16 ? 16 : CIN;  // padded column count
  constexpr int MB = COUT / 16, NBk = CP / 16;
  const int t = blockIdx.y;
  const int64_t chunk = blockIdx.x;
  const int lane = threadIdx.x, row = lane & 15, kq = lane >> 4;
  const int tx = t % 3, ty = (t / 3) % 3, tz = t / 9;
  const int ix = A.ox + 2, iy = A.oy + 2, iz = A.oz + 2;
  const int64_t ovol = (int64_t)A.ox * A.oy * A.oz, total = ovol * A.B;
  const int64_t o0 = chunk * A.chunk, o1 = o0 + A.chunk < total ? o0 + A.chunk : total;
  f4 acc[MB][NBk];
#pragma unroll
  for (int m = 0; m < MB; ++m)
#pragma unroll
    for (int n = 0; n < NBk; ++n) acc[m][n] = f4{0, 0, 0, 0};
  for (int64_t k0 = o0; k0 < o1; k0 += 32) {
    // this lane's 8 nodes: k0 + 8 kq + j
    int64_t src[8];
    int64_t onode[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int64_t o = k0 + 8 * kq + j;
      onode[j] = o < o1 ? o : -1;
      src[j] = -1;
      if (o < o1) {
        const int b = (int)(o / ovol);
        int64_t r = o - (int64_t)b * ovol;
        const int x = (int)(r % A.ox); r /= A.ox;
        const int y = (int)(r % A.oy), z = (int)(r / A.oy);
        src[j] = (((int64_t)b * iz + z + tz) * iy + y + ty) * ix + x + tx;
      }
    }
#pragma unroll
    for (int m = 0; m < MB; ++m) {
      bf8 a;
#pragma unroll
      for (int j = 0; j < 8; ++j) a[j] = onode[j] >= 0 ? A.dout[onode[j] * COUT + 16 * m + row] : (__bf16)0.0f;
#pragma unroll
      for (int n = 0; n < NBk; ++n) {
        const int ci = 16 * n + row;
        bf8 bv;
#pragma unroll
        for (int j = 0; j < 8; ++j) bv[j] = (src[j] >= 0 && ci < CIN) ? A.in[src[j] * CIN + ci] : (__bf16)0.0f;
        acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bv, acc[m][n], 0, 0, 0);
      }
    }
  }
  // C[co = 16 m + 4 kq + i][ci = 16 n + row]
  float* P = A.part + ((int64_t)chunk * 27 + t) * COUT * CP;
#pragma unroll
  for (int m = 0; m < MB; ++m)
#pragma unroll
    for (int n = 0; n < NBk; ++n)
#pragma unroll
      for (int i = 0; i < 4; ++i) P[(16 * m + 4 * kq + i) * CP + 16 * n + row] = acc[m][n][i];
}

// sum the chunk partials in a fixed order
__global__ void k_reduce_chunks(const float* __restrict__ part, int nchunk, int64_t n, float* __restrict__ out) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  float s = 0;
  for (int c = 0; c < nchunk; ++c) s += part[(int64_t)c * n + i];
  out[i] = s;
}

// ----------------------------------------------------------------- data movement
// Training crops: crop b has origin org[b] (periodic), pairs (p0, p1) with
// weights (w0, w1).  Input box (n+6)^3 of the residual combination (BF16, 8
// channels), target box n^3 (offset 3) of the correction combination (FP32).
struct CropArgs {
  const float* pr;  // pair store residuals [P][3][N]
  const float* pe;  // pair store corrections
  int64_t N;
  int nx, ny, nz;   // the network's periodic domain (nx <= sx)
  int sx;           // x row length of the grid storage
  int n;            // output crop edge
  const int* meta;  // per crop: ox, oy, oz, p0, p1
  const float* wts; // per crop: w0, w1
  __bf16* in;       // [B][(n+6)^3][8]
  float* tgt;       // [B][n^3][3]
  int B;
};
__global__ void k_make_crops(CropArgs A) {
  const int m = A.n + 6;
  const int64_t vin = (int64_t)m * m * m, vout = (int64_t)A.n * A.n * A.n;
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= vin * A.B) return;
  const int b = (int)(i / vin);
  int64_t r = i - (int64_t)b * vin;
  const int x = (int)(r % m); r /= m;
  const int y = (int)(r % m), z = (int)(r / m);
  const int* mt = A.meta + 5 * b;
  const int gx = wrapi((mt[0] + x) % A.nx, A.nx), gy = wrapi((mt[1] + y) % A.ny, A.ny), gz = wrapi((mt[2] + z) % A.nz, A.nz);
  const int64_t g = gx + (int64_t)A.sx * (gy + (int64_t)A.ny * gz);
  const float w0 = A.wts[2 * b], w1 = A.wts[2 * b + 1];
  const float* r0 = A.pr + (int64_t)mt[3] * 3 * A.N;
  const float* r1 = A.pr + (int64_t)mt[4] * 3 * A.N;
  bf8 v = zero8();
  for (int c = 0; c < 3; ++c) v[c] = (__bf16)(w0 * r0[c * A.N + g] + w1 * r1[c * A.N + g]);
  reinterpret_cast<bf8*>(A.in)[i] = v;
  if (x >= 3 && y >= 3 && z >= 3 && x < A.n + 3 && y < A.n + 3 && z < A.n + 3) {
    const int64_t o = (int64_t)b * vout + ((int64_t)(z - 3) * A.n + (y - 3)) * A.n + (x - 3);
    const float* e0 = A.pe + (int64_t)mt[3] * 3 * A.N;
    const float* e1 = A.pe + (int64_t)mt[4] * 3 * A.N;
    for (int c = 0; c < 3; ++c) A.tgt[o * 3 + c] = w0 * e0[c * A.N + g] + w1 * e1[c * A.N + g];
  }
}

// dL/dz for L = mean (z - e)^2 over crops, nodes, 3 channels; BF16 gradient
// for the backward convolutions; loss block partials.
__global__ __launch_bounds__(256) void k_loss_grad(int64_t nout, const float* __restrict__ z, const float* __restrict__ tgt,
                                                   __bf16* __restrict__ dz, float* __restrict__ part) {
  __shared__ float sh[256];
  const float scale = 2.0f / (float)(3 * nout);
  float acc = 0;
  for (int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; o < nout; o += (int64_t)gridDim.x * blockDim.x) {
    for (int c = 0; c < 16; ++c) {
      float d = 0;
      if (c < 3) {
        d = z[o * 16 + c] - tgt[o * 3 + c];
        acc += d * d;
      }
      dz[o * 16 + c] = (__bf16)(scale * d);
    }
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// Pair store: r_hat = r / rms(r), e_hat = e / rms(r), FP32.
__global__ void k_store_pair(int64_t n3, const double* __restrict__ r, const double* __restrict__ e, double inv,
                             float* __restrict__ pr, float* __restrict__ pe) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n3) return;
  pr[i] = (float)(r[i] * inv);
  pe[i] = (float)(e[i] * inv);
}
__global__ __launch_bounds__(256) void k_sumsq(int64_t n, const double* __restrict__ a, double* __restrict__ part) {
  __shared__ double sh[256];
  double s = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) s += a[i] * a[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// Adam on the FP32 master weights.
__global__ void k_adam(int n, float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                       float lr, float b1, float b2, float eps, float c1, float c2) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1 - b1) * gi, vi = b2 * v[i] + (1 - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Master weights [t][co][ci] (logical sizes) -> BF16 MFMA layouts:
//   forward  [t][co_pad][ci_pad]
//   backward (data) [26 - t][ci_pad'][co_pad'] (taps mirrored, roles swapped)
__global__ void k_pack(const float* __restrict__ w, int cout, int cin, int cop, int cip, int transpose,
                       __bf16* __restrict__ out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = 27 * cop * cip;
  if (i >= n) return;
  const int t = i / (cop * cip), r = i % (cop * cip), a = r / cip, bb = r % cip;
  float val = 0;
  if (!transpose) {
    if (a < cout && bb < cin) val = w[(t * cout + a) * cin + bb];
  } else {
    // output channel a = input channel of the layer, input channel bb = output channel of the layer
    if (a < cin && bb < cout) val = w[((26 - t) * cout + bb) * cin + a];
  }
  out[i] = (__bf16)val;
}

// gradient of the master layout from the padded wgrad result [t][co][cip]
__global__ void k_unpad_grad(const float* __restrict__ gp, int cout, int cin, int cop, int cip, float* __restrict__ g) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = 27 * cout * cin;
  if (i >= n) return;
  const int t = i / (cout * cin), r = i % (cout * cin), co = r / cin, ci = r % cin;
  g[i] = gp[(t * cop + co) * cip + ci];
}

inline dim3 g1(int64_t n) { return dim3((unsigned)((n + 255) / 256)); }

}  // namespace

// ===================================================================== host
// layer shapes: (cin, cout, cin_pad, cout_pad)
static const int LCIN[3] = {3, 32, 32}, LCOUT[3] = {32, 32, 3}, LCIP[3] = {8, 32, 32}, LCOP[3] = {32, 32, 16};

struct ge_cnn_state {
  float *w, *g, *m, *v;            // master weights, gradient, Adam moments (CNN_NW floats)
  __bf16 *wf[3], *wb[3];           // packed forward / backward weights
  __bf16 *act1, *act2;             // whole-grid activations [N][32]
  int64_t grid_cap;
  // training buffers
  __bf16 *t_in, *t_a1, *t_a2, *t_dz, *t_d2, *t_d1;
  float *t_z, *t_tgt, *t_part, *t_gpad, *t_loss;
  int *t_meta;
  float* t_wts;
  int t_B, t_n;
  // pair store
  float *pr, *pe;
  int npairs, cap_pairs, harvest;
  int adam_t;
  int ready;
};

extern "C" int ge_cnn_init(ge_ctx* c, uint32_t seed, int max_pairs);
static const int64_t CNN_OFF[4] = {0, 27 * 3 * 32, 27 * 3 * 32 + 27 * 32 * 32, 27 * 3 * 32 + 27 * 32 * 32 + 27 * 32 * 3};
#define CNN_NW (27 * 3 * 32 + 27 * 32 * 32 + 27 * 32 * 3)

template <typename P>
static int calloc_dev(ge_ctx* c, P** p, size_t bytes) {
  *p = nullptr;
  hipError_t e = hipMalloc((void**)p, bytes ? bytes : 8);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return ge_fail(c, GE_ERR_OOM, "CNN buffer allocation failed");
  }
  return GE_OK;
}

static ge_cnn_state* cnn(ge_ctx* c) { return (ge_cnn_state*)c->cnn; }

void ge_cnn_free(ge_ctx* c) {
  ge_cnn_state* s = cnn(c);
  if (!s) return;
  void* ptrs[] = {s->w, s->g, s->m, s->v, s->wf[0], s->wf[1], s->wf[2], s->wb[0], s->wb[1], s->wb[2], s->act1,
                  s->act2, s->t_in, s->t_a1, s->t_a2, s->t_dz, s->t_d2, s->t_d1, s->t_z, s->t_tgt, s->t_part,
                  s->t_gpad, s->t_loss, s->t_meta, s->t_wts, s->pr, s->pe};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  delete s;
  c->cnn = nullptr;
}

static int pack_weights(ge_ctx* c) {
  ge_cnn_state* s = cnn(c);
  for (int l = 0; l < 3; ++l) {
    int n = 27 * LCOP[l] * LCIP[l];
    hipLaunchKernelGGL(k_pack, g1(n), dim3(256), 0, c->stream, s->w + CNN_OFF[l], LCOUT[l], LCIN[l], LCOP[l], LCIP[l], 0,
                       s->wf[l]);
    // backward-data weights: output channels = this layer's inputs (padded), inputs = its outputs (padded)
    const int bco = l == 0 ? 32 : LCIP[l], bci = LCOP[l];
    n = 27 * bco * bci;
    hipLaunchKernelGGL(k_pack, g1(n), dim3(256), 0, c->stream, s->w + CNN_OFF[l], LCOUT[l], LCIN[l], bco, bci, 1,
                       s->wb[l]);
  }
  GE_HIP(c, hipGetLastError());
  return GE_OK;
}

static int cnn_setup(ge_ctx* c) {
  if (cnn(c)) return GE_OK;
  ge_cnn_state* s = new ge_cnn_state();
  std::memset(s, 0, sizeof(*s));
  c->cnn = s;
  int rc = GE_OK;
  if (!rc) rc = calloc_dev(c, &s->w, sizeof(float) * CNN_NW);
  if (!rc) rc = calloc_dev(c, &s->g, sizeof(float) * CNN_NW);
  if (!rc) rc = calloc_dev(c, &s->m, sizeof(float) * CNN_NW);
  if (!rc) rc = calloc_dev(c, &s->v, sizeof(float) * CNN_NW);
  for (int l = 0; l < 3 && !rc; ++l) {
    rc = calloc_dev(c, &s->wf[l], sizeof(__bf16) * 27 * LCOP[l] * LCIP[l]);
    if (!rc) rc = calloc_dev(c, &s->wb[l], sizeof(__bf16) * 27 * 32 * 32);
  }
  if (rc) {
    ge_cnn_free(c);
    return rc;
  }
  GE_HIP(c, hipMemsetAsync(s->m, 0, sizeof(float) * CNN_NW, c->stream));
  GE_HIP(c, hipMemsetAsync(s->v, 0, sizeof(float) * CNN_NW, c->stream));
  return GE_OK;
}

// Initial weights: the network starts near the identity map (channel pairs
// +x_i, -x_i through ReLU, recombined by the last layer) plus small
// counter-hashed noise, so that an untrained preconditioner does no harm.
static uint32_t hash32(uint32_t x) {
  x ^= x >> 16; x *= 0x7feb352dU; x ^= x >> 15; x *= 0x846ca68bU; x ^= x >> 16;
  return x;
}
static int cnn_init_weights(ge_ctx* c, uint32_t seed, double noise) {
  std::vector<float> h(CNN_NW, 0.0f);
  uint32_t k = 0;
  for (int l = 0; l < 3; ++l) {
    const double a = noise * std::sqrt(6.0 / (27.0 * LCIN[l]));
    for (int64_t i = CNN_OFF[l]; i < CNN_OFF[l + 1]; ++i) {
      const double u = (hash32(seed * 0x9E3779B9U + (k++)) + 0.5) / 4294967296.0;
      h[i] = (float)(a * (2 * u - 1));
    }
  }
  const int ctr = 13;  // centre tap
  for (int i = 0; i < 3; ++i) {
    h[CNN_OFF[0] + (ctr * 32 + 2 * i) * 3 + i] += 1.0f;       // L1: ch 2i = +x_i
    h[CNN_OFF[0] + (ctr * 32 + 2 * i + 1) * 3 + i] -= 1.0f;   //     ch 2i+1 = -x_i
    for (int j = 0; j < 2; ++j)                                // L2: pass both through
      h[CNN_OFF[1] + (ctr * 32 + 2 * i + j) * 32 + 2 * i + j] += 1.0f;
    h[CNN_OFF[2] + (ctr * 3 + i) * 32 + 2 * i] += 1.0f;        // L3: x_i = ch 2i - ch 2i+1
    h[CNN_OFF[2] + (ctr * 3 + i) * 32 + 2 * i + 1] -= 1.0f;
  }
  ge_cnn_state* s = cnn(c);
  GE_HIP(c, hipStreamSynchronize(c->stream));
  GE_HIP(c, hipMemcpyAsync(s->w, h.data(), sizeof(float) * CNN_NW, hipMemcpyHostToDevice, c->stream));
  s->adam_t = 0;
  GE_HIP(c, hipMemsetAsync(s->m, 0, sizeof(float) * CNN_NW, c->stream));
  GE_HIP(c, hipMemsetAsync(s->v, 0, sizeof(float) * CNN_NW, c->stream));
  s->ready = 1;
  int rc = pack_weights(c);
  GE_HIP(c, hipStreamSynchronize(c->stream));  // h goes out of scope
  return rc;
}

template <int CIN, int COUT, int MODE>
static void conv(ge_ctx* c, const ConvArgs& A) {
  const int64_t total = (int64_t)A.ox * A.oy * A.oz * A.B;
  const int64_t tiles = (total + 15) / 16;
  int64_t nb = (tiles + 3) / 4;
  if (nb > 4096) nb = 4096;
  hipLaunchKernelGGL((k_conv<CIN, COUT, MODE>), dim3((unsigned)nb), dim3(256), 0, c->stream, A);
}

template <int CIN, int COUT, bool IN_F64, bool OUT_F64>
static void conv_tile(ge_ctx* c, TileArgs A) {
  A.ntx = (A.nx + TLX - 1) / TLX;
  A.nty = (A.ny + TLY - 1) / TLY;
  A.ntiles = A.ntx * A.nty * ((A.nz + TLZ - 1) / TLZ);
  // resident workgroups per CU from the LDS footprint (160 KB per CU), 256 CUs
  constexpr int lds = (27 * COUT * CIN + THN * CIN) * 2;
  constexpr int per_cu = (160 * 1024) / lds < 4 ? (160 * 1024) / lds : 4;
  const int nb = A.ntiles < 256 * per_cu ? A.ntiles : 256 * per_cu;
  hipLaunchKernelGGL((k_conv_tile<CIN, COUT, IN_F64, OUT_F64>), dim3(nb), dim3(TNT), 0, c->stream, A);
}

// z = N(s v) / s on the whole periodic grid (v, z: device double [3][N]).
// On a walled grid the network's domain is periodic over the node planes
// that are not wholly held (an inflow plane is left out), and z = v on the
// held components, whose operator rows are the identity.
int ge_cnn_apply_grid(ge_ctx* c, const double* v, double* z, double scale) {
  ge_cnn_state* s = cnn(c);
  if (!s || !s->ready) return ge_fail(c, GE_ERR_STATE, "CNN weights not initialised");
  const int64_t N = c->G.N;
  if (s->grid_cap < N) {
    if (s->act1) { (void)hipFree(s->act1); s->act1 = nullptr; }
    if (s->act2) { (void)hipFree(s->act2); s->act2 = nullptr; }
    int rc = calloc_dev(c, &s->act1, sizeof(__bf16) * 32 * N);
    if (!rc) rc = calloc_dev(c, &s->act2, sizeof(__bf16) * 32 * N);
    if (rc) return rc;
    s->grid_cap = N;
  }
  TileArgs A;
  std::memset(&A, 0, sizeof(A));
  A.nx = cnn_nx(c->G); A.sx = c->G.n[0]; A.ny = c->G.n[1]; A.nz = c->G.n[2]; A.N = N; A.s = scale;
  A.v = v; A.w = s->wf[0]; A.out = s->act1;
  conv_tile<8, 32, true, false>(c, A);
  A.v = nullptr; A.in = s->act1; A.w = s->wf[1]; A.out = s->act2;
  conv_tile<32, 32, false, false>(c, A);
  A.in = s->act2; A.w = s->wf[2]; A.out = nullptr; A.z = z;
  conv_tile<32, 16, false, true>(c, A);
  if (walled(c->G)) {
    const int64_t np2 = 2 * (int64_t)c->G.n[1] * c->G.n[2];
    hipLaunchKernelGGL(k_hold_rows, dim3((unsigned)((np2 + 255) / 256)), dim3(256), 0, c->stream, c->G, v, z);
  }
  GE_HIP(c, hipGetLastError());
  return GE_OK;
}

static int ensure_train_buffers(ge_ctx* c, int B, int n) {
  ge_cnn_state* s = cnn(c);
  if (s->t_B == B && s->t_n == n) return GE_OK;
  void** old[] = {(void**)&s->t_in, (void**)&s->t_a1, (void**)&s->t_a2, (void**)&s->t_dz, (void**)&s->t_d2,
                  (void**)&s->t_d1, (void**)&s->t_z, (void**)&s->t_tgt, (void**)&s->t_part, (void**)&s->t_gpad,
                  (void**)&s->t_loss, (void**)&s->t_meta, (void**)&s->t_wts};
  for (auto p : old)
    if (*p) { (void)hipFree(*p); *p = nullptr; }
  const int64_t v6 = (int64_t)(n + 6) * (n + 6) * (n + 6), v4 = (int64_t)(n + 4) * (n + 4) * (n + 4),
                v2 = (int64_t)(n + 2) * (n + 2) * (n + 2), v0 = (int64_t)n * n * n;
  int rc = calloc_dev(c, &s->t_in, sizeof(__bf16) * 8 * v6 * B);
  if (!rc) rc = calloc_dev(c, &s->t_a1, sizeof(__bf16) * 32 * v4 * B);
  if (!rc) rc = calloc_dev(c, &s->t_a2, sizeof(__bf16) * 32 * v2 * B);
  if (!rc) rc = calloc_dev(c, &s->t_dz, sizeof(__bf16) * 16 * v0 * B);
  if (!rc) rc = calloc_dev(c, &s->t_d2, sizeof(__bf16) * 32 * v2 * B);
  if (!rc) rc = calloc_dev(c, &s->t_d1, sizeof(__bf16) * 32 * v4 * B);
  if (!rc) rc = calloc_dev(c, &s->t_z, sizeof(float) * 16 * v0 * B);
  if (!rc) rc = calloc_dev(c, &s->t_tgt, sizeof(float) * 3 * v0 * B);
  const int64_t nchunk = (v4 * B + 1023) / 1024;
  if (!rc) rc = calloc_dev(c, &s->t_part, sizeof(float) * nchunk * 27 * 32 * 32);
  if (!rc) rc = calloc_dev(c, &s->t_gpad, sizeof(float) * 27 * 32 * 32);
  if (!rc) rc = calloc_dev(c, &s->t_loss, sizeof(float) * 1024);
  if (!rc) rc = calloc_dev(c, &s->t_meta, sizeof(int) * 5 * B);
  if (!rc) rc = calloc_dev(c, &s->t_wts, sizeof(float) * 2 * B);
  if (rc) return rc;
  s->t_B = B;
  s->t_n = n;
  return GE_OK;
}

template <int CIN, int COUT>
static void wgrad(ge_ctx* c, const __bf16* in, const __bf16* dout, int B, int o, float* gpad) {
  ge_cnn_state* s = cnn(c);
  WgradArgs A;
  A.in = in; A.dout = dout; A.part = s->t_part; A.B = B; A.ox = A.oy = A.oz = o;
  A.chunk = 1024;
  const int64_t total = (int64_t)o * o * o * B;
  const int nchunk = (int)((total + A.chunk - 1) / A.chunk);
  hipLaunchKernelGGL((k_wgrad<CIN, COUT>), dim3(nchunk, 27), dim3(64), 0, c->stream, A);
  constexpr int CP = CIN < 16 ? 16 : CIN;
  const int64_t n = 27 * COUT * CP;
  hipLaunchKernelGGL(k_reduce_chunks, g1(n), dim3(256), 0, c->stream, s->t_part, nchunk, n, gpad);
}

// Forward + backward on the crops already in t_in / t_tgt; gradient into s->g,
// loss (mean squared error) returned.
static int train_step_grad(ge_ctx* c, double* loss) {
  ge_cnn_state* s = cnn(c);
  const int B = s->t_B, n = s->t_n;
  ConvArgs A;
  std::memset(&A, 0, sizeof(A));
  A.B = B;
  // forward (valid geometry): (n+6)^3 -> (n+4)^3 -> (n+2)^3 -> n^3
  A.ix = A.iy = A.iz = n + 6; A.ox = A.oy = A.oz = n + 4;
  A.in = s->t_in; A.w = s->wf[0]; A.out_bf = s->t_a1; A.relu = 1;
  conv<8, 32, CONV_VALID>(c, A);
  A.ix = A.iy = A.iz = n + 4; A.ox = A.oy = A.oz = n + 2;
  A.in = s->t_a1; A.w = s->wf[1]; A.out_bf = s->t_a2;
  conv<32, 32, CONV_VALID>(c, A);
  A.ix = A.iy = A.iz = n + 2; A.ox = A.oy = A.oz = n;
  A.in = s->t_a2; A.w = s->wf[2]; A.out_bf = nullptr; A.out_f32 = s->t_z; A.relu = 0;
  conv<32, 16, CONV_VALID>(c, A);
  // loss and dL/dz
  const int64_t nout = (int64_t)n * n * n * B;
  hipLaunchKernelGGL(k_loss_grad, dim3(256), dim3(256), 0, c->stream, nout, s->t_z, s->t_tgt, s->t_dz, s->t_loss);
  // layer 3: weight gradient and data gradient (masked by layer 2's ReLU)
  wgrad<32, 16>(c, s->t_a2, s->t_dz, B, n, s->t_gpad);
  hipLaunchKernelGGL(k_unpad_grad, g1(27 * 3 * 32), dim3(256), 0, c->stream, s->t_gpad, 3, 32, 16, 32, s->g + CNN_OFF[2]);
  std::memset(&A, 0, sizeof(A));
  A.B = B;
  A.ix = A.iy = A.iz = n; A.ox = A.oy = A.oz = n + 2;
  A.in = s->t_dz; A.w = s->wb[2]; A.out_bf = s->t_d2; A.mask = s->t_a2;
  conv<16, 32, CONV_FULL>(c, A);
  // layer 2
  wgrad<32, 32>(c, s->t_a1, s->t_d2, B, n + 2, s->t_gpad);
  hipLaunchKernelGGL(k_unpad_grad, g1(27 * 32 * 32), dim3(256), 0, c->stream, s->t_gpad, 32, 32, 32, 32, s->g + CNN_OFF[1]);
  A.ix = A.iy = A.iz = n + 2; A.ox = A.oy = A.oz = n + 4;
  A.in = s->t_d2; A.w = s->wb[1]; A.out_bf = s->t_d1; A.mask = s->t_a1;
  conv<32, 32, CONV_FULL>(c, A);
  // layer 1
  wgrad<8, 32>(c, s->t_in, s->t_d1, B, n + 4, s->t_gpad);
  hipLaunchKernelGGL(k_unpad_grad, g1(27 * 32 * 3), dim3(256), 0, c->stream, s->t_gpad, 32, 3, 32, 16, s->g + CNN_OFF[0]);
  GE_HIP(c, hipGetLastError());
  float lp[256];
  GE_HIP(c, hipMemcpyAsync(lp, s->t_loss, sizeof(lp), hipMemcpyDeviceToHost, c->stream));
  GE_HIP(c, hipStreamSynchronize(c->stream));
  double L = 0;
  for (int i = 0; i < 256; ++i) L += lp[i];
  *loss = L / (3.0 * (double)nout);
  return GE_OK;
}

int ge_cnn_harvesting(const ge_ctx* c) { return (c && c->cnn) ? ((ge_cnn_state*)c->cnn)->harvest : 0; }

// Master weights, Adam moments and step of the network (checkpoints).
int ge_cnn_export(ge_ctx* c, std::vector<float>& w, std::vector<float>& m, std::vector<float>& v, int& t,
                  int& cap) {
  ge_cnn_state* s = cnn(c);
  if (!s || !s->ready) return ge_fail(c, GE_ERR_STATE, "no learned preconditioner");
  w.resize(CNN_NW);
  m.resize(CNN_NW);
  v.resize(CNN_NW);
  GE_HIP(c, hipMemcpyAsync(w.data(), s->w, sizeof(float) * CNN_NW, hipMemcpyDeviceToHost, c->stream));
  GE_HIP(c, hipMemcpyAsync(m.data(), s->m, sizeof(float) * CNN_NW, hipMemcpyDeviceToHost, c->stream));
  GE_HIP(c, hipMemcpyAsync(v.data(), s->v, sizeof(float) * CNN_NW, hipMemcpyDeviceToHost, c->stream));
  GE_HIP(c, hipStreamSynchronize(c->stream));
  t = s->adam_t;
  cap = s->cap_pairs;
  return GE_OK;
}

int ge_cnn_import(ge_ctx* c, const float* w, const float* m, const float* v, int t, int cap) {
  int rc = ge_cnn_init(c, 0, cap);
  if (rc) return rc;
  ge_cnn_state* s = cnn(c);
  GE_HIP(c, hipMemcpyAsync(s->w, w, sizeof(float) * CNN_NW, hipMemcpyHostToDevice, c->stream));
  GE_HIP(c, hipMemcpyAsync(s->m, m, sizeof(float) * CNN_NW, hipMemcpyHostToDevice, c->stream));
  GE_HIP(c, hipMemcpyAsync(s->v, v, sizeof(float) * CNN_NW, hipMemcpyHostToDevice, c->stream));
  s->adam_t = t;
  rc = pack_weights(c);
  GE_HIP(c, hipStreamSynchronize(c->stream));  // the host arrays may go out of scope
  return rc;
}

// ----------------------------------------------------------------- C ABI
extern "C" {

int ge_cnn_init(ge_ctx* c, uint32_t seed, int max_pairs) {
  if (!c) return GE_ERR_ARG;
  if (c->G.dim != 3) return ge_fail(c, GE_ERR_ARG, "the CNN preconditioner is built for 3D grids");
  if (max_pairs < 0 || max_pairs > 1024) return ge_fail(c, GE_ERR_ARG, "max_pairs out of range (0..1024)");
  int rc = cnn_setup(c);
  if (rc) return rc;
  ge_cnn_state* s = cnn(c);
  if (!s->pr) s->cap_pairs = max_pairs ? max_pairs : 64;
  return cnn_init_weights(c, seed, 0.02);
}

int ge_cnn_size(void) { return CNN_NW; }

int ge_cnn_weights(ge_ctx* c, int set, float* host_w) {
  if (!c || !host_w) return GE_ERR_ARG;
  ge_cnn_state* s = cnn(c);
  if (!s) return ge_fail(c, GE_ERR_STATE, "ge_cnn_init first");
  GE_HIP(c, hipStreamSynchronize(c->stream));
  if (set) {
    GE_HIP(c, hipMemcpyAsync(s->w, host_w, sizeof(float) * CNN_NW, hipMemcpyHostToDevice, c->stream));
    s->ready = 1;
    int rc = pack_weights(c);
    GE_HIP(c, hipStreamSynchronize(c->stream));
    return rc;
  }
  GE_HIP(c, hipMemcpyAsync(host_w, s->w, sizeof(float) * CNN_NW, hipMemcpyDeviceToHost, c->stream));
  GE_HIP(c, hipStreamSynchronize(c->stream));
  return GE_OK;
}

int ge_cnn_apply_scaled(ge_ctx* c, const double* r, double* z, double scale) {
  if (!c || !r || !z) return GE_ERR_ARG;
  if (!(scale > 0.0 && scale < INFINITY)) return ge_fail(c, GE_ERR_ARG, "ge_cnn_apply_scaled: scale must be finite and positive");
  return ge_cnn_apply_grid(c, r, z, scale);
}

int ge_cnn_apply(ge_ctx* c, const double* r, double* z) {
  if (!c || !r || !z) return GE_ERR_ARG;
  // normalise by the RMS of r (the network is positively homogeneous)
  const int64_t n3 = 3 * c->G.N;
  hipLaunchKernelGGL(k_sumsq, dim3(256), dim3(256), 0, c->stream, n3, r, c->partials);
  double h[256];
  GE_HIP(c, hipMemcpyAsync(h, c->partials, sizeof(h), hipMemcpyDeviceToHost, c->stream));
  GE_HIP(c, hipStreamSynchronize(c->stream));
  double ss = 0;
  for (int i = 0; i < 256; ++i) ss += h[i];
  const double rms = std::sqrt(ss / (double)n3);
  return ge_cnn_apply_grid(c, r, z, rms > 0 ? 1.0 / rms : 1.0);
}

int ge_cnn_add_pair(ge_ctx* c, const double* r, const double* e) {
  if (!c || !r || !e) return GE_ERR_ARG;
  int rc = cnn_setup(c);
  if (rc) return rc;
  ge_cnn_state* s = cnn(c);
  const int64_t n3 = 3 * c->G.N;
  if (!s->pr) {
    if (s->cap_pairs < 1) s->cap_pairs = 64;
    rc = calloc_dev(c, &s->pr, sizeof(float) * n3 * s->cap_pairs);
    if (!rc) rc = calloc_dev(c, &s->pe, sizeof(float) * n3 * s->cap_pairs);
    if (rc) return rc;
  }
  hipLaunchKernelGGL(k_sumsq, dim3(256), dim3(256), 0, c->stream, n3, r, c->partials);
  double h[256];
  GE_HIP(c, hipMemcpyAsync(h, c->partials, sizeof(h), hipMemcpyDeviceToHost, c->stream));
  GE_HIP(c, hipStreamSynchronize(c->stream));
  double ss = 0;
  for (int i = 0; i < 256; ++i) ss += h[i];
  if (!(ss > 0)) return ge_fail(c, GE_ERR_ARG, "zero residual pair");
  const double inv = 1.0 / std::sqrt(ss / (double)n3);
  const int slot = s->npairs % s->cap_pairs;  // ring buffer: newest pairs replace the oldest
  hipLaunchKernelGGL(k_store_pair, g1(n3), dim3(256), 0, c->stream, n3, r, e, inv, s->pr + (int64_t)slot * n3,
                     s->pe + (int64_t)slot * n3);
  GE_HIP(c, hipGetLastError());
  s->npairs++;
  return GE_OK;
}

int ge_cnn_harvest(ge_ctx* c, int flags) {
  if (!c) return GE_ERR_ARG;
  if (flags & ~(GE_HARVEST_SOLUTION | GE_HARVEST_KRYLOV)) return ge_fail(c, GE_ERR_ARG, "unknown harvest flags");
  int rc = cnn_setup(c);
  if (rc) return rc;
  cnn(c)->harvest = flags;
  return GE_OK;
}

int ge_cnn_npairs(const ge_ctx* c) {
  if (!c || !c->cnn) return 0;
  ge_cnn_state* s = (ge_cnn_state*)c->cnn;
  return s->npairs < s->cap_pairs ? s->npairs : s->cap_pairs;
}

int ge_cnn_train(ge_ctx* c, const ge_train_cfg* cfg, ge_train_report* rep) {
  if (!c || !cfg) return GE_ERR_ARG;
  ge_cnn_state* s = cnn(c);
  if (!s || !s->ready) return ge_fail(c, GE_ERR_STATE, "ge_cnn_init first");
  const int np = ge_cnn_npairs(c);
  if (np < 1) return ge_fail(c, GE_ERR_STATE, "no training pairs (harvest or add pairs first)");
  const int B = cfg->batch, n = cfg->crop;
  if (B < 1 || B > 64 || n < 2 || n > 64) return ge_fail(c, GE_ERR_ARG, "batch (1..64) / crop (2..64)");
  auto t0 = std::chrono::steady_clock::now();
  int rc = ensure_train_buffers(c, B, n);
  if (rc) return rc;
  std::vector<int> meta(5 * B);
  std::vector<float> wts(2 * B);
  double first = 0, last = 0;
  uint32_t ctr = 0;
  for (int it = 0; it < cfg->iters; ++it) {
    for (int b = 0; b < B; ++b) {
      auto u = [&]() { return (hash32(cfg->seed * 0x85EBCA6BU + (ctr++) * 0x9E3779B9U) + 0.5) / 4294967296.0; };
      meta[5 * b + 0] = (int)(u() * cnn_nx(c->G));
      meta[5 * b + 1] = (int)(u() * c->G.n[1]);
      meta[5 * b + 2] = (int)(u() * c->G.n[2]);
      meta[5 * b + 3] = (int)(u() * np) % np;
      meta[5 * b + 4] = (int)(u() * np) % np;
      const double ang = 2.0 * M_PI * u();
      wts[2 * b] = (float)std::cos(ang);
      wts[2 * b + 1] = (float)std::sin(ang);
    }
    GE_HIP(c, hipMemcpyAsync(s->t_meta, meta.data(), sizeof(int) * 5 * B, hipMemcpyHostToDevice, c->stream));
    GE_HIP(c, hipMemcpyAsync(s->t_wts, wts.data(), sizeof(float) * 2 * B, hipMemcpyHostToDevice, c->stream));
    CropArgs CA;
    CA.pr = s->pr; CA.pe = s->pe; CA.N = c->G.N;
    CA.nx = cnn_nx(c->G); CA.sx = c->G.n[0]; CA.ny = c->G.n[1]; CA.nz = c->G.n[2];
    CA.n = n; CA.meta = s->t_meta; CA.wts = s->t_wts; CA.in = s->t_in; CA.tgt = s->t_tgt; CA.B = B;
    const int64_t vin = (int64_t)(n + 6) * (n + 6) * (n + 6) * B;
    hipLaunchKernelGGL(k_make_crops, g1(vin), dim3(256), 0, c->stream, CA);
    double L;
    if ((rc = train_step_grad(c, &L))) return rc;
    if (!std::isfinite(L)) return ge_fail(c, GE_ERR_NONFINITE, "non-finite training loss");
    if (it == 0) first = L;
    last = L;
    s->adam_t++;
    const float b1 = (float)cfg->beta1, b2 = (float)cfg->beta2;
    const float c1 = 1.0f - std::pow(b1, (float)s->adam_t), c2 = 1.0f - std::pow(b2, (float)s->adam_t);
    hipLaunchKernelGGL(k_adam, g1(CNN_NW), dim3(256), 0, c->stream, CNN_NW, s->w, s->g, s->m, s->v, (float)cfg->lr, b1,
                       b2, (float)cfg->eps, c1, c2);
    if ((rc = pack_weights(c))) return rc;
  }
  GE_HIP(c, hipStreamSynchronize(c->stream));
  if (rep) {
    rep->steps = cfg->iters;
    rep->loss_first = first;
    rep->loss_last = last;
    rep->pairs = np;
    rep->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  return GE_OK;
}

// Loss and gradient of the master weights for caller-provided crops (device):
// in_crops FP32 [B][(n+6)^3][3], tgt FP32 [B][n^3][3]; grad FP32 [ge_cnn_size()].
int ge_cnn_loss_grad(ge_ctx* c, int B, int n, const float* in_crops, const float* tgt, float* grad, double* loss) {
  if (!c || !in_crops || !tgt || !grad || !loss || B < 1 || n < 1) return GE_ERR_ARG;
  ge_cnn_state* s = cnn(c);
  if (!s || !s->ready) return ge_fail(c, GE_ERR_STATE, "ge_cnn_init first");
  int rc = ensure_train_buffers(c, B, n);
  if (rc) return rc;
  const int64_t vin = (int64_t)(n + 6) * (n + 6) * (n + 6) * B, vout = (int64_t)n * n * n * B;
  GE_HIP(c, hipStreamSynchronize(c->stream));
  // pack the FP32 crops into the BF16 8-channel layout
  std::vector<float> hin(3 * vin);
  GE_HIP(c, hipMemcpyAsync(hin.data(), in_crops, sizeof(float) * 3 * vin, hipMemcpyDeviceToHost, c->stream));
  GE_HIP(c, hipStreamSynchronize(c->stream));
  std::vector<__bf16> hb(8 * vin);
  for (int64_t i = 0; i < vin; ++i)
    for (int ch = 0; ch < 8; ++ch) hb[8 * i + ch] = (__bf16)(ch < 3 ? hin[3 * i + ch] : 0.0f);
  GE_HIP(c, hipMemcpyAsync(s->t_in, hb.data(), sizeof(__bf16) * 8 * vin, hipMemcpyHostToDevice, c->stream));
  GE_HIP(c, hipMemcpyAsync(s->t_tgt, tgt, sizeof(float) * 3 * vout, hipMemcpyDeviceToDevice, c->stream));
  if ((rc = train_step_grad(c, loss))) return rc;
  GE_HIP(c, hipMemcpyAsync(grad, s->g, sizeof(float) * CNN_NW, hipMemcpyDeviceToDevice, c->stream));
  GE_HIP(c, hipStreamSynchronize(c->stream));
  return GE_OK;
}

}  // extern "C"
