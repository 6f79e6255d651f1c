// Restarted GMRES in FP64 for the implicit E system.  The Arnoldi basis is
// orthogonalised by classical Gram-Schmidt applied twice (CGS2).  For restart
// lengths up to 32 the second pass of each vector is delayed into the next
// step's first pass (two reads of the basis per step, no separate
// normalisation; see the delayed-CGS2 section below); longer restarts run the
// plain CGS2 step, where each pass is one fused multi-dot and one fused
// multi-axpy and, for up to 16 basis vectors, the first pass's update and the
// second pass's dots share one read of the basis.  Dot products are block
// partial sums reduced in a fixed order, so every run gives the same bits.
// The Hessenberg column travels to the host once per iteration.
#include <chrono>
#include <cmath>
#include <vector>

#include "ge_internal.h"

namespace {

constexpr int KB = 256;       // threads per block
constexpr int KRED = 512;     // blocks of a multi-dot
constexpr int HSTRIDE = 64;   // layout of the small device buffer hdev

// part[i * KRED + b] = block b's share of V_i . w, i < NV
template <int NV>
__global__ __launch_bounds__(KB) void k_multidot(const double* __restrict__ V, int64_t ld, const double* __restrict__ w,
                                                 int64_t n, double* __restrict__ part) {
  __shared__ double sh[NV][KB];
  double a[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) a[i] = 0;
  for (int64_t k = blockIdx.x * (int64_t)KB + threadIdx.x; k < n; k += (int64_t)gridDim.x * KB) {
    const double wk = w[k];
#pragma unroll
    for (int i = 0; i < NV; ++i) a[i] += V[i * ld + k] * wk;
  }
#pragma unroll
  for (int i = 0; i < NV; ++i) sh[i][threadIdx.x] = a[i];
  __syncthreads();
  for (int s = KB / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s)
#pragma unroll
      for (int i = 0; i < NV; ++i) sh[i][threadIdx.x] += sh[i][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x < NV) part[threadIdx.x * KRED + blockIdx.x] = sh[threadIdx.x][0];
}

// out[i] = sum_b part[i * KRED + b] in a fixed tree order (one block per i),
// and add[i] += out[i] when add is given
__global__ __launch_bounds__(KB) void k_reduce(const double* __restrict__ part, double* __restrict__ out,
                                               double* __restrict__ add = nullptr) {
  __shared__ double sh[KB];
  const int i = blockIdx.x;
  double a = 0;
  for (int b = threadIdx.x; b < KRED; b += KB) a += part[i * KRED + b];
  sh[threadIdx.x] = a;
  __syncthreads();
  for (int s = KB / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[i] = sh[0];
    if (add) add[i] += sh[0];
  }
}

// w[k] += sign * sum_{i<nv} h[i] V_i[k]
__global__ __launch_bounds__(KB) void k_multiaxpy(double* __restrict__ w, const double* __restrict__ V, int64_t ld, int nv,
                                                  const double* __restrict__ h, double sign, int64_t n) {
  __shared__ double hs[HSTRIDE];
  if (threadIdx.x < nv) hs[threadIdx.x] = h[threadIdx.x];
  __syncthreads();
  for (int64_t k = blockIdx.x * (int64_t)KB + threadIdx.x; k < n; k += (int64_t)gridDim.x * KB) {
    double s = 0;
    for (int i = 0; i < nv; ++i) s += hs[i] * V[i * ld + k];
    w[k] += sign * s;
  }
}

// The second CGS pass fused into the first pass's update: w[k] -= sum_i h[i]
// V_i[k], then part[i * KRED + b] = block b's share of V_i . w (new w), with
// V_i[k] read once for both.  Same grid, element order and per-element
// arithmetic as k_multiaxpy followed by k_multidot, so the results are the
// same bits.
template <int NV>
__global__ __launch_bounds__(KB) void k_axpy_dot(double* __restrict__ w, const double* __restrict__ V, int64_t ld,
                                                 const double* __restrict__ h, int64_t n, double* __restrict__ part) {
  __shared__ double sh[NV][KB];
  __shared__ double hs[NV];
  if (threadIdx.x < NV) hs[threadIdx.x] = h[threadIdx.x];
  __syncthreads();
  double a[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) a[i] = 0;
  for (int64_t k = blockIdx.x * (int64_t)KB + threadIdx.x; k < n; k += (int64_t)gridDim.x * KB) {
    double v[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = V[i * ld + k];
    double s = 0;
#pragma unroll
    for (int i = 0; i < NV; ++i) s += hs[i] * v[i];
    const double wk = w[k] + (-1.0) * s;
    w[k] = wk;
#pragma unroll
    for (int i = 0; i < NV; ++i) a[i] += v[i] * wk;
  }
#pragma unroll
  for (int i = 0; i < NV; ++i) sh[i][threadIdx.x] = a[i];
  __syncthreads();
  for (int s2 = KB / 2; s2 > 0; s2 >>= 1) {
    if (threadIdx.x < s2)
#pragma unroll
      for (int i = 0; i < NV; ++i) sh[i][threadIdx.x] += sh[i][threadIdx.x + s2];
    __syncthreads();
  }
  if (threadIdx.x < NV) part[threadIdx.x * KRED + blockIdx.x] = sh[threadIdx.x][0];
}

// The second pass's update fused with the squared norm of its result:
// w[k] -= sum_{i<NV} h[i] V_i[k]; part[b] = block b's share of w . w.  The
// vector count is a template argument so that the NV loads of an element are
// issued together.
template <int NV>
__global__ __launch_bounds__(KB) void k_axpy_norm(double* __restrict__ w, const double* __restrict__ V, int64_t ld,
                                                  const double* __restrict__ h, int64_t n, double* __restrict__ part) {
  __shared__ double hs[NV];
  __shared__ double sh[KB];
  if (threadIdx.x < NV) hs[threadIdx.x] = h[threadIdx.x];
  __syncthreads();
  double a = 0;
  for (int64_t k = blockIdx.x * (int64_t)KB + threadIdx.x; k < n; k += (int64_t)gridDim.x * KB) {
    double v[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = V[i * ld + k];
    double s = 0;
#pragma unroll
    for (int i = 0; i < NV; ++i) s += hs[i] * v[i];
    const double wk = w[k] + (-1.0) * s;
    w[k] = wk;
    a += wk * wk;
  }
  sh[threadIdx.x] = a;
  __syncthreads();
  for (int s2 = KB / 2; s2 > 0; s2 >>= 1) {
    if (threadIdx.x < s2) sh[threadIdx.x] += sh[threadIdx.x + s2];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// v = w / sqrt(*nrm2)
__global__ void k_normalize(double* __restrict__ v, const double* __restrict__ w, const double* __restrict__ nrm2, int64_t n) {
  const double inv = 1.0 / sqrt(*nrm2);
  for (int64_t k = blockIdx.x * (int64_t)KB + threadIdx.x; k < n; k += (int64_t)gridDim.x * KB) v[k] = w[k] * inv;
}
// v = v / sqrt(*nrm2), in place
__global__ void k_normalize_inplace(double* __restrict__ v, const double* __restrict__ nrm2, int64_t n) {
  const double inv = 1.0 / sqrt(*nrm2);
  for (int64_t k = blockIdx.x * (int64_t)KB + threadIdx.x; k < n; k += (int64_t)gridDim.x * KB) v[k] = v[k] * inv;
}
// r = b - r
__global__ void k_residual(double* __restrict__ r, const double* __restrict__ b, int64_t n) {
  for (int64_t k = blockIdx.x * (int64_t)KB + threadIdx.x; k < n; k += (int64_t)gridDim.x * KB) r[k] = b[k] - r[k];
}
__global__ void k_add(double* __restrict__ x, const double* __restrict__ z, int64_t n) {
  for (int64_t k = blockIdx.x * (int64_t)KB + threadIdx.x; k < n; k += (int64_t)gridDim.x * KB) x[k] += z[k];
}
__global__ void k_sum2(double* __restrict__ a, const double* __restrict__ b, int nv) {
  int i = threadIdx.x;
  if (i < nv) a[i] += b[i];
}

// ---------------------------------------------------------------- delayed CGS2
// Arnoldi with the second Gram-Schmidt pass of each vector delayed into the
// next step's first pass (one read of the basis per pass instead of two).
// Step j holds the final orthonormal basis V_0 .. V_{j-1} and the candidate
// U_j = nrm_j u_j (u_j: the new direction after one projection, nrm_j its
// norm); z_j = u_j (or its preconditioned image) and Y = nrm_j A z_j.
//   pass A: s = V^T u_j, t = V^T A z_j, alpha = u_j . u_j, tau = u_j . A z_j
//   v_j = (u_j - V s) / rho, rho^2 = alpha - s . s   (the delayed second pass)
//   h_{<j,j} = t, h_jj = (tau - s . t) / rho          (first pass of A z_j)
//   pass B: V_j = v_j, U_{j+1} = A z_j - V t - h_jj v_j, and its squared norm
// The previous column is completed with s and rho (the relation A z_{j-1} =
// V h + h_{j,j-1} u_j rewritten in v_j).

// Pass A: rows i < NVC of part hold V_i . u, rows NVC + i hold V_i . y, and
// with TAIL the last two rows u . u and u . y (block partials, KRED blocks).
template <int NVC, bool TAIL>
__global__ __launch_bounds__(KB) void k_dc_dots(const double* __restrict__ V, int64_t ld, const double* __restrict__ u,
                                                const double* __restrict__ y, int64_t n, double* __restrict__ part) {
  constexpr int R = 2 * NVC + (TAIL ? 2 : 0);
  __shared__ double sh[R][KB];
  double a[R];
#pragma unroll
  for (int r = 0; r < R; ++r) a[r] = 0;
  for (int64_t k = blockIdx.x * (int64_t)KB + threadIdx.x; k < n; k += (int64_t)gridDim.x * KB) {
    const double uk = u[k], yk = y[k];
#pragma unroll
    for (int i = 0; i < NVC; ++i) {
      const double v = V[i * ld + k];
      a[i] += v * uk;
      a[NVC + i] += v * yk;
    }
    if (TAIL) {
      a[2 * NVC] += uk * uk;
      a[2 * NVC + 1] += uk * yk;
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) sh[r][threadIdx.x] = a[r];
  __syncthreads();
  for (int st = KB / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st)
#pragma unroll
      for (int r = 0; r < R; ++r) sh[r][threadIdx.x] += sh[r][threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x < R) part[threadIdx.x * KRED + blockIdx.x] = sh[threadIdx.x][0];
}

// Coefficients of step j in a fixed order (one thread).  D: V^T U_j (j),
// V^T Y (j), U_j . U_j, U_j . Y; *nrm2 = |U_j|^2.  C: s_i / rho (j), t_i (j),
// then 1 / (nrm rho), 1 / nrm, h_jj, rho, nrm.
__global__ void k_dc_coef(int j, const double* __restrict__ D, const double* __restrict__ nrm2, double* __restrict__ C) {
  if (threadIdx.x != 0) return;
  const double nrm = sqrt(*nrm2), inv = 1.0 / nrm;
  double ss = 0, st = 0;
  for (int i = 0; i < j; ++i) {
    const double si = D[i] * inv, ti = D[j + i] * inv;
    ss += si * si;
    st += si * ti;
  }
  const double al = D[2 * j] * inv * inv, ta = D[2 * j + 1] * inv * inv;
  const double r2 = al - ss;
  const double rho = sqrt(r2 > 0 ? r2 : 0.0);  // 0: breakdown, reported through the non-finite coefficients
  for (int i = 0; i < j; ++i) {
    C[i] = D[i] * inv / rho;
    C[j + i] = D[j + i] * inv;
  }
  C[2 * j] = inv / rho;
  C[2 * j + 1] = inv;
  C[2 * j + 2] = (ta - st) / rho;
  C[2 * j + 3] = rho;
  C[2 * j + 4] = nrm;
}

// Pass B: v = cu U_j - sum_i cs_i V_i (into vout), w = cy Y - sum_i ct_i V_i
// - chv v (into wout), part[b] = block b's share of w . w.
template <int NV>
__global__ __launch_bounds__(KB) void k_dc_update(const double* __restrict__ V, int64_t ld, const double* __restrict__ u,
                                                  const double* __restrict__ y, const double* __restrict__ C, int64_t n,
                                                  double* __restrict__ vout, double* __restrict__ wout,
                                                  double* __restrict__ part) {
  __shared__ double sh[KB];
  // the coefficients are the same for every thread: wave-uniform scalar
  // loads, so that all NV basis loads of an element are issued together
  typedef const __attribute__((address_space(4))) double* cdp;
  const cdp cc = reinterpret_cast<cdp>(reinterpret_cast<uintptr_t>(C));
  double cs[NV > 0 ? NV : 1], ct[NV > 0 ? NV : 1];
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    cs[i] = cc[i];
    ct[i] = cc[NV + i];
  }
  const double cu = cc[2 * NV], cy = cc[2 * NV + 1], chv = cc[2 * NV + 2];
  double acc = 0;
  for (int64_t k = blockIdx.x * (int64_t)KB + threadIdx.x; k < n; k += (int64_t)gridDim.x * KB) {
    double v[NV > 0 ? NV : 1];
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = V[i * ld + k];
    double sv = 0, sw = 0;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      sv += cs[i] * v[i];
      sw += ct[i] * v[i];
    }
    const double vk = cu * u[k] - sv;
    const double wk = cy * y[k] - sw - chv * vk;
    vout[k] = vk;
    wout[k] = wk;
    acc += wk * wk;
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int st = KB / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

inline dim3 vgrid(int64_t n) {
  int64_t b = (n + KB - 1) / KB;
  return dim3((unsigned)(b < 8192 ? b : 8192));
}

}  // namespace

// dots[i] = V_i . w for i < nv (device output)
static int multidot(ge_ctx* c, const double* V, int64_t ld, int nv, const double* w, int64_t n, double* dots) {
  for (int i0 = 0; i0 < nv; i0 += 8) {
    const int k = nv - i0 < 8 ? nv - i0 : 8;
    const double* Vi = V + (int64_t)i0 * ld;
    double* part = c->partials;
    switch (k) {
#define MD(K) case K: hipLaunchKernelGGL(k_multidot<K>, dim3(KRED), dim3(KB), 0, c->stream, Vi, ld, w, n, part); break;
      MD(1) MD(2) MD(3) MD(4) MD(5) MD(6) MD(7) MD(8)
#undef MD
    }
    hipLaunchKernelGGL(k_reduce, dim3(k), dim3(KB), 0, c->stream, part, dots + i0);
  }
  GE_HIP(c, hipGetLastError());
  return GE_OK;
}

// Passes 1b and 2 of CGS2 for nv <= 16 vectors (h1 from the first multi-dot):
// w -= V h1, h2 = V^T w, h1 += h2, w -= V h2, |w|^2, with V read twice
// instead of three times.
static int cgs2_fused(ge_ctx* c, double* w, const double* V, int64_t ld, int nv, double* h1, double* h2,
                      double* nrm2, int64_t n) {
  double* part = c->partials;
  switch (nv) {
#define AD(K) case K: hipLaunchKernelGGL(k_axpy_dot<K>, dim3(KRED), dim3(KB), 0, c->stream, w, V, ld, h1, n, part); break;
    AD(1) AD(2) AD(3) AD(4) AD(5) AD(6) AD(7) AD(8) AD(9) AD(10) AD(11) AD(12) AD(13) AD(14) AD(15) AD(16)
#undef AD
    default: return ge_fail(c, GE_ERR_ARG, "fused Gram-Schmidt takes at most 16 vectors");
  }
  hipLaunchKernelGGL(k_reduce, dim3(nv), dim3(KB), 0, c->stream, part, h2, h1);
  switch (nv) {
#define AN(K) case K: hipLaunchKernelGGL(k_axpy_norm<K>, dim3(KRED), dim3(KB), 0, c->stream, w, V, ld, h2, n, part); break;
    AN(1) AN(2) AN(3) AN(4) AN(5) AN(6) AN(7) AN(8) AN(9) AN(10) AN(11) AN(12) AN(13) AN(14) AN(15) AN(16)
#undef AN
  }
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(KB), 0, c->stream, part, nrm2);
  GE_HIP(c, hipGetLastError());
  return GE_OK;
}

// Layout of the small device buffer hdev (mirrored by the pinned hhost) for
// the delayed-CGS2 cycle, after the part the CGS2 cycle uses.
constexpr int DC_MAX = 32;  // restart lengths up to this run the delayed-CGS2 cycle
constexpr int DOFF = 256, COFF = 384, NOFF = 520;

// Pass A of step j into D: D[0, j) = V^T u, D[j, 2j) = V^T y, D[2j] = u . u,
// D[2j + 1] = u . y (the basis in chunks of 8 vectors; u and y with the last).
static int dc_dots(ge_ctx* c, const double* V, int64_t ld, int j, const double* u, const double* y, int64_t n,
                   double* D) {
  double* part = c->partials;
  if (j == 0) {
    hipLaunchKernelGGL((k_dc_dots<0, true>), dim3(KRED), dim3(KB), 0, c->stream, V, ld, u, y, n, part);
    hipLaunchKernelGGL(k_reduce, dim3(2), dim3(KB), 0, c->stream, part, D, nullptr);
  }
  for (int c0 = 0; c0 < j; c0 += 8) {
    const int k = j - c0 < 8 ? j - c0 : 8;
    const bool tail = c0 + k == j;
    const double* Vc = V + (int64_t)c0 * ld;
    switch (2 * k + (tail ? 1 : 0)) {
#define DD(K)                                                                                                  \
  case 2 * K:                                                                                                  \
    hipLaunchKernelGGL((k_dc_dots<K, false>), dim3(KRED), dim3(KB), 0, c->stream, Vc, ld, u, y, n, part);      \
    break;                                                                                                     \
  case 2 * K + 1:                                                                                              \
    hipLaunchKernelGGL((k_dc_dots<K, true>), dim3(KRED), dim3(KB), 0, c->stream, Vc, ld, u, y, n, part);       \
    break;
      DD(1) DD(2) DD(3) DD(4) DD(5) DD(6) DD(7) DD(8)
#undef DD
    }
    hipLaunchKernelGGL(k_reduce, dim3(k), dim3(KB), 0, c->stream, part, D + c0, nullptr);
    hipLaunchKernelGGL(k_reduce, dim3(k), dim3(KB), 0, c->stream, part + (int64_t)k * KRED, D + j + c0, nullptr);
    if (tail) hipLaunchKernelGGL(k_reduce, dim3(2), dim3(KB), 0, c->stream, part + (int64_t)2 * k * KRED, D + 2 * j, nullptr);
  }
  GE_HIP(c, hipGetLastError());
  return GE_OK;
}

// Pass B of step j (coefficients C on the device): vout = v_j, wout =
// U_{j+1}, *nrm2 = |U_{j+1}|^2.
static int dc_update(ge_ctx* c, const double* V, int64_t ld, int j, const double* u, const double* y,
                     const double* C, int64_t n, double* vout, double* wout, double* nrm2) {
  double* part = c->partials;
  switch (j) {
#define DU(K)                                                                                                      \
  case K:                                                                                                          \
    hipLaunchKernelGGL((k_dc_update<K>), dim3(KRED), dim3(KB), 0, c->stream, V, ld, u, y, C, n, vout, wout, part); \
    break;
    DU(0) DU(1) DU(2) DU(3) DU(4) DU(5) DU(6) DU(7) DU(8) DU(9) DU(10) DU(11) DU(12) DU(13) DU(14) DU(15)
    DU(16) DU(17) DU(18) DU(19) DU(20) DU(21) DU(22) DU(23) DU(24) DU(25) DU(26) DU(27) DU(28) DU(29) DU(30)
    DU(31)
#undef DU
    default: return ge_fail(c, GE_ERR_ARG, "delayed Gram-Schmidt takes at most 32 vectors");
  }
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(KB), 0, c->stream, part, nrm2, nullptr);
  GE_HIP(c, hipGetLastError());
  return GE_OK;
}

// min |beta e1 - H y| over the first k columns of the unrotated Hessenberg
// H ((m + 1) x m, row-major) by Givens rotations in column order: returns the
// residual norm and, when ys is given, the solution y (k values).
static double hess_lsq(const std::vector<double>& H, int m, int k, double beta, double* ys) {
  std::vector<double> R((size_t)(k + 1) * (k > 0 ? k : 1)), cs(k > 0 ? k : 1), sn(k > 0 ? k : 1), g(k + 1, 0.0);
  for (int i = 0; i <= k; ++i)
    for (int j = 0; j < k; ++j) R[(size_t)i * k + j] = H[(size_t)i * m + j];
  g[0] = beta;
  for (int j = 0; j < k; ++j) {
    for (int i = 0; i < j; ++i) {
      const double a0 = cs[i] * R[(size_t)i * k + j] + sn[i] * R[(size_t)(i + 1) * k + j];
      const double a1 = -sn[i] * R[(size_t)i * k + j] + cs[i] * R[(size_t)(i + 1) * k + j];
      R[(size_t)i * k + j] = a0;
      R[(size_t)(i + 1) * k + j] = a1;
    }
    const double a = R[(size_t)j * k + j], b = R[(size_t)(j + 1) * k + j];
    const double den = std::sqrt(a * a + b * b);
    cs[j] = den > 0 ? a / den : 1.0;
    sn[j] = den > 0 ? b / den : 0.0;
    R[(size_t)j * k + j] = den;
    R[(size_t)(j + 1) * k + j] = 0.0;
    g[j + 1] = -sn[j] * g[j];
    g[j] = cs[j] * g[j];
  }
  if (ys)
    for (int i = k - 1; i >= 0; --i) {
      double t = g[i];
      for (int l = i + 1; l < k; ++l) t -= R[(size_t)i * k + l] * ys[l];
      ys[i] = t / R[(size_t)i * k + i];
    }
  return std::fabs(g[k]);
}

static int precond_apply(ge_ctx* c, int precond, const double* x, double* y, int64_t n) {
  if (precond == GE_PC_JACOBI) return ge_launch_jacobi_apply(c, x, y);
  GE_HIP(c, hipMemcpyAsync(y, x, sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream));
  return GE_OK;
}

// Restart cycles of (flexible) GMRES with the delayed-CGS2 Arnoldi process.
// The update directions are the candidates U_j themselves (no
// preconditioner), their preconditioned images (network: Zb_j = nrm_j
// M(u_j)), or D^-1 applied to their combination (Jacobi); the last column of
// a cycle keeps its one-pass coefficients, and every cycle starts from the
// true residual, which decides convergence.
static int gmres_dcgs(ge_ctx* c, double tol, int maxit, int m, double bref, double cnn_scale, int& precond, int& it,
                      int& restarts, int& conv, double& rel, int& fallback) {
  const int64_t n = 3 * c->G.N;
  int rc;
  if (!c->Ub) {
    if (hipMalloc((void**)&c->Ub, sizeof(double) * n * (DC_MAX + 1)) != hipSuccess) {
      c->Ub = nullptr;
      (void)hipGetLastError();
      return ge_fail(c, GE_ERR_OOM, "GMRES candidate basis allocation failed");
    }
  }
  double* x = c->Eth;
  double* V = c->V;
  double* U = c->Ub;
  double* Y = c->kw;
  double* z = c->Zp;
  double* hd = c->hdev;
  double* hh = c->hhost;
  double* D = hd + DOFF;
  double* C = hd + COFF;
  double* nrm2 = hd + NOFF;
  std::vector<double> H((size_t)(m + 1) * m), nrm(m + 1), yv(m);
  while (true) {
    // r = b - A x into U_0, |r|^2
    if ((rc = ge_launch_apply_A(c, x, U))) return rc;
    hipLaunchKernelGGL(k_residual, vgrid(n), dim3(KB), 0, c->stream, U, c->rhs, n);
    if ((rc = multidot(c, U, n, 1, U, n, nrm2))) return rc;
    GE_HIP(c, hipMemcpyAsync(hh + NOFF, nrm2, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    GE_HIP(c, hipStreamSynchronize(c->stream));
    const double beta = std::sqrt(hh[NOFF]);
    if (!std::isfinite(beta)) return ge_fail(c, GE_ERR_NONFINITE, "non-finite residual in GMRES");
    const double rel_prev = rel;
    rel = beta / bref;
    if (rel <= tol) { conv = 1; break; }
    if (it >= maxit) break;
    if (precond == GE_PC_CNN && restarts > 0 && rel > 0.5 * rel_prev) {
      // a whole flexible cycle gained less than a factor 2: the network does
      // not help on this system; finish with plain GMRES from here
      precond = GE_PC_NONE;
      fallback = 1;
    }
    std::fill(H.begin(), H.end(), 0.0);
    nrm[0] = beta;
    int k = 0;
    bool abandon = false;
    for (int j = 0; j < m && it < maxit; ++j) {
      double* Uj = U + (int64_t)j * n;
      const double* av_in = Uj;
      if (precond == GE_PC_CNN) {
        double* zj = c->Zb + (int64_t)j * n;
        if ((rc = ge_cnn_apply_grid(c, Uj, zj, cnn_scale / nrm[j]))) return rc;
        av_in = zj;
      } else if (precond != GE_PC_NONE) {
        if ((rc = precond_apply(c, precond, Uj, z, n))) return rc;
        av_in = z;
      }
      if ((rc = ge_launch_apply_A(c, av_in, Y))) return rc;
      if ((rc = dc_dots(c, V, n, j, Uj, Y, n, D))) return rc;
      hipLaunchKernelGGL(k_dc_coef, dim3(1), dim3(64), 0, c->stream, j, D, nrm2, C);
      if ((rc = dc_update(c, V, n, j, Uj, Y, C, n, V + (int64_t)j * n, U + (int64_t)(j + 1) * n, nrm2))) return rc;
      GE_HIP(c, hipMemcpyAsync(hh + COFF, C, sizeof(double) * (NOFF - COFF + 1), hipMemcpyDeviceToHost, c->stream));
      GE_HIP(c, hipStreamSynchronize(c->stream));
      ++it;
      const double* cf = hh + COFF;
      const double hjj = cf[2 * j + 2], rho = cf[2 * j + 3], nn = std::sqrt(hh[NOFF]);
      bool finite = std::isfinite(hjj) && std::isfinite(rho) && std::isfinite(nn);
      for (int i = 0; i < 2 * j; ++i) finite = finite && std::isfinite(cf[i]);
      if (!finite && precond == GE_PC_CNN) {
        // the learned preconditioner produced NaN/Inf: drop this cycle and
        // continue with plain GMRES from the current iterate
        precond = GE_PC_NONE;
        fallback = 1;
        abandon = true;
        break;
      }
      if (!finite) return ge_fail(c, GE_ERR_NONFINITE, "non-finite Arnoldi vector");
      if (rho < 0.5) break;  // the candidate lies (nearly) in the basis: close the cycle at column j - 1
      // column j - 1 in the final basis: u_j = V s + rho v_j
      if (j > 0) {
        const double hp = H[(size_t)j * m + j - 1];
        for (int i = 0; i < j; ++i) H[(size_t)i * m + j - 1] += hp * cf[i] * rho;
        H[(size_t)j * m + j - 1] = hp * rho;
      }
      for (int i = 0; i < j; ++i) H[(size_t)i * m + j] = cf[j + i];
      H[(size_t)j * m + j] = hjj;
      H[(size_t)(j + 1) * m + j] = nn;
      nrm[j + 1] = nn;
      k = j + 1;
      if (hess_lsq(H, m, k, beta, nullptr) <= tol * bref || nn == 0.0) break;
    }
    if (abandon) continue;
    if (k == 0) return ge_fail(c, GE_ERR_NONFINITE, "GMRES breakdown at the first Arnoldi step");
    c->kr_last = k;
    hess_lsq(H, m, k, beta, yv.data());
    bool yfinite = true;
    for (int i = 0; i < k; ++i) yfinite = yfinite && std::isfinite(yv[i]);
    if (!yfinite) {
      // singular least-squares system: only a preconditioner that maps some
      // u_j to zero (or a null direction of A) gets here
      if (precond != GE_PC_CNN) return ge_fail(c, GE_ERR_NONFINITE, "singular GMRES least-squares system");
      precond = GE_PC_NONE;
      fallback = 1;
      continue;
    }
    double* yc = hh + 192;  // update coefficients y_j / nrm_j (the directions are nrm_j times unit)
    for (int i = 0; i < k; ++i) yc[i] = yv[i] / nrm[i];
    GE_HIP(c, hipMemcpyAsync(hd + 192, yc, sizeof(double) * k, hipMemcpyHostToDevice, c->stream));
    if (precond == GE_PC_NONE) {
      hipLaunchKernelGGL(k_multiaxpy, vgrid(n), dim3(KB), 0, c->stream, x, U, n, k, hd + 192, 1.0, n);
    } else if (precond == GE_PC_CNN) {
      hipLaunchKernelGGL(k_multiaxpy, vgrid(n), dim3(KB), 0, c->stream, x, c->Zb, n, k, hd + 192, 1.0, n);
    } else {
      GE_HIP(c, hipMemsetAsync(Y, 0, sizeof(double) * n, c->stream));
      hipLaunchKernelGGL(k_multiaxpy, vgrid(n), dim3(KB), 0, c->stream, Y, U, n, k, hd + 192, 1.0, n);
      if ((rc = precond_apply(c, precond, Y, z, n))) return rc;
      hipLaunchKernelGGL(k_add, vgrid(n), dim3(KB), 0, c->stream, x, z, n);
    }
    GE_HIP(c, hipGetLastError());
    ++restarts;
  }
  return GE_OK;
}

int ge_gmres(ge_ctx* c, double tol, int maxit, int m, int precond, ge_solve_report* rep) {
  // the solve's own wall time starts once the queued deposit work is done
  GE_HIP(c, hipStreamSynchronize(c->stream));
  auto t0 = std::chrono::steady_clock::now();
  const int64_t n = 3 * c->G.N;
  if (m < 1 || m > c->kr_m) return ge_fail(c, GE_ERR_ARG, "restart out of range (1.." + std::to_string(c->kr_m) + ")");
  if (precond != GE_PC_NONE && precond != GE_PC_JACOBI && precond != GE_PC_CNN)
    return ge_fail(c, GE_ERR_ARG, "unknown preconditioner");
  if (precond == GE_PC_CNN && !c->Zb) {
    // flexible GMRES keeps the preconditioned vectors z_j
    if (hipMalloc((void**)&c->Zb, sizeof(double) * n * c->kr_m) != hipSuccess) {
      c->Zb = nullptr;
      (void)hipGetLastError();
      return ge_fail(c, GE_ERR_OOM, "flexible GMRES basis allocation failed");
    }
  }
  const double cnn_scale = std::sqrt((double)n);  // basis vectors have unit norm: RMS = 1/sqrt(n)
  int fallback = 0;
  int rc;
  c->kr_last = 0;
  double* x = c->Eth;
  double* V = c->V;
  double* w = c->kw;
  double* z = c->Zp;
  double* hd = c->hdev;  // [0,64): h1, [64,128): h2, [128]: |w|^2, [192,256): y
  if (precond == GE_PC_JACOBI && (rc = ge_launch_jacobi_setup(c))) return rc;
  // ||b||
  double* hh = c->hhost;  // pinned mirror of hd: read-backs and the y upload are direct copies
  if ((rc = multidot(c, c->rhs, n, 1, c->rhs, n, hd + 128))) return rc;
  GE_HIP(c, hipMemcpyAsync(hh + 128, hd + 128, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  GE_HIP(c, hipStreamSynchronize(c->stream));
  double bnorm = std::sqrt(hh[128]);
  if (!(bnorm >= 0) || std::isinf(bnorm)) return ge_fail(c, GE_ERR_NONFINITE, "non-finite right-hand side");
  const double bref = bnorm > 0 ? bnorm : 1.0;
  int it = 0, restarts = 0, conv = 0;
  double rel = 0;
  if (m <= DC_MAX) {
    if ((rc = gmres_dcgs(c, tol, maxit, m, bref, cnn_scale, precond, it, restarts, conv, rel, fallback))) return rc;
  } else {
  std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), s(m + 1);
  double* y = hh + 192;  // host side of hd[192, 192 + m), m <= 64
  while (true) {
    // r = b - A x, beta = ||r||
    if ((rc = ge_launch_apply_A(c, x, V))) return rc;
    hipLaunchKernelGGL(k_residual, vgrid(n), dim3(KB), 0, c->stream, V, c->rhs, n);
    if ((rc = multidot(c, V, n, 1, V, n, hd + 128))) return rc;
    GE_HIP(c, hipMemcpyAsync(hh + 128, hd + 128, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    GE_HIP(c, hipStreamSynchronize(c->stream));
    const double beta = std::sqrt(hh[128]);
    if (!std::isfinite(beta)) return ge_fail(c, GE_ERR_NONFINITE, "non-finite residual in GMRES");
    const double rel_prev = rel;
    rel = beta / bref;
    if (rel <= tol) { conv = 1; break; }
    if (it >= maxit) break;
    if (precond == GE_PC_CNN && restarts > 0 && rel > 0.5 * rel_prev) {
      // a whole flexible cycle gained less than a factor 2: the network does
      // not help on this system; finish with plain GMRES from here
      precond = GE_PC_NONE;
      fallback = 1;
    }
    hipLaunchKernelGGL(k_normalize_inplace, vgrid(n), dim3(KB), 0, c->stream, V, hd + 128, n);
    std::fill(s.begin(), s.end(), 0.0);
    s[0] = beta;
    int k = 0;
    for (int j = 0; j < m && it < maxit; ++j) {
      double* vj = V + (int64_t)j * n;
      double* vn = V + (int64_t)(j + 1) * n;
      const double* av_in = vj;
      if (precond == GE_PC_CNN) {
        double* zj = c->Zb + (int64_t)j * n;
        if ((rc = ge_cnn_apply_grid(c, vj, zj, cnn_scale))) return rc;
        av_in = zj;
      } else if (precond != GE_PC_NONE) {
        if ((rc = precond_apply(c, precond, vj, z, n))) return rc;
        av_in = z;
      }
      if ((rc = ge_launch_apply_A(c, av_in, w))) return rc;
      // CGS2
      if ((rc = multidot(c, V, n, j + 1, w, n, hd))) return rc;
      if (j + 1 <= 16) {
        if ((rc = cgs2_fused(c, w, V, n, j + 1, hd, hd + HSTRIDE, hd + 128, n))) return rc;
      } else {
        hipLaunchKernelGGL(k_multiaxpy, vgrid(n), dim3(KB), 0, c->stream, w, V, n, j + 1, hd, -1.0, n);
        if ((rc = multidot(c, V, n, j + 1, w, n, hd + HSTRIDE))) return rc;
        hipLaunchKernelGGL(k_multiaxpy, vgrid(n), dim3(KB), 0, c->stream, w, V, n, j + 1, hd + HSTRIDE, -1.0, n);
        hipLaunchKernelGGL(k_sum2, dim3(1), dim3(HSTRIDE), 0, c->stream, hd, hd + HSTRIDE, j + 1);
        if ((rc = multidot(c, w, n, 1, w, n, hd + 128))) return rc;
      }
      hipLaunchKernelGGL(k_normalize, vgrid(n), dim3(KB), 0, c->stream, vn, w, hd + 128, n);
      GE_HIP(c, hipGetLastError());
      GE_HIP(c, hipMemcpyAsync(hh, hd, sizeof(double) * (2 * HSTRIDE + 1), hipMemcpyDeviceToHost, c->stream));
      GE_HIP(c, hipStreamSynchronize(c->stream));
      ++it;
      for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = hh[i];
      const double hn = std::sqrt(hh[128]);
      bool finite = std::isfinite(hn);
      for (int i = 0; i <= j; ++i) finite = finite && std::isfinite(hh[i]);
      if (!finite && precond == GE_PC_CNN) {
        // the learned preconditioner produced NaN/Inf: drop this cycle and
        // continue with plain GMRES from the current iterate
        precond = GE_PC_NONE;
        fallback = 1;
        k = -1;
        break;
      }
      if (!finite) return ge_fail(c, GE_ERR_NONFINITE, "non-finite Arnoldi vector");
      H[(size_t)(j + 1) * m + j] = hn;
      for (int i = 0; i < j; ++i) {
        const double a0 = cs[i] * H[(size_t)i * m + j] + sn[i] * H[(size_t)(i + 1) * m + j];
        const double a1 = -sn[i] * H[(size_t)i * m + j] + cs[i] * H[(size_t)(i + 1) * m + j];
        H[(size_t)i * m + j] = a0;
        H[(size_t)(i + 1) * m + j] = a1;
      }
      const double a = H[(size_t)j * m + j], bb = H[(size_t)(j + 1) * m + j];
      const double den = std::sqrt(a * a + bb * bb);
      cs[j] = den > 0 ? a / den : 1.0;
      sn[j] = den > 0 ? bb / den : 0.0;
      H[(size_t)j * m + j] = den;
      H[(size_t)(j + 1) * m + j] = 0.0;
      s[j + 1] = -sn[j] * s[j];
      s[j] = cs[j] * s[j];
      k = j + 1;
      if (std::fabs(s[j + 1]) <= tol * bref || hn == 0.0) break;
    }
    if (k < 0) continue;  // cycle abandoned (fallback)
    c->kr_last = k;
    // y = H^{-1} s; x += M^{-1} (V y)  (flexible: x += Z y)
    bool yfinite = true;
    for (int i = k - 1; i >= 0; --i) {
      double t = s[i];
      for (int l = i + 1; l < k; ++l) t -= H[(size_t)i * m + l] * y[l];
      y[i] = t / H[(size_t)i * m + i];
      yfinite = yfinite && std::isfinite(y[i]);
    }
    if (!yfinite) {
      // singular least-squares system: only a preconditioner that maps some
      // v_j to zero (or a null direction of A) gets here
      if (precond != GE_PC_CNN) return ge_fail(c, GE_ERR_NONFINITE, "singular GMRES least-squares system");
      precond = GE_PC_NONE;
      fallback = 1;
      continue;
    }
    GE_HIP(c, hipMemcpyAsync(hd + 192, y, sizeof(double) * k, hipMemcpyHostToDevice, c->stream));
    if (precond == GE_PC_NONE) {
      hipLaunchKernelGGL(k_multiaxpy, vgrid(n), dim3(KB), 0, c->stream, x, V, n, k, hd + 192, 1.0, n);
    } else if (precond == GE_PC_CNN) {
      hipLaunchKernelGGL(k_multiaxpy, vgrid(n), dim3(KB), 0, c->stream, x, c->Zb, n, k, hd + 192, 1.0, n);
    } else {
      GE_HIP(c, hipMemsetAsync(w, 0, sizeof(double) * n, c->stream));
      hipLaunchKernelGGL(k_multiaxpy, vgrid(n), dim3(KB), 0, c->stream, w, V, n, k, hd + 192, 1.0, n);
      if ((rc = precond_apply(c, precond, w, z, n))) return rc;
      hipLaunchKernelGGL(k_add, vgrid(n), dim3(KB), 0, c->stream, x, z, n);
    }
    GE_HIP(c, hipGetLastError());
    ++restarts;
  }
  }
  if (rep) {
    rep->iterations = it;
    rep->restarts = restarts;
    rep->converged = conv;
    rep->relres = rel;
    rep->bnorm = bnorm;
    rep->fallback = fallback;
    rep->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  return conv ? GE_OK : GE_WARN_NOT_CONVERGED;
}
