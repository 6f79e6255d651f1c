// Diagnostics without allocation: the FP64 energies, momenta and Gauss
// residual of ge_diagnostics with their reduction partials in a file-scope
// device array instead of the context's library-allocated buffer, read back
// through the pinned host buffer the context allocated at creation.
//
// The array is one per GPU (each device that loads the library holds its own
// copy until the process ends).  Host code never passes the array's name to
// a kernel: its device address is looked up once per device with
// hipGetSymbolAddress (ge_noalloc_setup, called by ge_create with that device
// current) and only that address is used.
#include <cstring>
#include <mutex>

#include "ge_internal.h"

// Capacity in doubles: the block partials of one reduction (4 quantities x
// GE_DIAG_BLOCKS blocks), then the 4 sums.  The reductions always run on
// GE_DIAG_BLOCKS blocks, so every grid and species size fits.
constexpr int GE_NOALLOC_DOUBLES = 4 * GE_DIAG_BLOCKS + 4;

static __device__ __align__(256) double scratch[GE_NOALLOC_DOUBLES];

namespace {

constexpr int GE_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[GE_MAX_DEVICES];  // device address of 'scratch' per device (null: not looked up)

// sums[k] = sum over b of part[k][b], b ascending: the same order as the
// host loop of ge_diagnostics, so both give the same bits
__global__ void k_sum_partials(const double* __restrict__ part, int nbk, double* __restrict__ sums) {
  const int k = threadIdx.x;
  if (k >= 4) return;
  double a = 0;
  for (int b = 0; b < nbk; ++b) a += part[k * nbk + b];
  sums[k] = a;
}

// reduce part (already written on the stream) into out4 on the host
int reduce_into(ge_ctx* c, double* ptr, double* out4) {
  double* sums = ptr + 4 * GE_DIAG_BLOCKS;
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(64), 0, c->stream, ptr, GE_DIAG_BLOCKS, sums);
  GE_HIP(c, hipGetLastError());
  GE_HIP(c, hipMemcpyAsync(c->hhost, sums, sizeof(double) * 4, hipMemcpyDeviceToHost, c->stream));
  GE_HIP(c, hipStreamSynchronize(c->stream));
  for (int k = 0; k < 4; ++k) out4[k] = c->hhost[k];
  return GE_OK;
}

}  // namespace

// Look up this device's address of the scratch array once (the context's
// device is current: ge_create runs on it).
int ge_noalloc_setup(ge_ctx* c) {
  int dev = 0;
  GE_HIP(c, hipGetDevice(&dev));
  if (dev < 0 || dev >= GE_MAX_DEVICES) return ge_fail(c, GE_ERR_ARG, "device index beyond the scratch table");
  c->device = dev;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    GE_HIP(c, hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_ptr[dev] = (double*)p;
  }
  return GE_OK;
}

extern "C" {

int ge_diagnostics_noalloc(ge_ctx* c, ge_diag* out) {
  if (!c || !out) return GE_ERR_ARG;
  if (c->push_pending)
    return ge_fail(c, GE_ERR_STATE, "a push is not settled yet (its far movers may need a re-sort that allocates): "
                                    "call ge_sync first");
  if (4 * GE_DIAG_BLOCKS + 4 > GE_NOALLOC_DOUBLES)
    return ge_fail(c, GE_ERR_ARG, "diagnostic reductions larger than the static scratch");
  double* ptr = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (c->device >= 0 && c->device < GE_MAX_DEVICES) ptr = g_scratch_ptr[c->device];
  }
  if (!ptr) return ge_fail(c, GE_ERR_STATE, "static scratch address not set up for this context's device");
  if (!c->hhost) return ge_fail(c, GE_ERR_STATE, "no pinned read-back buffer");
  std::memset(out, 0, sizeof(*out));
  out->nsp = c->nsp;
  double f[4];
  int rc = ge_launch_field_diag_part(c, ptr);
  if (!rc) rc = reduce_into(c, ptr, f);
  if (rc) return rc;
  const double k8 = c->G.dV / (8.0 * M_PI);
  out->W_E = f[0] * k8;
  out->W_B = f[1] * k8;
  out->gauss = f[3] > 0 ? std::sqrt(f[2] / f[3]) : std::sqrt(f[2]);
  for (int s = 0; s < c->nsp; ++s) {
    double m4[4];
    rc = ge_launch_particle_moments_part(c, s, ptr);
    if (!rc) rc = reduce_into(c, ptr, m4);
    if (rc) return rc;
    out->K[s] = 0.5 * c->sp[s].m * m4[0];
    for (int d = 0; d < 3; ++d) out->P[s][d] = c->sp[s].m * m4[1 + d];
  }
  return GE_OK;
}

}  // extern "C"
