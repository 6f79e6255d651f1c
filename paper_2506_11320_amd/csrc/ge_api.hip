// C ABI of the gfx950 GL-ECSIM library: context, buffers and step sequencing.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "ge_internal.h"

int ge_fail(ge_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

namespace {

template <typename P>
int dalloc(ge_ctx* c, P** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 8;
  hipError_t e = hipMalloc((void**)p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return ge_fail(c, GE_ERR_OOM, "hipMalloc of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e));
  }
  return GE_OK;
}
template <typename P>
void dfree(P*& p) {
  if (p) (void)hipFree((void*)p);
  p = nullptr;
}

// Read the flag block (synchronises): the errors raised since the last read,
// and the statistics of a push that has not been settled yet.  Far movers of
// that push are re-sorted here, before anything reads the particles again.
int check_flags(ge_ctx* c) {
  int h[GE_FL_COUNT];
  if (c->push_pending)
    for (int s = 0; s < c->nsp; ++s) {
      int rc = ge_launch_move_max(c, s);
      if (rc) return rc;
    }
  GE_HIP(c, hipMemcpyAsync(h, c->flags, sizeof(h), hipMemcpyDeviceToHost, c->stream));
  GE_HIP(c, hipStreamSynchronize(c->stream));
  bool any = false;
  for (int k = 0; k < GE_FL_COUNT; ++k) any = any || h[k] != 0;
  if (any) GE_HIP(c, hipMemsetAsync(c->flags, 0, sizeof(h), c->stream));
  std::string stuck;
  if (h[GE_FL_LOAD] && c->inject_pending) {
    // an injected particle named a cell outside the domain (or a ghost
    // cell): the pending injections are dropped before any re-sort indexes
    // with them
    for (int s = 0; s < c->nsp; ++s) c->sp[s].inj_n = 0;
  }
  if (c->push_pending || c->inject_pending) {
    const bool pushed = c->push_pending;
    c->push_pending = 0;
    c->inject_pending = 0;
    if (pushed) c->moves.pushes += 1;
    for (int s = 0; s < c->nsp; ++s) {
      SpeciesBuf& S = c->sp[s];
      int zero[4] = {0, 0, 0, 0};
      const int* st = pushed ? h + GE_FL_SPECIES + 4 * s : zero;
      float mv;
      std::memcpy(&mv, &st[1], sizeof(mv));
      c->moves.far[s] += st[0];
      c->moves.gone[s] += st[3];
      c->moves.injected[s] += S.inj_n;
      if (mv > c->moves.maxmove[s]) c->moves.maxmove[s] = mv;
      if (st[0] > 0 || st[3] > 0 || S.inj_n > 0) {
        // far movers, losses or injected particles: rebuild the cell order
        const int64_t n_new = S.nbuf - st[3] + S.inj_n;
        int rc = ge_launch_far_resort(c, s, st[0]);
        if (rc) return rc;
        S.n = S.nbuf = n_new;
        S.inj_n = 0;
        c->moves.resorts += 1;
      }
      if (st[2] > 0)
        stuck += " species " + std::to_string(s) + ": " + std::to_string(st[2]) + " particle(s), largest accepted move " +
                 std::to_string(mv) + " cells;";
    }
  }
  if (h[GE_FL_RUNS]) return ge_fail(c, GE_ERR_STATE, "internal: particle run bookkeeping mismatch in the push");
  if (h[GE_FL_LOAD])
    return ge_fail(c, GE_ERR_ARG, "particles not sorted by cell or cell index out of range (pending injections dropped)");
  if (h[GE_FL_NONFINITE])
    return ge_fail(c, GE_ERR_NONFINITE, "a pushed particle had a non-finite velocity or position and was kept in place:" + stuck);
  if (h[GE_FL_CFL])
    return ge_fail(c, GE_ERR_CFL, "a particle would have moved more than n - 2 cells along an axis of n cells in one "
                                  "step and was kept in place:" + stuck);
  return GE_OK;
}

// Settle a pending push (its far movers) before particles are read again.
int settle(ge_ctx* c) { return (c->push_pending || c->inject_pending) ? check_flags(c) : GE_OK; }

// add the elapsed time of the event pairs of the last step (stream idle)
void accumulate_timings(ge_ctx* c, double solve_s) {
  float ms;
  for (int k = 0; k < 5; ++k)
    if (hipEventElapsedTime(&ms, c->ev[2 * k], c->ev[2 * k + 1]) == hipSuccess) c->tsum[k] += ms * 1e-3;
  if (hipEventElapsedTime(&ms, c->ev[0], c->ev[10]) == hipSuccess) c->tsum[6] += ms * 1e-3;
  (void)hipGetLastError();
  c->tsum[5] += solve_s;
  c->tcnt += 1;
}

// ------------------------------------------------------------ checkpoint file
// Little-endian binary: magic, version, then the sections in the order of
// ge_checkpoint; a 64-bit FNV-1a checksum of every byte before it closes the
// file.
const char GE_CKPT_MAGIC[8] = {'G', 'E', 'C', 'K', 'P', 'T', '0', '1'};
constexpr uint32_t GE_CKPT_VERSION = 1;

struct CkptWriter {
  FILE* f = nullptr;
  uint64_t h = 1469598103934665603ull;
  bool ok = true;
  void put(const void* p, size_t n) {
    const unsigned char* b = (const unsigned char*)p;
    for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 1099511628211ull;
    if (ok && n && fwrite(p, 1, n, f) != n) ok = false;
  }
  template <typename T>
  void val(const T& v) { put(&v, sizeof(T)); }
};
struct CkptReader {
  FILE* f = nullptr;
  uint64_t h = 1469598103934665603ull;
  bool ok = true;
  void get(void* p, size_t n) {
    if (!ok) return;
    if (n && fread(p, 1, n, f) != n) { ok = false; return; }
    const unsigned char* b = (const unsigned char*)p;
    for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 1099511628211ull;
  }
  template <typename T>
  T val() { T v{}; get(&v, sizeof(T)); return v; }
};

// Device staging of one species' particles as four arrays (cell int32[n],
// off T[3n], v T[3n], w T[n]), each starting on a 256-byte boundary; the
// checkpoint file holds the same arrays back to back.
struct PartStage {
  size_t seg[4], at[4], bytes;
};
PartStage part_stage(int64_t n, size_t es) {
  PartStage P;
  P.seg[0] = 4 * (size_t)n;
  P.seg[1] = 3 * es * (size_t)n;
  P.seg[2] = 3 * es * (size_t)n;
  P.seg[3] = es * (size_t)n;
  size_t o = 0;
  for (int k = 0; k < 4; ++k) {
    P.at[k] = o;
    o += (P.seg[k] + 255) / 256 * 256;
  }
  P.bytes = o ? o : 256;
  return P;
}

// the grid and parameters written field by field (no struct padding)
void put_config(CkptWriter& W, const ge_grid& g, const ge_params& P) {
  W.val(g.dim);
  for (int d = 0; d < 3; ++d) W.val(g.n[d]);
  for (int d = 0; d < 3; ++d) W.val(g.dx[d]);
  W.val(P.theta); W.val(P.c); W.val(P.dt); W.val(P.lf_E); W.val(P.lf_B); W.val(P.beta_lim); W.val(P.a_mode);
  W.val(P.a_const); W.val(P.comoving); W.val(P.n_smooth_u); W.val(P.phi_u); W.val(P.precision); W.val(P.ns_j);
  W.val(P.dedner); W.val(P.ch_frac); W.val(P.dedner_damp); W.val(P.ns_e); W.val(P.limiter_lag);
}
bool same_config(CkptReader& R, const ge_grid& g, const ge_params& P) {
  bool same = R.val<int>() == g.dim;
  for (int d = 0; d < 3; ++d) same = (R.val<int>() == g.n[d]) && same;
  for (int d = 0; d < 3; ++d) same = (R.val<double>() == g.dx[d]) && same;
  same = (R.val<double>() == P.theta) && same;
  same = (R.val<double>() == P.c) && same;
  same = (R.val<double>() == P.dt) && same;
  same = (R.val<int>() == P.lf_E) && same;
  same = (R.val<int>() == P.lf_B) && same;
  same = (R.val<double>() == P.beta_lim) && same;
  same = (R.val<int>() == P.a_mode) && same;
  same = (R.val<double>() == P.a_const) && same;
  same = (R.val<int>() == P.comoving) && same;
  same = (R.val<int>() == P.n_smooth_u) && same;
  same = (R.val<double>() == P.phi_u) && same;
  same = (R.val<int>() == P.precision) && same;
  same = (R.val<int>() == P.ns_j) && same;
  same = (R.val<int>() == P.dedner) && same;
  same = (R.val<double>() == P.ch_frac) && same;
  same = (R.val<double>() == P.dedner_damp) && same;
  same = (R.val<int>() == P.ns_e) && same;
  same = (R.val<int>() == P.limiter_lag) && same;
  return same;
}

}  // namespace

extern "C" {

// reason of the calling thread's last refused ge_create
thread_local std::string g_create_err = "no refused ge_create";

const char* ge_last_error(const ge_ctx* ctx) { return ctx ? ctx->err.c_str() : g_create_err.c_str(); }

int ge_half_stencil(const ge_ctx* ctx) { return ctx ? ctx->nh : 0; }

int ge_create(const ge_grid* grid, const ge_params* params, void* hip_stream, ge_ctx** out) {
  if (!grid || !params || !out) {
    g_create_err = "ge_create: null grid, params or out";
    return GE_ERR_ARG;
  }
  *out = nullptr;
  ge_ctx* c = new ge_ctx();
  std::memset((void*)&c->G, 0, sizeof(c->G));
  c->grid = *grid;
  c->P = *params;
  c->stream = (hipStream_t)hip_stream;
  const int dim = grid->dim;
  auto bad = [&](const std::string& m) {
    // the caller gets no context on failure: the reason is kept per thread
    // for ge_last_error(NULL)
    delete c;
    g_create_err = "ge_create: " + m;
    return GE_ERR_ARG;
  };
  if (dim < 1 || dim > 3) return bad("dim");
  for (int d = 0; d < 3; ++d) {
    const bool xs = d == 0 && grid->bc_lo[0] == GE_BC_WALL &&
                    (grid->bc_hi[0] == GE_BC_WALL || grid->bc_hi[0] == GE_BC_INFLOW);
    if (!xs && (grid->bc_lo[d] != GE_BC_PERIODIC || grid->bc_hi[d] != GE_BC_PERIODIC))
      return bad("boundaries: every axis periodic, or x with a wall at x = 0 and a wall or an inflow plane at x = L");
  }
  const bool wall = grid->bc_lo[0] == GE_BC_WALL;
  if (wall && (params->dedner || params->ns_e))
    return bad("divergence cleaning and E smoothing need periodic axes");
  int64_t N = 1;
  for (int d = 0; d < 3; ++d) {
    if (d < dim) {
      if (grid->n[d] < 3 || !(grid->dx[d] > 0)) return bad("n/dx");
      N *= grid->n[d] + (d == 0 && wall ? 1 : 0);
    } else if (grid->n[d] != 1) {
      return bad("inactive axes need n = 1");
    }
  }
  if (N >= (int64_t)1 << 31) return bad("grid too large");
  if (!(params->theta >= 0.5 && params->theta <= 1.0) || !(params->dt > 0) || !(params->c > 0)) return bad("theta/dt/c");
  if (params->precision != GE_FP64 && params->precision != GE_FP32) return bad("precision");
  if (params->n_smooth_u < 0 || params->beta_lim < 0) return bad("n_smooth_u/beta_lim");
  if (params->ns_j < 0 || !(params->ch_frac >= 0) || !(params->dedner_damp >= 0)) return bad("ns_j/ch_frac/dedner_damp");
  if (params->ns_e < 0) return bad("ns_e");
  if (params->limiter_lag != GE_LAG_EN && params->limiter_lag != GE_PICARD1) return bad("limiter_lag");
  DGrid& G = c->G;
  G.dim = dim;
  G.N = N;
  G.dV = 1.0;
  for (int d = 0; d < 3; ++d) {
    G.n[d] = d < dim ? grid->n[d] : 1;
    G.dx[d] = d < dim ? grid->dx[d] : 1.0;
    G.idx[d] = 1.0 / G.dx[d];
    if (d < dim) G.dV *= G.dx[d];
  }
  G.bcl = grid->bc_lo[0];
  G.bch = wall ? grid->bc_hi[0] : GE_BC_PERIODIC;
  G.nxp = grid->n[0];
  if (wall) G.n[0] += 1;  // the ghost cell column
  grid_div_magic(G);
  G.colsh = visit_colsh(G);
  c->nsp = 0;
  c->nh = half_count(dim);
  c->ND = dim == 3 ? 27 : (dim == 2 ? 9 : 3);
  c->NC = 1 << dim;
  c->NR = c->ND;
  c->Q = (18 * c->NR + c->NC * (7 + GE_MAX_SPECIES) + 3) / 4 * 4;  // a multiple of 4 (cq_index)
  c->kr_m = 64;
  {
    int dev = 0;
    c->n_cu = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
      int n = 0;
      if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0) c->n_cu = n;
    }
    (void)hipGetLastError();
  }
  const size_t es = params->precision == GE_FP32 ? 4 : 8;
  int rc = GE_OK;
  double** f3[] = {&c->E, &c->B, &c->Eth, &c->Bn, &c->Jlab, &c->Jeff, &c->mm, &c->u, &c->utmp, &c->EM, &c->rhs, &c->Bnew,
                   &c->ccell, &c->kw, &c->kr, &c->kx, &c->Zp};
  for (auto p : f3)
    if (!rc) rc = dalloc(c, p, sizeof(double) * 3 * N);
  if (!rc) rc = dalloc(c, &c->rho, sizeof(double) * GE_MAX_SPECIES * N);
  if (!rc) rc = dalloc(c, &c->mass, sizeof(double) * N);
  if (!rc) rc = dalloc(c, &c->anode, sizeof(double) * N);
  if (!rc) rc = dalloc(c, &c->psi, sizeof(double) * N);
  if (!rc) rc = dalloc(c, &c->kE, sizeof(double) * 9 * N);
  if (!rc) rc = dalloc(c, &c->kB, sizeof(double) * 9 * N);
  if (!rc && c->P.precision == GE_FP32) rc = dalloc(c, &c->kEf, sizeof(float) * 9 * N);
  if (!rc) rc = dalloc(c, &c->jac, sizeof(double) * 9 * N);
  if (!rc) rc = dalloc(c, &c->node8, es * 8 * N);
  if (!rc) rc = dalloc(c, &c->Mt, es * c->nh * 9 * N);
  if (!rc) rc = dalloc(c, &c->M0, es * c->nh * 9 * N);
  if (!rc) rc = dalloc(c, &c->cellQ, es * (size_t)c->Q * ((N + GE_CQG - 1) / GE_CQG * GE_CQG));
  if (!rc) rc = dalloc(c, &c->seg_next, sizeof(int32_t) * GE_MAX_SPECIES * N);
  c->scan_nblocks = (N + 1023) / 1024;
  if (!rc) rc = dalloc(c, &c->scan_blocks, sizeof(int32_t) * (c->scan_nblocks + 1));
  if (!rc) rc = dalloc(c, &c->V, sizeof(double) * 3 * N * (c->kr_m + 1));
  if (!rc) rc = dalloc(c, &c->hdev, sizeof(double) * 1024);
  if (!rc && hipHostMalloc((void**)&c->hhost, sizeof(double) * 1024, hipHostMallocDefault) != hipSuccess) {
    c->hhost = nullptr;
    (void)hipGetLastError();
    rc = ge_fail(c, GE_ERR_OOM, "pinned host buffer allocation failed");
  }
  if (!rc) rc = dalloc(c, &c->partials, sizeof(double) * 32 * 512);  // up to 32 dots x 512 blocks
  if (!rc) rc = dalloc(c, &c->flags, sizeof(int) * GE_FL_COUNT);
  if (!rc) rc = ge_noalloc_setup(c);
  if (rc) {
    g_create_err = "ge_create: " + c->err;
    ge_destroy(c);
    return rc;
  }
  hipStream_t s = c->stream;
  (void)hipMemsetAsync(c->E, 0, sizeof(double) * 3 * N, s);
  (void)hipMemsetAsync(c->B, 0, sizeof(double) * 3 * N, s);
  (void)hipMemsetAsync(c->kE, 0, sizeof(double) * 9 * N, s);
  (void)hipMemsetAsync(c->kB, 0, sizeof(double) * 9 * N, s);
  if (c->kEf) (void)hipMemsetAsync(c->kEf, 0, sizeof(float) * 9 * N, s);
  (void)hipMemsetAsync(c->rho, 0, sizeof(double) * GE_MAX_SPECIES * N, s);
  (void)hipMemsetAsync(c->psi, 0, sizeof(double) * N, s);
  (void)hipMemsetAsync(c->flags, 0, sizeof(int) * GE_FL_COUNT, s);
  for (int k = 0; k < 11; ++k) (void)hipEventCreate(&c->ev[k]);
  for (int k = 0; k < 8; ++k) c->tsum[k] = 0;
  c->tcnt = 0;
  if (hipGetLastError() != hipSuccess) {
    g_create_err = "ge_create: a HIP call failed while clearing the fields";
    ge_destroy(c);
    return GE_ERR_HIP;
  }
  *out = c;
  return GE_OK;
}

void ge_destroy(ge_ctx* c) {
  if (!c) return;
  if (c->stream || true) (void)hipStreamSynchronize(c->stream);
  double** f[] = {&c->E, &c->B, &c->Eth, &c->Bn, &c->Jlab, &c->Jeff, &c->rho, &c->mm, &c->mass, &c->u, &c->utmp,
                  &c->EM, &c->anode, &c->psi, &c->kE, &c->kB, &c->rhs, &c->Bnew, &c->ccell, &c->jac, &c->V, &c->Zp,
                  &c->kw, &c->kr, &c->kx, &c->hdev, &c->partials, &c->scal};
  for (auto p : f) dfree(*p);
  if (c->hhost) (void)hipHostFree(c->hhost);
  dfree(c->node8);
  dfree(c->kEf);
  dfree(c->Mt);
  dfree(c->M0);
  dfree(c->cellQ);
  dfree(c->seg_next);
  dfree(c->scan_blocks);
  dfree(c->flags);
  for (int s = 0; s < c->nsp; ++s) {
    for (int b = 0; b < 2; ++b) {
      dfree(c->sp[s].rec[b]);
      dfree(c->sp[s].runs[b]);
    }
    dfree(c->sp[s].far);
    dfree(c->sp[s].inj_cell);
  }
  ge_far_free(c);
  for (int k = 0; k < 11; ++k)
    if (c->ev[k]) (void)hipEventDestroy(c->ev[k]);
  ge_cnn_free(c);
  dfree(c->Zb);
  dfree(c->Ub);
  delete c;
}

int ge_add_species(ge_ctx* c, const ge_species* sp, int64_t n, const int32_t* cell, const void* off, const void* v,
                   const void* w) {
  if (!c || !sp) return GE_ERR_ARG;
  if (c->nsp >= GE_MAX_SPECIES) return ge_fail(c, GE_ERR_ARG, "at most 4 species");
  if (c->have_deposit) return ge_fail(c, GE_ERR_STATE, "species must be added before the first deposit");
  if (n < 0 || n >= ((int64_t)1 << 31)) return ge_fail(c, GE_ERR_ARG, "particle count out of range (< 2^31)");
  if (n > 0 && (!cell || !off || !v || !w)) return ge_fail(c, GE_ERR_ARG, "null particle array");
  if (!(sp->m > 0)) return ge_fail(c, GE_ERR_ARG, "species mass must be positive");
  const int s = c->nsp;
  SpeciesBuf& S = c->sp[s];
  std::memset((void*)&S, 0, sizeof(S));
  S.q = sp->q;
  S.m = sp->m;
  S.beta = sp->q * c->P.dt / (2.0 * sp->m);
  S.n = n;
  S.nbuf = n;
  S.cap = n > 0 ? n : 1;
  const size_t es = c->P.precision == GE_FP32 ? 4 : 8;
  int rc = GE_OK;
  for (int b = 0; b < 2 && !rc; ++b) {
    rc = dalloc(c, &S.rec[b], es * GE_REC * (n > 0 ? n : 1));  // a valid record 0 even when empty
    if (!rc) rc = dalloc(c, &S.runs[b], sizeof(int32_t) * 2 * c->ND * c->G.N);
  }
  if (!rc) rc = dalloc(c, &S.far, sizeof(int32_t) * 4 * c->G.N);
  c->nsp = s + 1;  // so that ge_destroy frees partial allocations
  if (rc) {
    for (int b = 0; b < 2; ++b) {
      dfree(S.rec[b]); dfree(S.runs[b]);
    }
    dfree(S.far);
    c->nsp = s;
    return rc;
  }
  GE_HIP(c, hipMemsetAsync(S.far, 0, sizeof(int32_t) * 4 * c->G.N, c->stream));
  rc = ge_launch_load_species(c, s, cell, off, v, w);
  if (rc) return rc;
  rc = check_flags(c);
  if (rc) {
    for (int b = 0; b < 2; ++b) {
      dfree(S.rec[b]); dfree(S.runs[b]);
    }
    dfree(S.far);
    c->nsp = s;
    return rc;
  }
  return GE_OK;
}

int ge_set_fields(ge_ctx* c, const double* E, const double* B) {
  if (!c || !E || !B) return GE_ERR_ARG;
  const size_t bytes = sizeof(double) * 3 * c->G.N;
  GE_HIP(c, hipMemcpyAsync(c->E, E, bytes, hipMemcpyDeviceToDevice, c->stream));
  GE_HIP(c, hipMemcpyAsync(c->B, B, bytes, hipMemcpyDeviceToDevice, c->stream));
  return GE_OK;
}

int ge_deposit(ge_ctx* c) {
  if (!c) return GE_ERR_ARG;
  if (c->nsp == 0) return ge_fail(c, GE_ERR_STATE, "no species");
  int rc = settle(c);
  if (rc) return rc;
  if ((rc = ge_launch_node_avg(c))) return rc;
  (void)hipEventRecord(c->ev[2], c->stream);
  if ((rc = ge_launch_deposit(c))) return rc;
  (void)hipEventRecord(c->ev[3], c->stream);
  c->have_deposit = 1;
  if ((rc = ge_launch_grid_pass(c))) return rc;
  c->have_solve = 0;
  return GE_OK;
}

int ge_explicit_current(ge_ctx* c, double* J) {
  if (!c) return GE_ERR_ARG;
  if (c->nsp == 0) return ge_fail(c, GE_ERR_STATE, "no species");
  if (walled(c->G)) return ge_fail(c, GE_ERR_ARG, "the explicit-PIC path needs periodic axes");
  int rc = settle(c);
  if (rc) return rc;
  // moments -> smoothed bulk velocity -> current, then the ns_j passes
  if ((rc = ge_launch_explicit_linear(c, 0))) return rc;
  if ((rc = ge_launch_bulk_velocity(c))) return rc;
  if ((rc = ge_launch_explicit_linear(c, c->P.comoving ? 1 : 2))) return rc;
  if ((rc = ge_launch_smooth_current(c))) return rc;
  c->have_deposit = 0;
  c->have_solve = 0;
  if (J) GE_HIP(c, hipMemcpyAsync(J, c->Jeff, sizeof(double) * 3 * c->G.N, hipMemcpyDeviceToDevice, c->stream));
  return GE_OK;
}

int ge_explicit_step(ge_ctx* c) {
  if (!c) return GE_ERR_ARG;
  if (c->nsp == 0) return ge_fail(c, GE_ERR_STATE, "no species");
  if (walled(c->G)) return ge_fail(c, GE_ERR_ARG, "the explicit-PIC path needs periodic axes");
  int rc = settle(c);
  if (rc) return rc;
  // corner fields of the push: E^n (through c->Eth) and the node average of B^n
  GE_HIP(c, hipMemcpyAsync(c->Eth, c->E, sizeof(double) * 3 * c->G.N, hipMemcpyDeviceToDevice, c->stream));
  if ((rc = ge_launch_node_avg(c))) return rc;
  if ((rc = ge_launch_pack_node8(c, 0))) return rc;
  for (int s = 0; s < c->nsp; ++s)
    if ((rc = ge_launch_scan_counts(c, s))) return rc;
  for (int s = 0; s < c->nsp; ++s)
    if ((rc = ge_launch_push(c, s))) return rc;
  // far movers are re-sorted before the current passes read the cells
  c->push_pending = 1;
  if ((rc = check_flags(c))) return rc;
  // the current at (x^{n+1}, v^{n+1/2}), then the leapfrog
  if ((rc = ge_launch_explicit_linear(c, 0))) return rc;
  if ((rc = ge_launch_bulk_velocity(c))) return rc;
  if ((rc = ge_launch_explicit_linear(c, c->P.comoving ? 1 : 2))) return rc;
  if ((rc = ge_launch_smooth_current(c))) return rc;
  if ((rc = ge_launch_explicit_fields(c))) return rc;
  c->have_deposit = 0;
  c->have_solve = 0;
  c->steps += 1;
  return check_flags(c);
}

int ge_solve_fields(ge_ctx* c, double tol, int maxit, int restart, int precond, ge_solve_report* rep) {
  if (!c) return GE_ERR_ARG;
  if (!c->have_deposit) return ge_fail(c, GE_ERR_STATE, "ge_solve_fields before ge_deposit");
  if (!(tol > 0) || maxit < 1) return ge_fail(c, GE_ERR_ARG, "tol/maxit");
  GE_HIP(c, hipMemcpyAsync(c->Eth, c->E, sizeof(double) * 3 * c->G.N, hipMemcpyDeviceToDevice, c->stream));
  ge_solve_report r;
  std::memset(&r, 0, sizeof(r));
  int rc = ge_gmres(c, tol, maxit, restart, precond, &r);
  if (rc >= 0 && c->P.limiter_lag == GE_PICARD1 && c->P.lf_E) {
    // one Picard step of the limiter: coefficients from the first E^{n+theta},
    // then the system again, starting from that solution
    ge_solve_report r2;
    std::memset(&r2, 0, sizeof(r2));
    int kr = ge_launch_kappa_E(c, c->Eth);
    if (kr) return kr;
    rc = ge_gmres(c, tol, maxit, restart, precond, &r2);
    r2.iterations += r.iterations;
    r2.restarts += r.restarts;
    r2.seconds += r.seconds;
    r2.fallback |= r.fallback;
    r = r2;
  }
  if (rep) *rep = r;
  if (rc < 0) return rc;
  c->have_solve = 1;
  // training data for the learned preconditioner
  const int hv = (rc == GE_OK && precond != GE_PC_CNN) ? ge_cnn_harvesting(c) : 0;
  if (hv & GE_HARVEST_SOLUTION) {
    // (r0 = b - A E^n, e = E^{n+theta} - E^n)
    const int64_t n3 = 3 * c->G.N;
    int hr = ge_launch_apply_A(c, c->E, c->kw);
    if (!hr) hr = ge_launch_sub(c, c->rhs, c->kw, c->kw, n3);
    if (!hr) hr = ge_launch_sub(c, c->Eth, c->E, c->kx, n3);
    if (!hr) hr = ge_cnn_add_pair(c, c->kw, c->kx);
    if (hr) return hr;
  }
  if (hv & GE_HARVEST_KRYLOV) {
    // (A v_j, v_j) for the unit Arnoldi vectors of the last cycle (v_0 holds
    // the final residual by now and is skipped)
    for (int j = 1; j < c->kr_last; ++j) {
      const double* vj = c->V + (int64_t)j * 3 * c->G.N;
      int hr = ge_launch_apply_A(c, vj, c->kw);
      if (!hr) hr = ge_cnn_add_pair(c, c->kw, vj);
      if (hr) return hr;
    }
  }
  int fr = check_flags(c);
  return fr ? fr : rc;
}

int ge_push(ge_ctx* c) {
  if (!c) return GE_ERR_ARG;
  if (!c->have_solve) return ge_fail(c, GE_ERR_STATE, "ge_push needs E^{n+theta} (solve or ge_set GE_F_ETH)");
  int rc = settle(c);
  if (rc) return rc;
  // timed phase [0]: packing of the corner fields, the segment scans and the pushes
  (void)hipEventRecord(c->ev[0], c->stream);
  if ((rc = ge_launch_pack_node8(c, 0))) return rc;
  for (int s = 0; s < c->nsp; ++s)
    if ((rc = ge_launch_scan_counts(c, s))) return rc;
  (void)hipEventRecord(c->ev[10], c->stream);
  for (int s = 0; s < c->nsp; ++s)
    if ((rc = ge_launch_push(c, s))) return rc;
  (void)hipEventRecord(c->ev[1], c->stream);
  c->push_pending = 1;
  return GE_OK;
}

int ge_update_fields(ge_ctx* c) {
  if (!c) return GE_ERR_ARG;
  if (!c->have_solve) return ge_fail(c, GE_ERR_STATE, "ge_update_fields needs a solve");
  int rc = ge_launch_update(c);
  if (rc) return rc;
  c->have_solve = 0;
  c->have_deposit = 0;
  c->steps += 1;
  return GE_OK;
}

int ge_step(ge_ctx* c, double tol, int maxit, int restart, int precond, ge_solve_report* rep) {
  int rc = ge_deposit(c);
  if (rc) return rc;
  ge_solve_report r;
  std::memset(&r, 0, sizeof(r));
  int sr = ge_solve_fields(c, tol, maxit, restart, precond, &r);
  if (sr < 0) return sr;
  if (rep) *rep = r;
  if ((rc = ge_push(c))) return rc;
  if ((rc = ge_update_fields(c))) return rc;
  rc = check_flags(c);
  if (!rc) accumulate_timings(c, r.seconds);
  return rc ? rc : sr;
}

int ge_sync(ge_ctx* c) {
  if (!c) return GE_ERR_ARG;
  return check_flags(c);
}

int ge_gather(ge_ctx* c, int what, double* dst) {
  if (!c || !dst) return GE_ERR_ARG;
  const int64_t N = c->G.N;
  const double* src = nullptr;
  int64_t cnt = 3 * N;
  switch (what) {
    case GE_F_E: src = c->E; break;
    case GE_F_B: src = c->B; break;
    case GE_F_ETH: src = c->Eth; break;
    case GE_F_BN: src = c->Bn; break;
    case GE_F_J_LAB: src = c->Jlab; break;
    case GE_F_J_EFF: src = c->Jeff; break;
    case GE_F_RHO: src = c->rho; cnt = (int64_t)c->nsp * N; break;
    case GE_F_MM: src = c->mm; break;
    case GE_F_MASS: src = c->mass; cnt = N; break;
    case GE_F_U: src = c->u; break;
    case GE_F_EM: src = c->EM; break;
    case GE_F_MTILDE: return ge_launch_widen_M(c, c->Mt, dst);
    case GE_F_M0: return ge_launch_widen_M(c, c->M0, dst);
    case GE_F_KAPPA_E: src = c->kE; cnt = 9 * N; break;
    case GE_F_KAPPA_B: src = c->kB; cnt = 9 * N; break;
    case GE_F_RHS: src = c->rhs; break;
    case GE_F_PSI: src = c->psi; cnt = N; break;
    default: return ge_fail(c, GE_ERR_ARG, "unknown field id");
  }
  GE_HIP(c, hipMemcpyAsync(dst, src, sizeof(double) * cnt, hipMemcpyDeviceToDevice, c->stream));
  return GE_OK;
}

int ge_set(ge_ctx* c, int what, const double* src) {
  if (!c || !src) return GE_ERR_ARG;
  const int64_t N = c->G.N;
  double* dst = nullptr;
  switch (what) {
    case GE_F_E: dst = c->E; break;
    case GE_F_B: dst = c->B; break;
    case GE_F_ETH: dst = c->Eth; break;
    case GE_F_BN: dst = c->Bn; break;
    case GE_F_RHS: dst = c->rhs; break;
    case GE_F_PSI: dst = c->psi; break;
    default: return ge_fail(c, GE_ERR_ARG, "field id cannot be set");
  }
  GE_HIP(c, hipMemcpyAsync(dst, src, sizeof(double) * (what == GE_F_PSI ? 1 : 3) * N, hipMemcpyDeviceToDevice,
                           c->stream));
  if (what == GE_F_ETH) c->have_solve = 1;
  if (what == GE_F_BN) return ge_launch_pack_node8(c, 1);
  return GE_OK;
}

int ge_get_particles(ge_ctx* c, int s, int64_t n, int32_t* cell, void* off, void* v, void* w) {
  if (!c || s < 0 || s >= c->nsp) return GE_ERR_ARG;
  if (n != c->sp[s].n) return ge_fail(c, GE_ERR_ARG, "particle count mismatch");
  int rc = settle(c);
  if (rc) return rc;
  if (n == 0) return GE_OK;  // an empty species: nothing to copy, the pointers may be null
  if (!cell || !off || !v || !w) return ge_fail(c, GE_ERR_ARG, "null output");
  return ge_launch_get_particles(c, s, cell, off, v, w);
}

int ge_apply_operator(ge_ctx* c, const double* x, double* y) {
  if (!c || !x || !y) return GE_ERR_ARG;
  return ge_launch_apply_A(c, x, y);
}

int ge_diagnostics(ge_ctx* c, ge_diag* out) {
  if (!c || !out) return GE_ERR_ARG;
  std::memset(out, 0, sizeof(*out));
  out->nsp = c->nsp;
  double f[4];
  int rc = settle(c);
  if (rc) return rc;
  rc = ge_launch_field_diag(c, f);
  if (rc) return rc;
  const double k8 = c->G.dV / (8.0 * M_PI);
  out->W_E = f[0] * k8;
  out->W_B = f[1] * k8;
  out->gauss = f[3] > 0 ? std::sqrt(f[2] / f[3]) : std::sqrt(f[2]);
  for (int s = 0; s < c->nsp; ++s) {
    double m4[4];
    if ((rc = ge_launch_particle_moments(c, s, m4))) return rc;
    out->K[s] = 0.5 * c->sp[s].m * m4[0];
    for (int d = 0; d < 3; ++d) out->P[s][d] = c->sp[s].m * m4[1 + d];
  }
  return check_flags(c);
}

int ge_inject(ge_ctx* c, int s, int64_t m, const int32_t* cell, const void* off, const void* v, const void* w) {
  if (!c || s < 0 || s >= c->nsp) return GE_ERR_ARG;
  if (m < 0) return ge_fail(c, GE_ERR_ARG, "negative particle count");
  if (m == 0) return GE_OK;
  if (!cell || !off || !v || !w) return ge_fail(c, GE_ERR_ARG, "null particle array");
  if (c->have_deposit || c->have_solve)
    return ge_fail(c, GE_ERR_STATE, "ge_inject between a deposit and its field update");
  SpeciesBuf& S = c->sp[s];
  if (S.nbuf + S.inj_n + m >= ((int64_t)1 << 31)) return ge_fail(c, GE_ERR_ARG, "species would exceed 2^31 particles");
  int rc = ge_launch_inject_pack(c, s, m, cell, off, v, w);
  if (rc) return rc;
  c->inject_pending = 1;
  return GE_OK;
}

int64_t ge_step_count(const ge_ctx* c) { return c ? c->steps : -1; }

int64_t ge_species_count(const ge_ctx* c, int s) { return (c && s >= 0 && s < c->nsp) ? c->sp[s].n : -1; }

int ge_checkpoint(ge_ctx* c, const char* path) {
  if (!c || !path) return GE_ERR_ARG;
  if (c->have_deposit || c->have_solve)
    return ge_fail(c, GE_ERR_STATE, "ge_checkpoint between a deposit and its field update");
  int rc = settle(c);
  if (rc) return rc;
  const int64_t N = c->G.N;
  const size_t es = c->P.precision == GE_FP32 ? 4 : 8;
  CkptWriter W;
  W.f = std::fopen(path, "wb");
  if (!W.f) return ge_fail(c, GE_ERR_ARG, std::string("cannot open ") + path + " for writing");
  W.put(GE_CKPT_MAGIC, 8);
  W.val(GE_CKPT_VERSION);
  put_config(W, c->grid, c->P);
  W.val(c->steps);
  W.val(c->nsp);
  for (int s = 0; s < c->nsp; ++s) {
    W.val(c->sp[s].q);
    W.val(c->sp[s].m);
    W.val(c->sp[s].n);
  }
  // fields
  std::vector<double> hf(3 * N);
  const double* fsrc[3] = {c->E, c->B, c->psi};
  const int64_t fcnt[3] = {3 * N, 3 * N, N};
  for (int k = 0; k < 3 && !rc; ++k) {
    if (hipMemcpyAsync(hf.data(), fsrc[k], sizeof(double) * fcnt[k], hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
      rc = ge_fail(c, GE_ERR_HIP, "checkpoint: field read-back failed");
    else
      W.put(hf.data(), sizeof(double) * fcnt[k]);
  }
  // particles in cell order, one species at a time (device staging, then host)
  for (int s = 0; s < c->nsp && !rc; ++s) {
    const int64_t n = c->sp[s].n;
    if (n == 0) continue;
    char* dbuf = nullptr;
    const PartStage PS = part_stage(n, es);
    if (hipMalloc((void**)&dbuf, PS.bytes) != hipSuccess) {
      (void)hipGetLastError();
      rc = ge_fail(c, GE_ERR_OOM, "checkpoint: particle staging allocation failed");
      break;
    }
    rc = ge_launch_get_particles(c, s, (int32_t*)(dbuf + PS.at[0]), dbuf + PS.at[1], dbuf + PS.at[2],
                                 dbuf + PS.at[3]);
    std::vector<char> hb(PS.seg[0] + PS.seg[1] + PS.seg[2] + PS.seg[3]);
    size_t o = 0;
    for (int k = 0; k < 4 && !rc; ++k) {
      if (hipMemcpyAsync(hb.data() + o, dbuf + PS.at[k], PS.seg[k], hipMemcpyDeviceToHost, c->stream) != hipSuccess)
        rc = ge_fail(c, GE_ERR_HIP, "checkpoint: particle read-back failed");
      o += PS.seg[k];
    }
    if (!rc && hipStreamSynchronize(c->stream) != hipSuccess)
      rc = ge_fail(c, GE_ERR_HIP, "checkpoint: particle read-back failed");
    (void)hipFree(dbuf);
    if (!rc) W.put(hb.data(), hb.size());
  }
  // learned preconditioner
  int has_cnn = c->cnn ? 1 : 0;
  std::vector<float> cw, cm, cv;
  int ct = 0, ccap = 0;
  if (!rc && has_cnn && ge_cnn_export(c, cw, cm, cv, ct, ccap) != GE_OK) has_cnn = 0;
  if (!rc) {
    W.val(has_cnn);
    if (has_cnn) {
      const int nw = (int)cw.size();
      W.val(nw);
      W.put(cw.data(), sizeof(float) * nw);
      W.put(cm.data(), sizeof(float) * nw);
      W.put(cv.data(), sizeof(float) * nw);
      W.val(ct);
      W.val(ccap);
    }
    const uint64_t sum = W.h;
    W.val(sum);
  }
  const bool ok = W.ok;
  if (std::fclose(W.f) != 0 && !rc) return ge_fail(c, GE_ERR_ARG, std::string("cannot write ") + path);
  if (!rc && !ok) return ge_fail(c, GE_ERR_ARG, std::string("cannot write ") + path);
  return rc;
}

int ge_restore(ge_ctx* c, const char* path) {
  if (!c || !path) return GE_ERR_ARG;
  if (c->nsp != 0) return ge_fail(c, GE_ERR_STATE, "ge_restore needs a context without species");
  CkptReader R;
  R.f = std::fopen(path, "rb");
  if (!R.f) return ge_fail(c, GE_ERR_ARG, std::string("cannot open ") + path);
  long fsize = -1;
  if (std::fseek(R.f, 0, SEEK_END) == 0) fsize = std::ftell(R.f);
  std::rewind(R.f);
  auto fail = [&](int code, const std::string& m) {
    std::fclose(R.f);
    return ge_fail(c, code, "ge_restore: " + m);
  };
  char magic[8];
  R.get(magic, 8);
  if (!R.ok || std::memcmp(magic, GE_CKPT_MAGIC, 8) != 0) return fail(GE_ERR_ARG, "not a checkpoint file");
  if (R.val<uint32_t>() != GE_CKPT_VERSION) return fail(GE_ERR_ARG, "unknown checkpoint version");
  if (!same_config(R, c->grid, c->P)) return fail(GE_ERR_ARG, "grid or parameters differ from the checkpoint's");
  const int64_t steps = R.val<int64_t>();
  const int nsp = R.val<int>();
  if (!R.ok || nsp < 0 || nsp > GE_MAX_SPECIES) return fail(GE_ERR_ARG, "truncated or corrupt header");
  double q[GE_MAX_SPECIES], m[GE_MAX_SPECIES];
  int64_t n[GE_MAX_SPECIES];
  for (int s = 0; s < nsp; ++s) {
    q[s] = R.val<double>();
    m[s] = R.val<double>();
    n[s] = R.val<int64_t>();
    if (!R.ok || n[s] < 0 || n[s] >= ((int64_t)1 << 31)) return fail(GE_ERR_ARG, "truncated or corrupt header");
  }
  const int64_t N = c->G.N;
  const size_t es = c->P.precision == GE_FP32 ? 4 : 8;
  {
    // the declared sizes must fit in the file before anything is allocated
    uint64_t need = sizeof(double) * 7 * (uint64_t)N;
    for (int s = 0; s < nsp; ++s) need += (uint64_t)n[s] * (4 + 7 * es);
    if (fsize < 0 || need > (uint64_t)fsize) return fail(GE_ERR_ARG, "truncated file");
  }
  std::vector<double> E(3 * N), B(3 * N), psi(N);
  R.get(E.data(), sizeof(double) * 3 * N);
  R.get(B.data(), sizeof(double) * 3 * N);
  R.get(psi.data(), sizeof(double) * N);
  std::vector<std::vector<char>> parts(nsp);
  for (int s = 0; s < nsp && R.ok; ++s) {
    parts[s].resize((size_t)n[s] * (4 + 7 * es));
    R.get(parts[s].data(), parts[s].size());
  }
  const int has_cnn = R.val<int>();
  std::vector<float> cw, cm, cv;
  int ct = 0, ccap = 0;
  if (R.ok && has_cnn) {
    const int nw = R.val<int>();
    if (!R.ok || nw != ge_cnn_size()) return fail(GE_ERR_ARG, "network size differs");
    cw.resize(nw); cm.resize(nw); cv.resize(nw);
    R.get(cw.data(), sizeof(float) * nw);
    R.get(cm.data(), sizeof(float) * nw);
    R.get(cv.data(), sizeof(float) * nw);
    ct = R.val<int>();
    ccap = R.val<int>();
  }
  const uint64_t want = R.h;
  const uint64_t sum = R.val<uint64_t>();
  if (!R.ok) return fail(GE_ERR_ARG, "truncated file");
  if (sum != want) return fail(GE_ERR_ARG, "checksum mismatch (corrupt file)");
  std::fclose(R.f);
  // species through the loading path (cell order is kept: the file holds them sorted)
  for (int s = 0; s < nsp; ++s) {
    char* dbuf = nullptr;
    const PartStage PS = part_stage(n[s], es);
    if (hipMalloc((void**)&dbuf, PS.bytes) != hipSuccess) {
      (void)hipGetLastError();
      return ge_fail(c, GE_ERR_OOM, "ge_restore: particle staging allocation failed");
    }
    int rc = GE_OK;
    size_t o = 0;
    for (int k = 0; k < 4 && !rc; ++k) {
      if (PS.seg[k] &&
          hipMemcpyAsync(dbuf + PS.at[k], parts[s].data() + o, PS.seg[k], hipMemcpyHostToDevice, c->stream) != hipSuccess)
        rc = ge_fail(c, GE_ERR_HIP, "ge_restore: particle upload failed");
      o += PS.seg[k];
    }
    if (!rc && hipStreamSynchronize(c->stream) != hipSuccess) rc = ge_fail(c, GE_ERR_HIP, "ge_restore: particle upload failed");
    ge_species sp{q[s], m[s]};
    if (!rc)
      rc = ge_add_species(c, &sp, n[s], (const int32_t*)(dbuf + PS.at[0]), dbuf + PS.at[1], dbuf + PS.at[2],
                          dbuf + PS.at[3]);
    (void)hipFree(dbuf);
    if (rc) return rc;
  }
  GE_HIP(c, hipMemcpyAsync(c->E, E.data(), sizeof(double) * 3 * N, hipMemcpyHostToDevice, c->stream));
  GE_HIP(c, hipMemcpyAsync(c->B, B.data(), sizeof(double) * 3 * N, hipMemcpyHostToDevice, c->stream));
  GE_HIP(c, hipMemcpyAsync(c->psi, psi.data(), sizeof(double) * N, hipMemcpyHostToDevice, c->stream));
  GE_HIP(c, hipStreamSynchronize(c->stream));
  if (has_cnn) {
    int rc = ge_cnn_import(c, cw.data(), cm.data(), cv.data(), ct, ccap);
    if (rc) return rc;
  }
  c->steps = steps;
  return GE_OK;
}

int ge_moves(ge_ctx* c, ge_move_report* out) {
  if (!c || !out) return GE_ERR_ARG;
  int rc = settle(c);
  std::memset(out, 0, sizeof(*out));
  for (int s = 0; s < c->nsp; ++s) {
    out->far_moves[s] = c->moves.far[s];
    out->max_move[s] = c->moves.maxmove[s];
    out->gone[s] = c->moves.gone[s];
    out->injected[s] = c->moves.injected[s];
  }
  out->resorts = c->moves.resorts;
  out->pushes = c->moves.pushes;
  std::memset(&c->moves, 0, sizeof(c->moves));
  return rc;
}

int ge_timings(ge_ctx* c, double* out8) {
  if (!c || !out8) return GE_ERR_ARG;
  for (int k = 0; k < 8; ++k) out8[k] = c->tcnt ? c->tsum[k] / c->tcnt : 0.0;
  out8[7] = c->tcnt;
  for (int k = 0; k < 8; ++k) c->tsum[k] = 0;
  c->tcnt = 0;
  return GE_OK;
}

}  // extern "C"
