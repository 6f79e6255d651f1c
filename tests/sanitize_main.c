/*
 * Memory and undefined-behaviour check of the CPU side: every routine of the
 * FP64 oracle and the input generator run on small periodic and walled grids
 * in one, two and three dimensions.  Built with gcc -fsanitize=address,undefined
 * by tests/test_sanitize.py; a sanitizer report aborts the run.  Not a parity
 * test: it only exercises the code paths.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../synth/gen.c"
#include "../oracle/glecsim_oracle.h"

static double* zeros(int64_t n) {
  double* p = (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
  if (!p) { fprintf(stderr, "out of memory\n"); exit(2); }
  return p;
}

/* one oracle step on a grid of nx[dim] physical cells; bc = 0 periodic, 1 wall/wall, 2 wall/inflow */
static int run_case(int dim, const int nx[3], int bc, int profile) {
  synth_cfg c;
  memset(&c, 0, sizeof(c));
  c.dim = dim;
  for (int d = 0; d < 3; ++d) { c.n[d] = d < dim ? nx[d] : 1; c.dx[d] = d < dim ? 0.5 : 1.0; }
  if (bc) c.n[0] += 1;  /* the ghost cell layer of a walled x axis */
  c.ppc = 5;
  c.nsp = 2;
  c.q[0] = -1.0; c.q[1] = 1.0;
  c.m[0] = 1.0; c.m[1] = 25.0;
  c.vth[0] = 0.05; c.vth[1] = 0.01;
  c.seed = 7u;
  c.profile = profile;
  c.n0 = 1.0 / (4.0 * M_PI);
  c.u0[0] = bc ? -0.15 : 0.05;
  c.B0[0] = 0.1; c.B0[1] = 0.05;
  c.lambda = 1.0; c.nb = 0.1; c.Bh = 0.5; c.psi = 0.01;
  c.dsheet[0] = -0.02; c.dsheet[1] = 0.1;
  c.ghost_x = bc ? 1 : 0;
  c.dt_inj = 0.5;

  or_grid G;
  memset(&G, 0, sizeof(G));
  G.dim = dim;
  for (int d = 0; d < 3; ++d) { G.n[d] = c.n[d]; G.dx[d] = c.dx[d]; }
  G.bc_lo = bc ? 1 : 0;
  G.bc_hi = bc;
  or_params P = {0.5, 1.0, 0.5};
  const int64_t N = or_nnodes(&G);
  if (N != synth_ncells(&c)) return 1;

  double *E = zeros(3 * N), *B = zeros(3 * N), *Bn = zeros(3 * N);
  synth_fields(&c, E, B);
  or_node_avg(&G, B, Bn);

  double *x[2], *v[2], *w[2];
  int64_t np[2];
  for (int s = 0; s < 2; ++s) {
    const int64_t cap = N * c.ppc;
    int32_t* cell = (int32_t*)calloc((size_t)cap, sizeof(int32_t));
    double *off = zeros(3 * cap), *vs = zeros(3 * cap), *ws = zeros(cap);
    np[s] = synth_particles(&c, s, 0, N, cell, off, vs, ws, 0);
    x[s] = zeros(3 * np[s]); v[s] = zeros(3 * np[s]); w[s] = zeros(np[s]);
    for (int64_t p = 0; p < np[s]; ++p) {
      int64_t rem = cell[p];
      for (int d = 0; d < 3; ++d) {
        const int64_t ic = d < dim ? rem % G.n[d] : 0;
        if (d < dim) rem /= G.n[d];
        x[s][3 * p + d] = d < dim ? ((double)ic + off[d * np[s] + p]) * G.dx[d] : 0.0;
        v[s][3 * p + d] = vs[d * np[s] + p];
      }
      w[s][p] = ws[p];
    }
    free(cell); free(off); free(vs); free(ws);
    /* injected particles of a walled grid (their buffers sized by a first call) */
    const int64_t need = synth_inflow(&c, s, 3, 0, NULL, NULL, NULL, NULL, 0);
    if (need > 0) {
      int32_t* ic = (int32_t*)calloc((size_t)need, sizeof(int32_t));
      double *io = zeros(3 * need), *iv = zeros(3 * need), *iw = zeros(need);
      if (synth_inflow(&c, s, 3, need, ic, io, iv, iw, 0) != need) return 2;
      free(ic); free(io); free(iv); free(iw);
    }
  }

  const int64_t NM = 27 * 9 * N;
  double *J = zeros(3 * N), *JC = zeros(3 * N), *rho = zeros(N), *mm = zeros(3 * N), *mass = zeros(N);
  double *Ms[2] = {zeros(NM), zeros(NM)}, *Mt = zeros(NM);
  const double beta[2] = {c.q[0] * P.dt / (2.0 * c.m[0]), c.q[1] * P.dt / (2.0 * c.m[1])};
  for (int s = 0; s < 2; ++s)
    or_deposit_species(&G, c.q[s], c.m[s], beta[s], np[s], x[s], v[s], w[s], Bn, NULL, J, Ms[s], rho, mm, mass);
  for (int64_t i = 0; i < NM; ++i) Mt[i] = beta[0] * Ms[0][i] + beta[1] * Ms[1][i];
  double *u = zeros(3 * N), *EM = zeros(3 * N), *a = zeros(N);
  or_bulk_velocity(&G, mm, mass, u);
  or_smooth(&G, u, 3, 5, 0.5);
  or_motional(&G, u, Bn, EM);
  {
    double *r2 = zeros(N), *m2 = zeros(3 * N), *ms2 = zeros(N), *Mtmp = zeros(NM);
    for (int s = 0; s < 2; ++s)
      or_deposit_species(&G, c.q[s], c.m[s], beta[s], np[s], x[s], v[s], w[s], Bn, u, JC, Mtmp, r2, m2, ms2);
    free(r2); free(m2); free(ms2); free(Mtmp);
  }
  double* Jeff = zeros(3 * N);
  or_current_eff(&G, JC, Mt, EM, Jeff);
  for (int64_t g = 0; g < N; ++g) a[g] = sqrt(u[g] * u[g] + u[N + g] * u[N + g] + u[2 * N + g] * u[2 * N + g]);
  double *kE = zeros(9 * N), *kB = zeros(9 * N), *b = zeros(3 * N), *Eth = zeros(3 * N), *y = zeros(3 * N);
  or_kappa_E(&G, E, a, 1.0, kE);
  or_kappa_B(&G, B, a, 1.0, kB);
  or_rhs(&G, &P, E, B, Jeff, b);
  memcpy(Eth, E, sizeof(double) * 3 * N);
  double relres = 0.0;
  const int it = or_gmres(&G, &P, Mt, kE, b, Eth, 1e-10, 300, 30, &relres);
  if (it < 0 || !(relres < 1e-8)) return 3;
  or_apply_A(&G, &P, Mt, kE, Eth, y);
  double *Bnew = zeros(3 * N), *Enew = zeros(3 * N), *div = zeros(N), *cn = zeros(3 * N), *cc = zeros(3 * N);
  double *Dy = zeros(3 * N), *My = zeros(3 * N);
  or_update_B(&G, &P, B, Eth, kB, Bnew);
  or_update_E(3 * N, P.theta, E, Eth, Enew);
  or_div_nc(&G, Enew, div);
  or_curl_nc(&G, Enew, cn);
  or_curl_cn(&G, Bnew, cc);
  or_diffusion(&G, kE, Eth, Dy);
  or_mass_apply(&G, Mt, Eth, My);
  double gs[2];
  or_gauss_sums(&G, Enew, rho, gs);
  for (int s = 0; s < 2; ++s) {
    double *xn = zeros(3 * np[s]), *vn = zeros(3 * np[s]);
    int* keep = (int*)calloc((size_t)(np[s] > 0 ? np[s] : 1), sizeof(int));
    for (int64_t p = 0; p < np[s]; ++p) keep[p] = 1;
    or_push_species(&G, beta[s], P.dt, np[s], x[s], v[s], Eth, Bn, xn, vn, keep);
    free(xn); free(vn); free(keep);
  }
  if (3 * N <= 300) {  /* dense operator and its direct solve on the smallest grids */
    double *Ad = zeros(9 * N * N), *xs = zeros(3 * N);
    or_dense_A(&G, &P, Mt, kE, Ad);
    if (or_dense_solve(3 * N, Ad, b, xs) != 0) return 4;
    free(Ad); free(xs);
  }
  for (int i = 0; i < 2; ++i) { free(x[i]); free(v[i]); free(w[i]); free(Ms[i]); }
  free(E); free(B); free(Bn); free(J); free(JC); free(rho); free(mm); free(mass); free(Mt); free(u); free(EM);
  free(a); free(Jeff); free(kE); free(kB); free(b); free(Eth); free(y); free(Bnew); free(Enew); free(div);
  free(cn); free(cc); free(Dy); free(My);
  printf("dim %d grid %dx%dx%d bc %d profile %d: %lld + %lld particles, GMRES %d iterations, relres %.2e\n", dim,
         G.n[0], G.n[1], G.n[2], bc, profile, (long long)np[0], (long long)np[1], it, relres);
  return 0;
}

int main(void) {
  const int n1[3] = {12, 1, 1}, n2[3] = {6, 5, 1}, n3[3] = {5, 4, 3};
  int rc = 0;
  rc |= run_case(1, n1, 0, 0);
  rc |= run_case(1, n1, 2, 0);
  rc |= run_case(2, n2, 0, 2);
  rc |= run_case(2, n2, 1, 0);
  rc |= run_case(3, n3, 0, 2);
  rc |= run_case(3, n3, 2, 0);
  double adv[32];
  for (int i = 0; i < 32; ++i) adv[i] = (i > 8 && i < 16) ? 1.0 : 0.0;
  or_advect(32, adv, 0.4, 1.0, 20, -1.0);
  printf("done rc %d\n", rc);
  return rc;
}
