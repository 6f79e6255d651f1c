/* FP64 CPU oracle of the GL-ECSIM particle pass (test infrastructure only).
 * Own header: nothing here is shared with the GPU library. */
#ifndef GLECSIM_ORACLE_H
#define GLECSIM_ORACLE_H
#include <stdint.h>

/* bc_lo, bc_hi: boundaries of the x axis, 0 periodic (both), or bc_lo = 1 (a
 * conducting, reflecting wall at x = 0) with bc_hi = 1 (wall) or 2 (inflow) at
 * x = L.  Walled grids store n[0] = nx + 1 points along x: nodes 0..nx, the
 * physical cells 0..nx-1 and one ghost cell nx (the inflow's upstream B). */
typedef struct { int dim; int n[3]; double dx[3]; int bc_lo, bc_hi; } or_grid;
typedef struct { double theta, c, dt; } or_params;

int64_t or_nnodes(const or_grid* G);
int or_shape(const or_grid* G, const double x[3], int64_t nodes[8], double W[8]);
void or_alpha(double beta, const double B[3], double alpha[9]);
void or_node_avg(const or_grid* G, const double* Bc, double* Bn);
void or_deposit_species(const or_grid* G, double qs, double ms, double beta_s, int64_t np, const double* x,
                        const double* v, const double* w, const double* Bn, const double* u_node, double* J,
                        double* M, double* rho, double* mm, double* mass);
void or_bulk_velocity(const or_grid* G, const double* mm, const double* mass, double* u);
void or_filter_axis(const or_grid* G, double* f, int ncomp, double phi, int stride, int axis);
void or_smooth(const or_grid* G, double* f, int ncomp, int npass, double phi);
void or_motional(const or_grid* G, const double* u, const double* Bn, double* EM);
void or_mass_apply(const or_grid* G, const double* M, const double* x, double* y);
void or_current_eff(const or_grid* G, const double* JC, const double* Mtilde, const double* EM, double* Jeff);
double or_limiter(double num, double den, double beta);
void or_kappa_E(const or_grid* G, const double* E, const double* a_node, double beta, double* kappa);
void or_kappa_B(const or_grid* G, const double* B, const double* a_node, double beta, double* kappa);
void or_curl_nc(const or_grid* G, const double* E, double* out);
void or_curl_cn(const or_grid* G, const double* B, double* out);
void or_div_nc(const or_grid* G, const double* E, double* out);
void or_gauss_sums(const or_grid* G, const double* E, const double* rho_node, double out[2]);
void or_diffusion(const or_grid* G, const double* kappa, const double* F, double* out);
void or_apply_A(const or_grid* G, const or_params* P, const double* Mtilde, const double* kappaE, const double* x,
                double* y);
void or_rhs(const or_grid* G, const or_params* P, const double* En, const double* Bc, const double* Jeff, double* b);
void or_update_B(const or_grid* G, const or_params* P, const double* Bc, const double* Eth, const double* kappaB,
                 double* Bnew);
void or_update_E(int64_t n3, double theta, const double* En, const double* Eth, double* Enew);
void or_push_species(const or_grid* G, double beta_s, double dt, int64_t np, const double* x, const double* v,
                     const double* Eth, const double* Bn, double* xnew, double* vnew, int* keep);
int or_gmres(const or_grid* G, const or_params* P, const double* Mtilde, const double* kappaE, const double* b,
             double* x, double tol, int maxit, int restart, double* relres_out);
void or_dense_A(const or_grid* G, const or_params* P, const double* Mtilde, const double* kappaE, double* Ad);
int or_dense_solve(int64_t n, const double* A, const double* b, double* x);
void or_advect(int n, double* u, double nu, double beta, int nsteps, double phi_override);
#endif
