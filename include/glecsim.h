/*
 * glecsim.h -- C ABI of the MI355X (gfx950) GL-ECSIM particle pass.
 *
 * Method: Chen, Zhou & Toth, "Suppressing spurious oscillations and particle
 * noise in particle-in-cell simulations" (arXiv 2506.11320), built on the
 * energy-conserving semi-implicit PIC scheme (ECSIM).  The library runs one
 * PIC step on one GPU:
 *
 *   deposit   particles -> comoving current J_eff and mass matrices
 *             (Sec. 3.1: predicted current, alpha, mass matrix M_{s,gg'},
 *             comoving decomposition, modified E system)
 *   solve     implicit E^{n+theta} (Sec. 2.1 eq. ECSIM-E with the mass term
 *             of Sec. 3.1 and the limited Lax-Friedrichs diffusion of
 *             Sec. 2.2) by restarted GMRES in FP64
 *   update    B^{n+1} with the limited LF flux (Sec. 2.2 eqs. 1d-b-diss,
 *             flux-b), E^{n+1} from the theta-method (Sec. 2.1)
 *   push      implicit mover (Sec. 3.1), then the particles are re-binned
 *             by cell with a stable integer sort
 *
 * Mesh: E at nodes, B at cell centres (Sec. 2.1); node (i,j,k) at
 * (i dx, j dy, k dz), cell (i,j,k) centred at ((i+1/2) dx, ...).  Active
 * axes are periodic (x may instead end in walls or an inflow plane, see
 * ge_grid) and need at least 3 cells.  Grid arrays are
 * component-major [ncomp][N], linear index i + nx*(j + ny*k), N = cells =
 * nodes.  Units are the normalised Gaussian units of the paper (c, 4 pi).
 *
 * Conventions for every function:
 *  - Return value: GE_OK (0), a negative error code, or a positive warning.
 *    ge_last_error() returns the message of the last failure of a context.
 *  - Pointers documented as "device" are GPU memory owned by the caller and
 *    only read or written during the call (or its stream work); the library
 *    never frees them.  The library owns its own buffers (particles,
 *    mass matrices, Krylov basis) and frees them in ge_destroy().
 *  - All GPU work is enqueued on the stream given to ge_create().  Calls that
 *    return host data (ge_solve_fields, ge_diagnostics, ge_sync, ge_step)
 *    synchronise that stream; the others are asynchronous.
 *  - A context is not thread-safe; use one per host thread.
 */
#ifndef GLECSIM_H
#define GLECSIM_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  GE_OK = 0,
  GE_ERR_ARG = -1,        /* invalid argument or unsupported configuration */
  GE_ERR_OOM = -2,        /* device allocation failed */
  GE_ERR_HIP = -3,        /* a HIP runtime call failed */
  GE_ERR_CFL = -4,        /* a particle would have moved more than n - 2 cells
                             along an axis of n cells in one step (it was kept
                             where it was; the message names the species) */
  GE_ERR_NONFINITE = -5,  /* NaN or Inf met in the solve, or a non-finite
                             particle velocity or position after a push */
  GE_ERR_STATE = -6,      /* call out of order (e.g. push before a solve) */
  GE_WARN_NOT_CONVERGED = 1 /* GMRES hit maxit; best iterate kept */
};

enum { GE_FP64 = 0, GE_FP32 = 1 };           /* particle and mass-matrix precision */
enum { GE_A_LIGHT = 0, GE_A_BULK = 1 };      /* diffusion speed a: c, or |u| */
enum { GE_PC_NONE = 0, GE_PC_JACOBI = 1, GE_PC_CNN = 2 };  /* GMRES preconditioner */
enum { GE_LAG_EN = 0, GE_PICARD1 = 1 };      /* E limiter: lagged to E^n, or one Picard step */
enum { GE_BC_PERIODIC = 0, GE_BC_WALL = 1, GE_BC_INFLOW = 2 };  /* boundary kinds (ge_grid) */

typedef struct ge_ctx ge_ctx;

typedef struct {
  int dim;        /* 1, 2 or 3 active axes (x, then y, then z) */
  int n[3];       /* cells per axis; n[d] >= 3 for active d, 1 otherwise */
  double dx[3];   /* spacing per active axis */
  /* Boundary kinds of the low and high end of each axis.  Every axis is
   * GE_BC_PERIODIC except, optionally, x: bc_lo[0] = GE_BC_WALL (a conducting,
   * specularly reflecting wall at x = 0) with bc_hi[0] = GE_BC_WALL or
   * GE_BC_INFLOW (x = L: E held at its value, upstream B in the ghost cell,
   * particles leave through it; new ones come through ge_inject).  The paper
   * runs its shocks as flows against a boundary (Sec. 4.3, 4.4) but prints no
   * boundary discretisation; the readings: a wall is the mirror plane of the
   * domain (tangential E and normal B odd, normal E and tangential B even),
   * the tangential E on a wall and all of E on an inflow plane are held, no
   * LF flux crosses a boundary (phi = 0 on the face next to a wall), the
   * filter mirrors (normal component odd), and no image charge is deposited.
   * A walled grid stores n[0] + 1 points along x: nodes 0..n[0], the cells
   * 0..n[0]-1 and a ghost cell n[0] (the inflow's upstream B), so every array
   * below has N = (n[0] + 1) n[1] n[2] entries per component. */
  int bc_lo[3], bc_hi[3];
} ge_grid;

typedef struct {
  double theta;       /* time-centring, 0.5 <= theta <= 1 (Sec. 2.1) */
  double c;           /* speed of light */
  double dt;          /* time step */
  int lf_E, lf_B;     /* limited LF diffusion in the E solve / B update (Sec. 2.2) */
  double beta_lim;    /* MC limiter beta (Sec. 2.2); 0 = unlimited first order */
  int a_mode;         /* GE_A_LIGHT (a = a_const) or GE_A_BULK (a = |u|) */
  double a_const;     /* diffusion speed for GE_A_LIGHT */
  int comoving;       /* 1: comoving-frame current (Sec. 3.1), 0: lab frame */
  int n_smooth_u;     /* filter passes for u (Sec. 3.1 uses 5) */
  double phi_u;       /* filter weight (0.5) */
  int precision;      /* GE_FP64 or GE_FP32 (particles, deposit, mass matrices) */
  /* Current smoothing (Sec. 3.2): ns_j passes of the Sec. 2.4 filter (stride 1,
   * weight phi_u, each pass sweeping x, y, z) on the comoving-frame current
   * J_C = J_lab - (1/dV) M0 u (J_lab in the lab frame) before the E_M term is
   * added.  0 = off; the paper uses 1 to 3. */
  int ns_j;
  /* Hyperbolic/parabolic divergence cleaning of B (Sec. 2.3): a cell-centred
   * scalar psi with psi^{n+1} = (psi^n - dt c_h^2 div B^n) exp(-dedner_damp)
   * and B^{n+1} -= dt grad psi^{n+1} (central differences at cell centres),
   * c_h = ch_frac * min dx / dt.  The paper uses ch_frac = 0.8 and
   * dedner_damp = dt c_h^2 / c_p^2 = 0.1.  0 = off. */
  int dedner;
  double ch_frac;
  double dedner_damp;
  /* Electric-field smoothing, the alternative to the LF diffusion that Sec. 4.1
   * compares against (filter of Sec. 2.4): ns_e passes on E^{n+1} right after
   * its update, strides 1, 2, 1, ..., weight phi_u, each pass sweeping x, y,
   * z.  0 = off (the method itself uses the LF diffusion instead). */
  int ns_e;
  /* The E limiter's smoothness ratio r_E uses the unknown E^{n+theta}
   * (Sec. 2.2), which makes the implicit system nonlinear.  GE_LAG_EN takes
   * r_E from E^n (one linear solve per step); GE_PICARD1 then takes one Picard
   * step: the LF coefficients from that first E^{n+theta}, and the system
   * solved again starting from it (twice the solve work). */
  int limiter_lag;
} ge_params;

typedef struct { double q, m; } ge_species;   /* charge and mass per physical particle */

typedef struct {
  int iterations;      /* matvecs spent */
  int restarts;
  int converged;       /* 1 if ||b - A x|| <= tol ||b|| on the true residual */
  double relres;       /* final true relative residual */
  double bnorm;
  double seconds;      /* host wall time of the solve (after queued work) */
  int fallback;        /* 1 if the learned preconditioner failed and plain GMRES finished */
} ge_solve_report;

typedef struct {
  double W_E, W_B;     /* field energies sum |E|^2 dV/8pi (nodes), sum |B|^2 dV/8pi (cells) */
  double K[4];         /* kinetic energy per species, sum 1/2 m w |v|^2 */
  double P[4][3];      /* momentum per species, sum m w v */
  double gauss;        /* ||div_NC E - 4 pi rho_c|| / ||4 pi rho_c||, rho_c = cell mean of node charge */
  int nsp;
} ge_diag;

/* ------------------------------------------------------------------ setup */

/* Create a context.  grid, params: host structs, copied.  hip_stream: a
 * hipStream_t (NULL = the null stream).  *out receives the context.
 * Errors: GE_ERR_ARG for an invalid grid/params, GE_ERR_OOM/HIP. */
int ge_create(const ge_grid* grid, const ge_params* params, void* hip_stream, ge_ctx** out);

/* Free every library-owned buffer.  Accepts NULL. */
void ge_destroy(ge_ctx* ctx);

/* Message of the last failed call on ctx (never NULL).  With ctx NULL: the
 * reason the calling thread's last refused ge_create gave (ge_create returns
 * no context to ask). */
const char* ge_last_error(const ge_ctx* ctx);

/* Add a species of n macro-particles (Sec. 3.1: macro-particles with charge
 * q_s w_p and mass m_s w_p).  All arrays are device memory, read only:
 *   cell[n]      int32 linear cell index, non-decreasing (sorted by cell)
 *   off[3*n]     position inside the cell in units of dx, in [0,1), layout
 *                [3][n]; components of inactive axes are ignored
 *   v[3*n]       velocity, layout [3][n]
 *   w[n]         weight (physical particles per macro-particle)
 * off, v, w are double for GE_FP64 and float for GE_FP32.  Positions are
 * taken as x^{n+1/2} and velocities as v^n.  The data are copied into
 * library-owned buffers.  At most 4 species; call before the first deposit.
 * Errors: GE_ERR_ARG if unsorted, out of range or too many species. */
int ge_add_species(ge_ctx* ctx, const ge_species* sp, int64_t n, const int32_t* cell, const void* off,
                   const void* v, const void* w);

/* Add m particles to species s (new particles entering through an inflow
 * plane, Sec. 4.3-4.4's driven shocks), with the layout of ge_add_species:
 * cell[m] int32 (a cell of the domain, not the ghost), off[3][m], v[3][m],
 * w[m] (device, read during the call).  They join the species at the next
 * synchronising call (with the particles of the last push): in their cell
 * they follow the particles already there, in the given order.  Call between
 * steps (not between a deposit and its field update).  The library grows its
 * particle buffers as needed. */
int ge_inject(ge_ctx* ctx, int s, int64_t m, const int32_t* cell, const void* off, const void* v, const void* w);

/* Copy initial fields: E at nodes, B at cell centres; device double [3][N]. */
int ge_set_fields(ge_ctx* ctx, const double* E_nodes, const double* B_cells);

/* --------------------------------------------------------- step components */

/* Particle-to-grid pass at the current positions (Sec. 3.1): node-averaged
 * B, alpha per particle, lab current, mass matrices
 * Mtilde = sum_s beta_s M_s and M0 = sum_s M_s (half stencil), charge
 * and mass moments; then the smoothed bulk velocity u (n_smooth_u passes of
 * the digital filter of Sec. 2.4), E_M = -u x B, the effective current
 * J_eff = J_lab - (1/dV)(M0 u + Mtilde E_M) (comoving) or J_lab, the LF
 * coefficients (Sec. 2.2, limiter lagged to E^n) and the right-hand side
 * b = E^n + c theta dt curl B^n - 4 pi theta dt J_eff.  Asynchronous. */
int ge_deposit(ge_ctx* ctx);

/* Solve A E^{n+theta} = b (Sec. 2.1/2.2/3.1) by restarted GMRES(restart) in
 * FP64, starting from E^n, until ||b - A x|| <= tol ||b||.  precond:
 * GE_PC_NONE, GE_PC_JACOBI (node 3x3 block diagonal, right-preconditioned) or
 * GE_PC_CNN (flexible GMRES with the learned network of ge_cnn_*, 3D only;
 * on a walled grid the preconditioned vector keeps the input's values on the
 * held boundary components, whose operator rows are the identity (see
 * ge_cnn_apply); falls back to plain GMRES from the current iterate if the network returns
 * NaN/Inf or a restart cycle reduces the residual by less than a factor 2).  If harvesting is
 * on (ge_cnn_harvest), a converged GE_PC_NONE/JACOBI solve also stores
 * training pairs: (b - A E^n, E^{n+theta} - E^n) and/or (A v_j, v_j) for the
 * Arnoldi vectors v_j of its last cycle.
 * report: host struct, may be NULL.  Synchronises.  Returns GE_OK,
 * GE_WARN_NOT_CONVERGED, or an error (GE_ERR_STATE before ge_deposit). */
int ge_solve_fields(ge_ctx* ctx, double tol, int maxit, int restart, int precond, ge_solve_report* report);

/* Implicit mover (Sec. 3.1) with E^{n+theta} from the last solve and the
 * node-averaged B^n of the last deposit, then the stable re-binning of every
 * species by cell.  A particle may move up to n - 2 cells along an axis of n
 * cells (its new position relative to its old cell in [-(n - 2), n - 1) cells;
 * further, the periodic wrap could bring it back next to its old cell):
 * moves of at most one cell are re-binned inside the push; if any
 * particle moved further, the next call that reads the particles (ge_deposit,
 * ge_push, ge_get_particles, ge_diagnostics, ge_sync, ge_step's own end, ...)
 * synchronises once and runs a stable re-sort of that species, so that the
 * order is always the stable sort by cell of the previous order.
 * Asynchronous; GE_ERR_CFL (a longer move: the particle is kept in place) and
 * GE_ERR_NONFINITE are reported by that next call. */
int ge_push(ge_ctx* ctx);

/* B^{n+1} = B^n - c dt curl E^{n+theta} + dt D_B(B^n) and
 * E^{n+1} = (E^{n+theta} - (1 - theta) E^n)/theta.  Asynchronous. */
int ge_update_fields(ge_ctx* ctx);

/* One full step: deposit, solve, push, update.  Synchronises. */
int ge_step(ge_ctx* ctx, double tol, int maxit, int restart, int precond, ge_solve_report* report);

/* Steps completed on this context (field updates of ge_update_fields /
 * ge_step and explicit steps), restored by ge_restore. */
int64_t ge_step_count(const ge_ctx* ctx);

/* Macro-particles of species s (-1 if there is no such species). */
int64_t ge_species_count(const ge_ctx* ctx, int s);

/* Checkpoint of the state between steps to the file at path (host string):
 * grid and parameters, the step count, E^n, B^n, the cleaning scalar psi,
 * every species (charge, mass and its particles in cell order) and, if the
 * learned preconditioner exists, its master weights, Adam moments and step
 * (not its pair store).  Settles the last push first; synchronises.  Errors:
 * GE_ERR_STATE between a deposit and its field update, GE_ERR_ARG if the file
 * cannot be written. */
int ge_checkpoint(ge_ctx* ctx, const char* path);

/* Restore a checkpoint into a context created with the same grid and
 * parameters and with no species yet.  Continuing from the restored state
 * gives the same bits as continuing the run that wrote it (the particle
 * order is the cell order of the run).  Synchronises.  Errors: GE_ERR_ARG for
 * a missing, truncated or corrupt file (checksum) or a grid/parameter
 * mismatch, GE_ERR_STATE if the context already has species. */
int ge_restore(ge_ctx* ctx, const char* path);

/* Current of an explicit PIC step at the particles' present positions and
 * velocities (Sec. 3.1, its explicit form).  Comoving frame on:
 * J_g = (1/dV) sum_{s,p} q_s w_p (v_p - u(x_p)) W(x_p - x_g), with u the bulk
 * velocity after n_smooth_u filter passes, interpolated to the particle with
 * the same weights W; comoving frame off: the lab current
 * (1/dV) sum q w v W.  Then ns_j filter passes (Sec. 3.2).  Two passes over
 * the particles, no mass matrices: the moments (-> u, also left in GE_F_MASS,
 * GE_F_MM and GE_F_U), then the current.  The moments and current of the
 * implicit step are overwritten, so ge_solve_fields needs a new ge_deposit
 * afterwards (GE_ERR_STATE otherwise).  J: device [3][N] FP64, may be NULL
 * (the result stays readable as GE_F_J_EFF).  Asynchronous. */
int ge_explicit_current(ge_ctx* ctx, double* J);

/* One explicit PIC step that uses that current (the paper states the current
 * for explicit codes but no explicit integrator; this is the leapfrog it
 * writes for the 1D Yee scheme, Sec. 2.1, on this node/cell mesh).  The
 * particle state is read as (x^n, v^{n-1/2}), the fields as E^n, B^n:
 *   v^{n+1/2}: Boris push with E^n and the node-averaged B^n at x^n (the
 *   mover of ge_push with E^n in place of E^{n+theta}); x^{n+1} = x^n +
 *   dt v^{n+1/2}; re-binning;
 *   J from ge_explicit_current at (x^{n+1}, v^{n+1/2});
 *   B^{n+1/2} = B^n - (c dt/2) curl_NC E^n, E^{n+1} = E^n + c dt curl_CN
 *   B^{n+1/2} - 4 pi dt J, B^{n+1} = B^{n+1/2} - (c dt/2) curl_NC E^{n+1}.
 * theta, the LF terms and the cleaning are not used.  Stable for
 * c dt < min dx / sqrt(dim).  Synchronises; returns GE_ERR_CFL like
 * ge_sync if a particle moved a cell or more. */
int ge_explicit_step(ge_ctx* ctx);

/* Wait for the stream and settle the last push (see ge_push); returns
 * GE_ERR_CFL or GE_ERR_NONFINITE if a push kept a particle in place since the
 * last check, else GE_OK. */
int ge_sync(ge_ctx* ctx);

/* Particle moves since the last call (host struct), per species: particles
 * that moved more than one cell along some axis in one push, and the largest
 * move in cells (max over pushes and axes of |v_d| dt / dx_d); then the stable
 * re-sorts those moves needed and the pushes counted.  Synchronises (settles
 * the last push) and resets the counters. */
typedef struct {
  int64_t far_moves[4];
  double max_move[4];
  int resorts;
  int pushes;
  int64_t gone[4];       /* particles that left through an inflow plane */
  int64_t injected[4];   /* particles added by ge_inject */
} ge_move_report;
int ge_moves(ge_ctx* ctx, ge_move_report* out);

/* ------------------------------------------------------- inputs and outputs */

enum {
  GE_F_E = 0,        /* E^n at nodes            [3][N] */
  GE_F_B = 1,        /* B^n at cells            [3][N] */
  GE_F_ETH = 2,      /* E^{n+theta}             [3][N] */
  GE_F_BN = 3,       /* B averaged to nodes     [3][N] */
  GE_F_J_LAB = 4,    /* lab current             [3][N] */
  GE_F_J_EFF = 5,    /* effective current       [3][N] */
  GE_F_RHO = 6,      /* charge density per species [nsp][N] */
  GE_F_MM = 7,       /* sum_s m_s sum_p w v W   [3][N] */
  GE_F_MASS = 8,     /* sum_s m_s sum_p w W     [N] */
  GE_F_U = 9,        /* smoothed bulk velocity  [3][N] */
  GE_F_EM = 10,      /* motional field -u x B   [3][N] */
  GE_F_MTILDE = 11,  /* sum_s beta_s M_s, half stencil [nh][9][N] */
  GE_F_M0 = 12,      /* sum_s M_s, half stencil [nh][9][N] */
  GE_F_KAPPA_E = 13, /* E diffusion coefficients [3 axes][3 comps][N] */
  GE_F_KAPPA_B = 14, /* B diffusion coefficients [3 axes][3 comps][N] */
  GE_F_RHS = 15,     /* right-hand side b       [3][N] */
  GE_F_PSI = 16      /* divergence-cleaning scalar at cells [N] */
};
/* Half stencil: nh = 14 (3D), 5 (2D), 2 (1D) offsets o with M_{g,g+o}
 * stored at node g: o = 0 first, then every o != 0 whose last nonzero
 * component (z, then y, then x) is +1, enumerated z-major then y then x.
 * M_{g+o,g} equals M_{g,g+o} (the same 3x3, not transposed), entry e = 3i+j. */

/* Copy an internal field to dst (device double, the layout above).
 * GE_F_MTILDE/M0 are widened to double for GE_FP32. */
int ge_gather(ge_ctx* ctx, int what, double* dst);

/* Overwrite an internal field from src (device double, same layout).  Only
 * GE_F_E, GE_F_B, GE_F_ETH, GE_F_BN and GE_F_RHS may be set; it lets a caller
 * drive one component from known inputs (e.g. a push with a given E^{n+theta}). */
int ge_set(ge_ctx* ctx, int what, const double* src);

/* Number of half-stencil offsets (14, 5 or 2). */
int ge_half_stencil(const ge_ctx* ctx);

/* Particles of species s in sorted order (by cell, stable), into device
 * arrays: cell[n] int32, off[3][n], v[3][n], w[n] (double for GE_FP64,
 * float for GE_FP32).  n must equal the species' count; for an empty species
 * (n = 0) it returns GE_OK at once and the pointers may be null. */
int ge_get_particles(ge_ctx* ctx, int s, int64_t n, int32_t* cell, void* off, void* v, void* w);

/* y = A x for the current operator (device double [3][N]); the matvec of the
 * solve.  Asynchronous. */
int ge_apply_operator(ge_ctx* ctx, const double* x, double* y);

/* FP64 energies, momenta and Gauss residual (host struct).  Synchronises. */
int ge_diagnostics(ge_ctx* ctx, ge_diag* out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid it): ge_diagnostics
 * without any allocation.  Same results as ge_diagnostics, bit for bit (same
 * kernels, same summation order); its reduction partials live in a static
 * device array of 4 x 256 + 4 doubles per GPU, which every reduction fits
 * (they always run on 256 blocks).  It allocates nothing, reads back through
 * the pinned host buffer of the context, and synchronises.  Every call on a
 * GPU shares that GPU's array: calls that overlap on one GPU (other threads,
 * other contexts) race.  Errors: GE_ERR_STATE if a push is not settled yet
 * (call ge_sync first: settling may re-sort far movers, which allocates on
 * first use) or if the context has no scratch address for its device. */
int ge_diagnostics_noalloc(ge_ctx* ctx, ge_diag* out);

/* Mean seconds per ge_step() since the last call, from HIP events recorded on
 * the context's stream around each kernel group; host array of 8:
 *   [0] push + re-binning kernels (all species: corner-field packing,
 *       segment scans, pushes; a re-sort of far movers is not included)
 *                                                 [1] deposit kernel
 *   [2] node assembly kernel                      [3] rest of the grid pass
 *   [4] field update kernels                      [5] solve (host wall time)
 *   [6] the part of [0] before the pushes: corner-field packing and the
 *       segment scans (the re-binning's own kernels; the pushes record the
 *       direction runs as they write)            [7] number of steps averaged
 * The accumulators are reset by the call. */
int ge_timings(ge_ctx* ctx, double* out8);

/* ------------------------------------------------ learned preconditioner */
/* Not from the paper: a 3-layer 3x3x3 convolutional network z = N(r)
 * (3 -> 32 -> 32 -> 3 channels, ReLU after the first two, no bias), BF16 MFMA
 * with FP32 accumulation, trained on (residual, correction) pairs of the solves
 * and used as a flexible right preconditioner; the GMRES residual decides:
 * the solve must still reach ||b - A x|| <= tol ||b||. */
typedef struct {
  int crop;       /* output crop edge in nodes (input crop = crop + 6) */
  int batch;      /* crops per step (1..64) */
  int iters;      /* optimiser steps */
  double lr, beta1, beta2, eps;  /* Adam */
  uint32_t seed;  /* crop origins and pair mixing */
} ge_train_cfg;
typedef struct {
  int steps, pairs;
  double loss_first, loss_last;  /* mean squared error of the first and last step */
  double seconds;
} ge_train_report;

enum { GE_HARVEST_SOLUTION = 1, GE_HARVEST_KRYLOV = 2 };  /* ge_cnn_harvest flags */

/* Create (or reset) the network with weights near the identity map plus
 * small seeded noise, and reset the Adam state (3D grids only).  max_pairs:
 * capacity of the pair store (1..1024, 0 = 64), fixed by the first call;
 * each pair takes 24 N bytes of device memory. */
int ge_cnn_init(ge_ctx* ctx, uint32_t seed, int max_pairs);
/* Number of FP32 master weights: layers [27 taps][cout][cin] for
 * (cin, cout) = (3, 32), (32, 32), (32, 3), concatenated. */
int ge_cnn_size(void);
/* Copy the master weights to (set = 0) or from (set = 1) host_w[ge_cnn_size()]. */
int ge_cnn_weights(ge_ctx* ctx, int set, float* host_w);
/* z = N(r) on the whole periodic grid, r normalised by its RMS and the
 * output scaled back (device double [3][N]).  On a walled grid the network
 * sees a domain periodic along x over the node planes that are not wholly
 * held (an inflow plane is left out), and z = r on the held components.
 * Synchronises. */
int ge_cnn_apply(ge_ctx* ctx, const double* r, double* z);
/* z = N(scale r) / scale: ge_cnn_apply with the input scale given by the
 * caller instead of 1 / RMS(r) (the form the flexible GMRES of ge_solve uses,
 * where the Krylov vectors' norms are known), so no reduction and no host
 * round trip.  scale must be finite and positive (else GE_ERR_ARG); since
 * the network is positively homogeneous, scale only sets where the BF16
 * activations sit (scale r of RMS near 1 is what the network was trained on).
 * Same walled-grid behaviour as ge_cnn_apply.  Asynchronous. */
int ge_cnn_apply_scaled(ge_ctx* ctx, const double* r, double* z, double scale);
/* Pair harvesting from converged solves: 0 = off, else an OR of
 * GE_HARVEST_SOLUTION (the pair (b - A E^n, E^{n+theta} - E^n)) and
 * GE_HARVEST_KRYLOV (the exact pairs (A v_j, v_j) of the last cycle's Arnoldi
 * vectors, one extra matvec each). */
int ge_cnn_harvest(ge_ctx* ctx, int flags);
/* Store a (residual, correction) pair (device double [3][N]); the store keeps
 * the newest max_pairs pairs (ge_cnn_init).  Synchronises. */
int ge_cnn_add_pair(ge_ctx* ctx, const double* r, const double* e);
/* Number of stored pairs. */
int ge_cnn_npairs(const ge_ctx* ctx);
/* Train with Adam on random crops of random unit-norm combinations of two
 * stored pairs (mean squared error).  Synchronises. */
int ge_cnn_train(ge_ctx* ctx, const ge_train_cfg* cfg, ge_train_report* report);
/* Loss and gradient for caller crops (device FP32): in_crops [B][(n+6)^3][3],
 * tgt [B][n^3][3]; grad [ge_cnn_size()] (device FP32); loss on the host. */
int ge_cnn_loss_grad(ge_ctx* ctx, int B, int n, const float* in_crops, const float* tgt, float* grad, double* loss);

#ifdef __cplusplus
}
#endif
#endif
