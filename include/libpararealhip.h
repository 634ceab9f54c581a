/*
 * libpararealhip -- Krylov-subspace-enhanced Parareal for the linear 2D
 * acoustic-advection system on one AMD MI355X (gfx950), FP64 throughout.
 *
 * Method: Ruprecht & Krause, "Explicit parallel-in-time integration of a
 * linear acoustic-advection system" (Computers & Fluids), Section 2
 * (Algorithm 2 with the modified coarse propagator of eq. modifiedCoarse and
 * the fine images of eq. Genhance) applied to eq. acousticAd with the
 * discretisation of Section 3 and Section 3.2.
 *
 * Problem.  u_t + U u_x + c_s p_x = alpha_1 (div u)_x,
 *           w_t + U w_x + c_s p_z = alpha_2 (div u)_z,
 *           p_t + U p_x + c_s (u_x + w_z) = 0
 * on the periodic rectangle [0,Lx) x [0,Lz) with nx x nz equal cells,
 * constant advection velocity U along x (eq. acousticAd with the damping of
 * Section 3.2 and the coefficients of eq. dampingCoeff).
 *
 * State layout (every state, on host or device):
 *     double q[3][nz][nx]      field order u, w, p; x fastest (row-major);
 *                              d = 3*nx*nz doubles, cell (i,j) centred at
 *                              ((i+1/2)Lx/nx, (j+1/2)Lz/nz).
 * A set of states is contiguous: state s starts at q + s*d.
 *
 * Time slicing: one window of P slices of length T/P (Section 2.1); the
 * fine propagator F takes n_f = (T/P)/dt_f RK-3 steps, the coarse
 * propagator G takes n_g = (T/P)/dt_g partially split steps.
 *
 * Memory.  Every entry point that takes state pointers has a `mem`
 * argument: PR_MEM_HOST (pageable host memory; the call copies in and out
 * and returns after the result is on the host) or PR_MEM_DEVICE (device
 * pointers on the context's device, e.g. torch tensors; work is enqueued
 * on the context's stream and the call returns after that stream has
 * drained).  Buffers passed in are owned by the caller.  The context owns
 * its device arena (iterates, basis S, the fine-minus-coarse images of the
 * basis, scratch).
 *
 * Errors.  Every int-returning call returns PR_OK (0) or a negative code.
 * On error, output buffers are left untouched and pr_last_error(ctx)
 * describes the failure.  A context is single-threaded; a server is safe
 * to call from several host threads.
 */
#ifndef LIBPARAREALHIP_H
#define LIBPARAREALHIP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  PR_OK = 0,
  PR_EINVAL = -1,     /* bad argument (sizes, step ratios, null pointers)   */
  PR_ENOMEM = -2,     /* device allocation failed / footprint over budget   */
  PR_EDEVICE = -3,    /* HIP runtime error                                  */
  PR_EUNSTABLE = -4,  /* F or G amplifies some Fourier mode (rho > 1+1e-12) */
  PR_EAGAIN = -5,     /* served request still pending                       */
  PR_EBUSY = -6,      /* server queue full                                  */
  PR_EDIVERGED = -7,  /* non-finite iterate                                 */
  PR_ENOTFOUND = -8   /* unknown ticket                                     */
};

enum { PR_MEM_HOST = 0, PR_MEM_DEVICE = 1 };

/* How the fine sweep is launched.
 *   PR_FORM_BATCHED:   one fused-step launch per RK-3 step covers every
 *     slice of the sweep (and, in the server, every resident solve); each
 *     iteration's sweep is replayed from a captured HIP graph.
 *   PR_FORM_PLAIN:     one fused-step launch per slice per RK-3 step, slices
 *     in turn.
 *   PR_FORM_STAGEWISE: unfused comparison form, three stage launches per
 *     RK-3 step over all slices, neighbours read from global memory.  For
 *     right-hand sides with per-row and per-column advective weights (see
 *     fine_acoustic_order) it is the only form, and an RK-3 step is one
 *     launch that runs the three stages on tiles held in LDS.
 * All forms give bitwise-identical fine results for the fused forms and
 * results equal to rounding for the stagewise form. */
enum { PR_FORM_BATCHED = 0, PR_FORM_PLAIN = 1, PR_FORM_STAGEWISE = 2 };

/* Which pair of propagators.
 *   PR_SCHEME_SPLIT (default): those of Section 3.2.  F is RK-3 with
 *     fifth-order upwind advection, fourth-order centred acoustics and
 *     divergence damping (nu_f).  G is partially split forward Euler with
 *     N_sound forward-backward acoustic substeps and damping (nu_c).
 *     The advection velocity is (U + gamma (z - Lz/2), V - gamma (x - Lx/2))
 *     with V and gamma from pr_opts (eq. adVel); by default (U, 0).
 *   PR_SCHEME_RK3: those of the instability example of Section 3.1.  F is
 *     RK-3 with the sixth-order centred advective flux; G is RK-3 with the
 *     first-order upwind flux (step dt_g).  Both use second-order centred
 *     acoustic fluxes and no damping (nu_f, nu_c and n_sound are unused).
 *     Advection is along x and z with velocity (U, pr_opts.V).  Every sweep
 *     runs the unfused stage kernels (the form is ignored); the server does
 *     not accept this scheme. */
enum { PR_SCHEME_SPLIT = 0, PR_SCHEME_RK3 = 1 };

typedef struct pr_grid {
  int32_t nx, nz;   /* cells along x and z, each >= 8                  */
  double Lx, Lz;    /* domain lengths (> 0)                            */
  double T;         /* end time of the window (> 0)                    */
} pr_grid;

typedef struct pr_opts {
  double nu_f;            /* fine divergence damping nu_f (Section 3.2: 0.005) */
  double nu_c;            /* coarse divergence damping nu_c (0.1)              */
  int32_t n_sound;        /* acoustic substeps per coarse step N_sound (4)     */
  double rank_tol;        /* keep a new basis direction if its residual norm
                             exceeds rank_tol times the largest raw column
                             norm seen (1e-10)                                 */
  int32_t form;           /* PR_FORM_BATCHED (default) or PR_FORM_PLAIN        */
  int32_t skip_converged; /* 1 (default): in iteration k skip the fine
                             propagation of slices i < k, whose inputs are
                             bitwise those of iteration k-1 (Section 2.1:
                             after k iterations slices 0..k are exact)         */
  int32_t tile_nt;        /* fine-sweep threads per workgroup: 128, 192 or 256
                             (tiles with an x-halo), or nx when nx is 128, 256
                             or 512 (one workgroup per periodic row, no halo);
                             0 = autotune                                      */
  int32_t tile_zc;        /* fine-sweep output rows per workgroup (multiple of
                             4), 0 = autotune                                  */
  int32_t windows;        /* parallel steps M_p of Section 2.1: [0, T] is
                             integrated in `windows` sequential windows of P
                             slices, each slice T / (windows * P) long; every
                             window starts from the previous window's final
                             state with an empty subspace (the initialization
                             of Algorithm 2).  1 (default) = one window.  With
                             dt_g = T / (windows * P) every slice is one
                             coarse step, as in the paper's runs.  The server
                             accepts only 1.                                   */
  int32_t scheme;         /* PR_SCHEME_SPLIT (default) or PR_SCHEME_RK3       */
  double V;               /* constant part of the advection velocity along z
                             (default 0); U (an argument of pr_create) is the
                             one along x                                        */
  double stop_tol;        /* stopping criterion of Section 2.1: 0 (default)
                             runs exactly K iterations; > 0 ends a window
                             after the first iteration k whose error
                             estimate r^k = max_i ||q^{k+1}_i - q^k_i|| /
                             max_i ||q^{k+1}_i|| (Euclidean norms of whole
                             states, i = 1..P) is <= stop_tol, K being the
                             maximum.  Costs one copy and two norm passes
                             over the iterates per iteration.  The server
                             accepts only 0.                                   */
  double gamma;           /* rotation rate of the solid-body part of the
                             advection velocity, PR_SCHEME_SPLIT only: the
                             velocity is (U + gamma (z - Lz/2), V - gamma
                             (x - Lx/2)), eq. adVel of Section 3.2 with
                             gamma = pi and U = V = 0 (one revolution in
                             T = 2).  Default 0.                               */
  int32_t fine_acoustic_order; /* order of the centred acoustic differences
                             of F in PR_SCHEME_SPLIT: 4 (default) or 2
                             (Section 3 computes the acoustic fluxes of both
                             propagators to second order).  PR_SCHEME_RK3
                             always uses 2.

                             With V != 0, gamma != 0 or fine_acoustic_order
                             = 2, F runs in PR_FORM_STAGEWISE (per-row and
                             per-column advective weights, one launch per
                             RK-3 step) and each coarse step evaluates the
                             slow tendency of G from per-row and per-column
                             weights; the server accepts none of these.      */
  int32_t coarse_order;   /* order of the upwind slow tendency of G in
                             PR_SCHEME_SPLIT: 1 (default, the main runs of
                             Section 3.2) or 3 (its less diffusive G; the
                             slow tendency then comes from per-row and
                             per-column weights, as with V or gamma).
                             Forward Euler on the frozen third-order tendency
                             grows on long waves, so with a constant velocity
                             pr_create returns PR_EUNSTABLE.  The server
                             accepts only 1.                                   */
} pr_opts;

typedef struct pr_ctx pr_ctx;
typedef struct pr_server pr_server;

/* Phase timings of the last pr_solve (device time from HIP events on the
 * context stream, milliseconds) and the basis dimension after each
 * iteration. */
typedef struct pr_stats {
  double ms_total, ms_coarse_init, ms_fine, ms_update, ms_chain;
  int32_t iterations;
  int32_t rank[64];         /* dim S^k after iteration k (k < 64)         */
  int64_t fine_point_steps; /* grid points x RK-3 steps done by the sweeps */
  double residual[64];      /* r^k after iteration k (k < 64) when
                               stop_tol > 0, else 0                        */
  int32_t tile_nt, tile_zc; /* tile of the fused fine step in the sweep
                               over the most slices (threads per workgroup,
                               output rows per workgroup), as set in
                               pr_opts or chosen by the autotuner; 0 when
                               the sweeps ran in the stage form           */
} pr_stats;

/* Fills the defaults listed above. */
void pr_opts_default(pr_opts* o);

/* Host-only check of the von Neumann amplification of F (one RK-3 step of
 * the fine semi-discretisation) and G (one partially split coarse step),
 * Section 3 and Section 3.2.  Scans every discrete Fourier mode when
 * nx*nz <= 65536, else a 256 x 256 sample of phase angles that contains the
 * axis modes.  Writes the largest spectral radii found.  The scan is exact
 * for a constant velocity.  With pr_opts.gamma != 0 the coefficients vary
 * in space and no Fourier mode is invariant: the radii are then those of
 * the symbols frozen at the four extreme velocity pairs of the grid (the
 * largest and smallest x-velocity of a row with the largest and smallest
 * z-velocity of a column), a local estimate that may exceed 1 for a stable
 * propagator.  Returns PR_EINVAL for bad parameters, else PR_OK.  Never
 * touches the GPU. */
int pr_check_stability(const pr_grid* g, double c_s, double U, double dt_f,
                       double dt_g, const pr_opts* o, double* rho_f,
                       double* rho_g);

/* Device bytes a context needs for P slices and a basis of up to P*K
 * vectors: (2*P*K + 4*P + 4) * d * 8 plus small tables. */
int pr_footprint(const pr_grid* g, int32_t P, int32_t K, size_t* bytes);

/* Creates a context for one problem: grid, sound speed c_s, advection
 * velocity U (along x), fine step dt_f (delta t), coarse step dt_g
 * (Delta t), P slices over [0, T] (Section 2.1).  pr_create uses the
 * default options and the null (default) stream of device 0's current
 * device.  pr_create_ex takes options and a hipStream_t (NULL = default
 * stream).  PR_EINVAL: nx or nz < 8, P < 1, non-positive lengths or steps,
 * (T/P)/dt_f or (T/P)/dt_g not an integer within 1e-9 relative,
 * n_sound < 1, an option out of range.  PR_EUNSTABLE: pr_check_stability
 * finds rho > 1 + 1e-12 for a constant velocity (gamma = 0; with gamma != 0
 * the frozen-coefficient estimate is not enforced).  Device memory is
 * allocated lazily by the first call that needs it, except the per-row and
 * per-column stage weights ((nx + nz) * 14 doubles), allocated here when the
 * options need them. */
int pr_create(const pr_grid* g, double c_s, double U, double dt_f,
              double dt_g, int32_t P, pr_ctx** out);
int pr_create_ex(const pr_grid* g, double c_s, double U, double dt_f,
                 double dt_g, int32_t P, const pr_opts* o, void* hip_stream,
                 pr_ctx** out);
void pr_destroy(pr_ctx* ctx);
/* Switches the fine-sweep launch form (PR_FORM_*) of an existing context. */
int pr_set_form(pr_ctx* ctx, int32_t form);
/* on = 0 replaces the FP64 MFMA kernels of the subspace update with plain
 * FMA kernels of the same blocking (cross-check); default on. */
int pr_set_mfma(pr_ctx* ctx, int32_t on);

/* Fine propagator over one slice for `nslices` independent states
 * (Algorithm 2, parallel predictor step; F of Section 3.2: n_f steps of the
 * three-stage Runge-Kutta scheme with 5th-order upwind advection along the
 * velocity of pr_opts (U, V, gamma), centred acoustic terms of order
 * opts.fine_acoustic_order and divergence damping nu_f; with
 * PR_SCHEME_RK3 the F of Section 3.1).
 * Q, FQ: [nslices][3][nz][nx]; FQ[s] = F(Q[s]).  Q and FQ must not overlap.
 * The launch form follows opts.form.  1 <= nslices <= 4096. */
int pr_fine_sweep(pr_ctx* ctx, const double* Q, double* FQ, int32_t nslices,
                  int mem);

/* Coarse propagator over one slice (n_g partially split forward-Euler steps
 * with N_sound forward-backward acoustic substeps and the upwind slow
 * tendency of order opts.coarse_order, Section 3.2; with PR_SCHEME_RK3 the
 * G of Section 3.1), or, with
 * use_krylov != 0, the modified coarse propagator of eq. modifiedCoarse,
 * K(q) = G((I - P)q) + F(P q), with the context's current basis (eq.
 * Genhance).  q, gq: one state each; they may alias. */
int pr_coarse_step(pr_ctx* ctx, const double* q, double* gq, int use_krylov,
                   int mem);

/* Subspace update (Section 2.2, eq. subspaceUpdate): appends the span of the
 * m states Q[0..m) to the context's basis S, with their fine images
 * FQ[s] = F(Q[s]) (caller-computed) giving F(S) by linearity (eq. Genhance).
 * Directions whose residual after projection onto the basis falls below the
 * rank tolerance are dropped.  *rank_out (may be NULL) receives dim S.
 * PR_ENOMEM if the basis would exceed its capacity of P*max(K,1) vectors
 * set by the last pr_solve or by pr_reserve_basis (default P*P, at most
 * 4096). */
int pr_krylov_update(pr_ctx* ctx, const double* Q, const double* FQ,
                     int32_t m, int32_t* rank_out, int mem);
/* Empties the basis (S^0 = F(S^0) = empty, Algorithm 2 initialisation). */
int pr_krylov_reset(pr_ctx* ctx);
/* Sets the basis capacity (vectors) used by pr_krylov_update. */
int pr_reserve_basis(pr_ctx* ctx, int32_t max_vectors);

/* KSE-Parareal (Algorithm 2) with K iterations from u0 over [0, T]:
 * coarse initialisation, then K times {fine sweep over all slices, subspace
 * update, serial correction}.  U_K: [3][nz][nx], the iterate q^K_P at t = T.
 * slices_or_NULL: if not NULL, [P+1][3][nz][nx] receives q^K_0..q^K_P.
 * K = 0 returns the coarse prediction; K >= P returns the serial fine
 * solution F^P(u0) bitwise.  The result is linear in u0.  PR_EDIVERGED if
 * an iterate is not finite. */
int pr_solve(pr_ctx* ctx, const double* u0, int32_t K, double* U_K,
             double* slices_or_NULL, int mem);
/* Same as pr_solve with the original Parareal (Algorithm 1, S = empty). */
int pr_solve_parareal(pr_ctx* ctx, const double* u0, int32_t K, double* U_K,
                      double* slices_or_NULL, int mem);

/* Serial fine reference: F applied nslices times to u0 (q_seq of
 * eq. errorDef when nslices = P).  out: one state. */
int pr_serial_fine(pr_ctx* ctx, const double* u0, int32_t nslices,
                   double* out, int mem);

/* Statistics of the last pr_solve. */
int pr_get_stats(const pr_ctx* ctx, pr_stats* s);

/* Continuous-batching server on one device.  Requests are admitted while
 * their footprint (pr_footprint) fits hbm_budget_bytes (0 = 90% of free
 * device memory) and fewer than max_inflight solves are resident; each
 * solve's iterates and basis stay on the device between iterations, and
 * the fine sweeps of all resident solves that are in their sweep phase are
 * fused into shared launches.  pr_submit copies u0 (host memory) and
 * returns a ticket; PR_EBUSY if the queue (4096 requests) is full,
 * PR_EINVAL / PR_EUNSTABLE as pr_create.  pr_poll returns PR_EAGAIN while
 * the request is pending; on completion it copies q^K_P to U_K (host,
 * may be NULL), writes the submit-to-completion latency in seconds, and
 * forgets the ticket.  pr_cancel drops a pending or running request. */
int pr_server_create(int device, size_t hbm_budget_bytes,
                     int32_t max_inflight, pr_server** out);
int pr_submit(pr_server* s, const pr_grid* g, double c_s, double U,
              double dt_f, double dt_g, int32_t P, int32_t K,
              const double* u0, uint64_t* ticket);
int pr_submit_ex(pr_server* s, const pr_grid* g, double c_s, double U,
                 double dt_f, double dt_g, int32_t P, int32_t K,
                 const pr_opts* o, const double* u0, uint64_t* ticket);
int pr_poll(pr_server* s, uint64_t ticket, double* U_K, double* latency_s);
int pr_cancel(pr_server* s, uint64_t ticket);
/* Blocks until every submitted request has completed or been cancelled. */
int pr_server_drain(pr_server* s);
void pr_server_destroy(pr_server* s);

const char* pr_strerror(int code);
const char* pr_last_error(const pr_ctx* ctx);
const char* pr_server_last_error(const pr_server* s);

#ifdef __cplusplus
}
#endif

#endif /* LIBPARAREALHIP_H */
