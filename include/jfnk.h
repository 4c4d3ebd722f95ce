/*
 * jfnk.h - C ABI of the MI355X (gfx950) symmetry-preserving Jacobian-free
 * Newton-Krylov hot path for the dry nonhydrostatic model.
 *
 * Problem statement followed (section 2.5): find u with L(u) = f(u^n) where
 * L(u) = 2u/dt - F(u) and f(u^n) = 2u^n/dt + F(u^n) (trapezoidal step, eq. 5),
 * F the spatially discrete operator of equations 1-3 (eq. 4).  Newton solves
 * J(u) du = -R(u), R(u) = L(u) - f (eq. 8), by GMRES with the Jacobian applied
 * matrix-free as the Frechet derivative of R (eq. 9), right-preconditioned by the
 * physics-based field-block preconditioner (section 2.5.2).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every array argument is a DEVICE pointer owned by the caller, allocated on the
 *   device that was current when the context was created.  Host-side structs
 *   (options, info) are plain host memory owned by the caller.
 * - A state vector holds n_f fields, field-major and x fastest:
 *   index = ((f * nz + k) * ny + j) * nx + i.  2D problems have ny = 1 and fields
 *   (u, w, p', theta'); 3D problems fields (u, v, w, p', theta').  p' is the Exner
 *   perturbation c_p pi' and theta' the potential-temperature perturbation.
 *   Cell-centred grid x_i = (i + 1/2) dx; walls lie on the domain faces.
 * - Precision: JFNK_F64 arrays are double, JFNK_F32 arrays are float.  Reductions
 *   (norms, Arnoldi dot products) accumulate in FP64 in both cases; the Givens /
 *   least-squares step of GMRES is FP64.
 * - Calls enqueue work on the context's HIP stream.  Calls that must take a
 *   convergence decision (jfnk_gmres, jfnk_newton_step) synchronise that stream
 *   before they return; the others return without synchronising.
 * - A context is not thread safe; use one context per host thread.
 * - No entry point allocates device memory except jfnk_create and jfnk_net_init
 *   (both freed by jfnk_destroy).
 *
 * Return codes: JFNK_OK (0); JFNK_NOT_CONVERGED (1, soft: outputs hold the last
 * iterate and the info struct is filled); JFNK_ERR_ARG (-1, invalid argument:
 * null pointer, a dimension below 8, dt <= 0, m > max_m, unsupported option);
 * JFNK_ERR_HIP (-2, a HIP runtime error); JFNK_ERR_NONFINITE (-3, a residual or
 * Krylov norm is NaN or infinite).  jfnk_last_error() returns a message for the
 * last failing call on the calling thread.
 */
#ifndef JFNK_H
#define JFNK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    JFNK_OK = 0,
    JFNK_NOT_CONVERGED = 1,
    JFNK_ERR_ARG = -1,
    JFNK_ERR_HIP = -2,
    JFNK_ERR_NONFINITE = -3
};

typedef enum { JFNK_F64 = 0, JFNK_F32 = 1 } jfnk_dtype;
typedef enum { JFNK_PC_NONE = 0, JFNK_PC_PHYSICS = 1, JFNK_PC_LEARNED = 2 } jfnk_pc_kind;
/* STABLE: [R(u+eps v) - R(u)]/eps with every bilinear term expanded (equal to the
 *         literal quotient in exact arithmetic, no cancellation);
 * LITERAL: the quotient evaluated as written;  ANALYTIC: the eps -> 0 limit.   */
typedef enum { JFNK_JV_STABLE = 0, JFNK_JV_LITERAL = 1, JFNK_JV_ANALYTIC = 2 } jfnk_jv_mode;
/* Gram-Schmidt form of the Arnoldi step of jfnk_gmres (the GMRES of Saad and
 * Schultz that section 2.5.1 relies on; the paper does not fix the form).
 * CGS2: classical Gram-Schmidt applied twice, three passes over the basis and
 *       three reductions per iteration.
 * ONE_REDUCTION: the second projection and the normalization of each basis
 *       vector are delayed to the next iteration, whose single reduction
 *       provides them (two passes over the basis per iteration); a column of
 *       the Hessenberg matrix is final one iteration later.  Equal to CGS2 in
 *       exact arithmetic.  Used when m < 32 and the vectors hold fewer than
 *       2^30 values (for the ensemble: m < 32); CGS2 otherwise.               */
typedef enum { JFNK_ORTHO_CGS2 = 0, JFNK_ORTHO_ONE_REDUCTION = 1 } jfnk_ortho;
typedef enum {
    JFNK_CLOSURE_CONST_K = 0,
    JFNK_CLOSURE_SMAGORINSKY = 1,
    JFNK_CLOSURE_NONE = 2,
    JFNK_CLOSURE_DEARDORFF = 3
} jfnk_closure;
typedef enum { JFNK_BC_FREE_SLIP = 0, JFNK_BC_NO_SLIP_BOTTOM = 1, JFNK_BC_PERIODIC = 2 } jfnk_bc;

/* Physical problem (equations 1-3 with the constants of section 2.1).
 * Background: theta_bar = theta0 + beta z with beta = n_bv^2 theta0 / g, Exner
 * background p_bar with dp_bar/dz = -g/theta_bar and p_bar(0) = cp.  kappa_div is
 * the coefficient of (p_bar + p') div u in the Exner equation (<= 0: R/cv).
 * Closure (section 2.4): Smagorinsky nu = (cs Delta)^2 sqrt(2 S:S), Delta the
 * geometric mean spacing, heat diffusivity nu/pr_t; or constant k_m, k_h; or
 * the anisotropic coefficients of Eq. 7:
 * K_m = cs^(4/3) eps^(1/3) (dx dy)^(2/3), K_M = cs^(4/3) eps^(1/3) dz^(4/3) with
 * eps = nu S:S, K_h = (1 + 2l/sqrt(dx dy)) K_m, K_H = (1 + 2l/dz) K_M (dy = dx in
 * 2D), the mixing length
 * l = min(0.75 sqrt(2e) / n_bv, Delta) with e = (eps Delta)^(2/3) (l = Delta for
 * n_bv = 0); the vertical coefficient carries every stress component with a z
 * index and the vertical heat flux.
 * Surface heat flux (section 3.2): h0 [W m^-2] over a strip of width strip_width
 * centred at x = strip_center, top-hat (strip_shape 0) or tanh profile (1, with
 * half-width units and steepness strip_xi); converted with rho0 = p_ref/(R theta0)
 * to Q = H/(rho0 cp) and applied as Q/dz in the lowest cell.
 * convection = 0 drops the convective terms; energy_test = 1 replaces
 * kappa (p_bar + p') by kappa cp and drops w dp_bar/dz (a frozen-coefficient
 * operator that conserves a quadratic energy).  dd_p is the order parameter of
 * the Deslauriers-Dubuc derivative (section 2.3): 2 (5 points) or, outside a
 * batch, 3 (9 points; halos twice as deep).                                     */
typedef struct {
    int32_t dim, nx, ny, nz;          /* 2 or 3; grid points per direction (ny = 1 in 2D) */
    double lx, ly, lz, dt;            /* domain [m], time step [s]                       */
    double theta0, g, cp, cv, rgas, p_ref;
    double kappa_div;
    double n_bv;
    int32_t closure;                  /* jfnk_closure */
    double cs, pr_t, k_m, k_h;
    int32_t bc_lateral;               /* JFNK_BC_FREE_SLIP or JFNK_BC_PERIODIC */
    int32_t bc_vertical;              /* jfnk_bc */
    double h0, strip_width, strip_center;
    int32_t strip_shape;
    double strip_xi;
    int32_t convection;
    int32_t energy_test;
    int32_t dd_p;
} jfnk_problem;

typedef struct {
    int32_t m;                 /* restart length (<= max_m of the context)              */
    int32_t max_restarts;      /* total iterations <= m * max_restarts                   */
    double tol;                /* stop when the least-squares residual <= tol * ||rhs||  */
    int32_t pc;                /* jfnk_pc_kind                                           */
    int32_t jv;                /* jfnk_jv_mode                                           */
    int32_t sweeps;            /* physics preconditioner Jacobi sweeps (>= 0)            */
    int32_t max_iters;         /* hard cap on iterations (<= 0: m * max_restarts)        */
    int32_t ortho;             /* jfnk_ortho: Gram-Schmidt form of the Arnoldi step      */
    int32_t no_judge;          /* 1: a learned-preconditioner solve is not judged by the
                                  physics-based one (it runs to its iteration budget and
                                  falls back only when it does not converge); 2: nor does
                                  it fall back (x and info are the learned solve's, e.g.
                                  after a fixed iteration count)                         */
} jfnk_gmres_opts;

typedef struct {
    int32_t iters, restarts, converged;
    double res0, res_est;
    double* h_out;             /* optional HOST buffer of (m+1)*m doubles, row-major:
                                  receives the Hessenberg of the last cycle before the
                                  Givens rotations (NULL: not returned)                  */
    int32_t fallback;          /* 1: the physics-based preconditioner produced x although
                                  the learned one was asked for (see jfnk_gmres)         */
    double res_true;           /* ||rhs - J x|| of the returned x (jfnk_gmres only; -1
                                  where not computed)                                    */
} jfnk_gmres_info;

typedef struct {
    double rtol;               /* stop when ||R|| <= max(rtol ||R(u0)||, atol)           */
    double atol_factor;        /* atol = atol_factor * ||2 u^n / dt||                     */
    int32_t max_newton;
    int32_t inner;             /* jfnk_dtype of the Krylov solve and Jv (F32 = mixed)     */
    jfnk_gmres_opts gm;        /* gm.tol is ignored: the forcing term sets it            */
    int32_t forcing;           /* 0: Eisenstat-Walker choice 2, 1: fixed eta            */
    double eta;                /* fixed forcing term                                     */
    double eta_floor;          /* lower bound on the forcing term                        */
    float* rec_r;              /* optional DEVICE buffers of rec_cap FP32 state vectors:  */
    float* rec_du;             /* the rhs -R and Krylov solution du of each Newton       */
    int32_t rec_cap;           /* iteration are appended (training pairs of the learned  */
    int32_t* rec_count;        /* preconditioner); rec_count (HOST) counts them.  NULL /  */
                               /* 0 disables recording.                                   */
    int32_t rec_krylov;        /* 1: record instead, for every FGMRES iteration of an FP32 */
                               /* solve, the pair (J z_j, z_j) of a preconditioned Krylov */
                               /* direction z_j and its image                             */
} jfnk_newton_opts;

typedef struct {
    int32_t newton_iters, gmres_iters_total, converged, fallbacks;
    double res0, res_final;
} jfnk_newton_info;

typedef struct jfnk_ctx jfnk_ctx;

/* Create a context for one problem on the current HIP device.  hip_stream is a
 * hipStream_t (NULL: the null stream).  max_m bounds the GMRES restart length;
 * the workspace (Krylov bases V and Z of max_m+1 vectors in both precisions,
 * temporaries, background profiles) is allocated here, sized for the grid.
 * Sets up the background state and surface flux (section 2.1, section 3.2).      */
int jfnk_create(const jfnk_problem* prob, int32_t max_m, void* hip_stream, jfnk_ctx** out);
int jfnk_destroy(jfnk_ctx* ctx);
const char* jfnk_last_error(void);
/* Rebind the stream a context enqueues on.                                       */
int jfnk_set_stream(jfnk_ctx* ctx, void* hip_stream);

/* f = 2 u^n / dt + F(u^n)   (equation 5, right-hand side).  FP64.               */
int jfnk_rhs(jfnk_ctx* ctx, const double* u_n, double* f);

/* R = 2 u / dt - F(u) - f   (sections 2.5 and 2.5.1, R = L(u) - f).  FP64.  f may be NULL
 * (treated as zero).                                                             */
int jfnk_residual(jfnk_ctx* ctx, const double* u, const double* f, double* R);

/* Same operators in either precision: out = F(u) (what = 0), 2u/dt + F(u)
 * (what = 1) or 2u/dt - F(u) - f (what = 2).                                      */
int jfnk_apply_F(jfnk_ctx* ctx, jfnk_dtype dt, int32_t what, const void* u, const void* f, void* out);

/* Jv = J(u) v, the Frechet derivative of R at u in direction v (equation 9).
 * eps <= 0 selects eps = sqrt(eps_mach) max(||u||, sqrt(N)) / ||v|| with eps_mach
 * of the dtype (2^-52 or 2^-23); ignored by ANALYTIC.  u, v, Jv share the dtype.
 * v = 0 gives Jv = 0 in every mode.                                              */
int jfnk_jv(jfnk_ctx* ctx, jfnk_dtype dt, jfnk_jv_mode mode, const void* u, const void* v,
            double eps, void* Jv);

/* z ~ P(u)^{-1} r, the physics-based preconditioner (section 2.5.2): field-block
 * diagonal of L with u frozen, 2/dt + C(u; .) - D.(K D .), applied by Jacobi
 * sweeps (z0 = r/d, z <- z + (r - P z)/d).  JFNK_PC_NONE copies r.  u, r, z share
 * the dtype; r and z must not alias.                                             */
int jfnk_precond_apply(jfnk_ctx* ctx, jfnk_pc_kind pc, jfnk_dtype dt, const void* u,
                       const void* r, void* z, int32_t sweeps);

/* Right-preconditioned flexible restarted GMRES(m) (Saad and Schultz) for
 * J(u) x = rhs with x0 = 0, the Arnoldi step of o->ortho (jfnk_ortho), Givens
 * rotations and back substitution in FP64.  x is output only.  info->res_true
 * receives the true residual of x (one more Jv).
 * The learned preconditioner (FP32 only, parameters set) is judged by the
 * physics-based one (section 2.5.2): it runs only when a physics-preconditioned
 * solve of this context is on record and stops at the end of the first cycle
 * whose mean log residual reduction per iteration falls short of that solve's;
 * the system is then solved with the physics-based preconditioner, as it is when
 * no record exists or the learned solve does not converge or breaks down (a
 * non-finite Krylov vector or solution) (info->fallback = 1).  Every converged
 * physics-preconditioned solve (here or inside jfnk_newton_step) updates the
 * record.                                                                         */
int jfnk_gmres(jfnk_ctx* ctx, jfnk_dtype dt, const void* u, const void* rhs, void* x,
               const jfnk_gmres_opts* opts, jfnk_gmres_info* info);

/* One trapezoidal step by inexact Newton (equation 8): u_np1 holds the initial
 * guess on entry (usually a copy of u_n) and the solution on return.  FP64 outer
 * residual, update and norms; inner Krylov solve in opts->inner, each judged as in
 * jfnk_gmres when the learned preconditioner is asked for; after a solve in which
 * the learned preconditioner fell back, the remaining solves of the step use the
 * physics-based one (info->fallbacks counts the solves it took over; the learned
 * attempts' iterations count in gmres_iters_total).                               */
int jfnk_newton_step(jfnk_ctx* ctx, const double* u_n, double* u_np1,
                     const jfnk_newton_opts* opts, jfnk_newton_info* info);

/* 2-norm of a vector of n values (FP64 accumulation), result to a host double.   */
int jfnk_norm(jfnk_ctx* ctx, jfnk_dtype dt, const void* x, int64_t n, double* out);

/* Autotuner: times every compiled tile shape (64 x 4, 64 x 8, 64 x 16 points)
 * of the residual, Jv and preconditioner-sweep kernels, and the row-marching
 * residual and Jv (a 64-column strip walking down 32, 64 or 256 rows), in both
 * precisions on this context's grid (HIP events: one warm-up launch, then the
 * fastest of three groups of five timed launches, on a deterministic non-zero
 * fill of the Krylov workspace) and
 * keeps the fastest for the context (near-ties within 3% go to the 64 x 8 tile,
 * then to the lowest variant); tile_rows (HOST, 6
 * entries, may be NULL) receives the rows per workgroup of the choices (4, 8,
 * 16: tiles; 32, 64, 256: marching) for (F64 residual, F32 residual, F64 Jv,
 * F32 Jv, F64 sweep, F32 sweep).  Overwrites the Krylov workspace; synchronises. */
int jfnk_tune(jfnk_ctx* ctx, int32_t* tile_rows);

/* Pins the launch shape of one stencil stage (what the autotuner would choose):
 * stage 0 residual / F, 1 Jv, 2 preconditioner sweep; dtype JFNK_F64 or
 * JFNK_F32; variant 0, 1, 2 = tiles of 64 x 4, 64 x 8, 64 x 16 points, 3, 4, 5 =
 * row marching over 32, 64, 256 rows (residual and Jv only).  The FP64 Jv has
 * no 64 x 16 tile (its LDS would exceed a CU's).  3D contexts take only the
 * FP32 Jv (stage 1): variant 7 = one z-marching launch that keeps the stress and
 * heat-flux differences in LDS and registers (the default), 6 = two launches
 * with those differences in an HBM buffer between them.
 * Returns JFNK_ERR_ARG for anything else.                                       */
int jfnk_set_variant(jfnk_ctx* ctx, int32_t stage, int32_t dtype, int32_t variant);

/* Kernel timing with HIP events recorded on the context stream around each
 * launch (resolved lazily, no synchronisation per launch).  Kernel classes:
 * 0 Jv, 1 residual/rhs, 2 physics preconditioner (diagonal start and sweeps),
 * 3 Arnoldi (the three Gram-Schmidt passes of one iteration with their
 * finishing reductions and the Givens step), 4 other, 5 learned preconditioner
 * (network application).  enable != 0 starts recording and clears the counters:
 * a bit mask of the classes recorded (bit k: class k; -1 all), 0 stops.
 * bytes receives the algorithmic HBM bytes of the recorded launches (each array
 * element moved once per launch); for class 5 it receives the algorithmic flops
 * (2 per weight and grid point) instead.                                        */
int jfnk_timing_enable(jfnk_ctx* ctx, int32_t enable);
int jfnk_timing_read(jfnk_ctx* ctx, int32_t kernel_class, double* total_ms, int64_t* launches,
                     double* bytes);

/* ---- nonlinear physics-based preconditioning (section 2.5.2) ----------------
 * The preconditioned system R~(u) = u - P^{-1}(u)[f - L(u) + P(u)u], with the
 * preconditioning operator acting on u inside the bracket, is
 * R~(u) = P^{-1}(u) R(u): P^{-1}(u) is the physics-based field-block
 * preconditioner of jfnk_precond_apply with its coefficients frozen at u
 * (`sweeps` Jacobi sweeps).  Its roots are those of R.  FP64, 2D and 3D.       */
/* out = R~(u) for the right-hand side f (DEVICE FP64 state vectors; out must not
 * alias u or f).                                                                */
int jfnk_nlpc_residual(jfnk_ctx* ctx, const double* u, const double* f, double* out, int32_t sweeps);
/* One trapezoidal step on the preconditioned system: method 0 the fixed-point
 * iteration u <- u - R~(u) (at most o->max_newton iterations); method 1 inexact
 * Newton-GMRES on R~ without further preconditioning, Jacobian-vector products
 * [R~(u + eps v) - R~(u)]/eps (eps as for jfnk_jv), Eisenstat-Walker forcing on
 * ||R~|| (o->forcing = 0) or fixed o->eta.  Options used: rtol, atol_factor,
 * max_newton, forcing, eta, eta_floor, gm.m, gm.max_restarts, gm.sweeps.  Both
 * stop on the unpreconditioned residual, ||R(u)|| <= max(rtol ||R(u^n)||,
 * atol_factor ||2u^n/dt||).  u_np1 holds the initial guess on entry.  Returns
 * JFNK_NOT_CONVERGED (soft) when the iteration limit is reached.                */
int jfnk_nlpc_step(jfnk_ctx* ctx, const double* u_n, double* u_np1, const jfnk_newton_opts* o, int32_t method,
                   jfnk_newton_info* info);

/* ---- learned right preconditioner ------------------------------------------
 * z = (dt/2) r + s N(r / s), s the RMS of r over all fields and points (1 for
 * r = 0), N = conv(n_f->16) GELU conv(16->16) GELU conv(16->16) GELU
 * conv(16->n_f), zero padding, exact (erf) GELU.  2D: 3x3 kernels with a
 * dilation d_l per layer (taps at d_l (-1, 0, 1); dilations 1, 2, 4, 8 give a
 * dense 31 x 31 receptive field).  3D: 3x3x3 kernels, dilation 1.  An approximate
 * inverse of J in the spirit of the paper's cheap preconditioners (section 2.5.2);
 * nonlinear in r, hence used inside the flexible GMRES.  Parameters: one flat
 * FP32 vector, per layer W[co][ci][kz][kx] (2D) or W[co][ci][kz][ky][kx] (3D),
 * tap offset (kz-1, ...), then b[co].
 * Inference (JFNK_PC_LEARNED, jfnk_net_apply with bf16 = 1) runs in BF16 on the
 * matrix cores with FP32 accumulation; training in FP32 with FP32 Adam moments.
 * Vectors r, z, du are FP32 device arrays in the state layout.                  */
/* Allocate the network workspace (the only allocating call besides
 * jfnk_create) and set the per-layer dilations (HOST, 4 entries in [1, 8], NULL:
 * all 1; 3D problems accept only 1); n_params receives the parameter count.     */
int jfnk_net_init(jfnk_ctx* ctx, const int32_t* dilations, int64_t* n_params);
/* Copy FP32 parameters from / to HOST memory (n must equal the count); setting
 * resets the Adam state.                                                         */
int jfnk_net_set_params(jfnk_ctx* ctx, const float* theta_host, int64_t n);
int jfnk_net_get_params(jfnk_ctx* ctx, float* theta_host, int64_t n);
/* z = learned preconditioner applied to r; bf16 = 1: BF16 MFMA, 0: FP32.       */
int jfnk_net_apply(jfnk_ctx* ctx, int32_t bf16, const float* r, float* z);
/* Training loss of a pair (r, du) with J du = r:
 *   JFNK_NET_LOSS_SOLUTION        ||z(r) - du||^2 / ||du||^2 (default)
 *   JFNK_NET_LOSS_REST_JACOBIAN   ||J0 (z(r) - du)||^2 / ||J0 du||^2, J0 the
 *       Jacobian of R (eq. 5) at the state of rest with the closure off: the
 *       acoustic-gravity terms of eqs. 1-3 about the hydrostatic background.  It
 *       weighs the error as the residual J z - r that right-preconditioned GMRES
 *       sees; its gradient uses the exact transpose of J0 (with mirror walls the
 *       transpose of a derivative is minus the derivative of the opposite
 *       parity).  Needs energy_test = 0.  Errors: JFNK_ERR_ARG.                   */
typedef enum { JFNK_NET_LOSS_SOLUTION = 0, JFNK_NET_LOSS_REST_JACOBIAN = 1 } jfnk_net_loss;
int jfnk_net_set_loss(jfnk_ctx* ctx, int32_t kind);
/* Mean over a batch of pairs (r_b, du_b) (batch consecutive state vectors) of the
 * selected loss (to a host double) and its gradient (to a HOST float array of
 * n_params, or NULL), FP32 forward and backward.  A pair with du = 0 (nothing
 * to be relative to) contributes zero loss and gradient.                        */
int jfnk_net_loss_grad(jfnk_ctx* ctx, const float* r, const float* du, int32_t batch, double* loss,
                       float* grad_host);
/* One Adam step (beta 0.9 / 0.999, eps 1e-8) with learning rate lr on that loss;
 * loss receives the loss before the step (host double, may be NULL).
 * crop_dims (HOST, 3 entries nx, ny, nz, or NULL for the context's grid): the
 * pairs are crops of that size, each vector [n_f][nz][ny][nx] (a convolution does
 * not depend on the domain it slides over, so a network trained on crops applies
 * to the full grid); every entry must be within the context's grid (ny = 1 in
 * 2D) and at least 1, and crops take the solution-space loss only.  Errors:
 * JFNK_ERR_ARG.                                                                  */
int jfnk_net_train_step(jfnk_ctx* ctx, const float* r, const float* du, int32_t batch, const int32_t* crop_dims,
                        float lr, double* loss);

/* ---- batched ensemble (2D) ------------------------------------------------
 * Independent problems of uneven grid sizes solved together: every stage of the
 * Newton-Krylov iteration (residual, preconditioner, Jv, Gram-Schmidt passes,
 * Givens step) is one launch over all instances, instances that have converged
 * drop out through a device mask.  Batch state vectors hold the instances'
 * vectors back to back (instance i at element offsets[i], each in the layout of a
 * single problem).  The inner solve is FP32 FGMRES with the physics-based (or no)
 * preconditioner; the Newton residual, update and norms are FP64.              */
typedef struct jfnk_batch jfnk_batch;
/* Allocates the batch workspace for ninst problems (host array): 2D problems with
 * nx, nz >= 8 and one order parameter dd_p (2 or 3, section 2.3) for all of
 * them.  Errors: JFNK_ERR_ARG.                                                   */
int jfnk_batch_create(const jfnk_problem* probs, int32_t ninst, int32_t max_m, void* hip_stream,
                      jfnk_batch** out);
int jfnk_batch_destroy(jfnk_batch* batch);
/* total: elements of a batch state vector; offsets (HOST, ninst + 1, or NULL).   */
int jfnk_batch_size(jfnk_batch* batch, int64_t* total, int64_t* offsets);
/* F / rhs / residual of every instance (what as in jfnk_apply_F), FP64.          */
int jfnk_batch_apply_F(jfnk_batch* batch, int32_t what, const double* u, const double* f, double* out);
/* One trapezoidal step of every instance (opts->inner must be JFNK_F32; the
 * recording fields are ignored; opts->gm.ortho selects the Arnoldi step as in
 * jfnk_gmres); infos: HOST array of ninst results.
 * use_graph = 1 keeps every decision of a restart cycle on the device (per
 * instance: which instances work, their iteration counts, convergence against
 * the forcing term, the columns of the least-squares update, who restarts) and
 * replays each cycle as one captured HIP graph, captured on the first call (and
 * again when m, the sweeps, the preconditioner, the Gram-Schmidt form or the
 * iteration limit change); the host waits once per cycle instead of twice per
 * Krylov iteration.  use_graph = 0 takes those decisions on the host.  Both give
 * the same results.                                                             */
int jfnk_batch_newton_step(jfnk_batch* batch, const double* u_n, double* u_np1, const jfnk_newton_opts* opts,
                           jfnk_newton_info* infos, int32_t use_graph);
/* Autotuner of the batched residual, Jv and sweep kernels (tile heights 4, 8,
 * 16); tile_rows (HOST, 3 entries, may be NULL) receives the choices.           */
int jfnk_batch_tune(jfnk_batch* batch, int32_t* tile_rows);

/* ---- Jv without a context, allocating nothing -------------------------------
 * For callers that cannot allocate device memory: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc.  The same product as
 * jfnk_jv (STABLE or ANALYTIC mode, the context-free default launch shape) for
 * the problem *prob, enqueued on hip_stream (NULL: the null stream) without
 * creating a context: u, v and Jv are the caller's device arrays; the
 * background profiles and the reductions of the automatic step (eps <= 0) use
 * a fixed per-GPU array of the library (about 115 KB, held until the process
 * ends) and no call allocates or frees memory.  Limits: nz <= 4096; 3D problems
 * in FP32 with dd_p = 2 only.  Every call on a GPU shares that GPU's array, so
 * calls that overlap on one GPU (other streams or host threads) race; calls
 * enqueued on one stream are ordered.  Errors: JFNK_ERR_ARG (invalid argument
 * or a limit exceeded), JFNK_ERR_HIP.                                          */
int jfnk_jv_noalloc(const jfnk_problem* prob, jfnk_dtype dt, jfnk_jv_mode mode, const void* u, const void* v,
                    double eps, void* Jv, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* JFNK_H */
