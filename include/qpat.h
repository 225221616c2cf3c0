/*
 * qpat.h -- C ABI of libqpat, the MI355X (gfx950) implementation of the
 * matrix-free Jacobian / priorconditioned-LSQR path of
 *
 *   A. Hannukainen, N. Hyvonen, H. Majander, T. Tarvainen, "Efficient
 *   inclusion of total variation type priors in quantitative photoacoustic
 *   tomography" (SIAM J. Imaging Sci. 2016; arXiv:1512.02796).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - All array arguments are caller-owned, contiguous DEVICE pointers (for
 *   example a torch tensor's data_ptr() on the GPU the context was created
 *   on). The library never frees them and keeps none of them after the call
 *   returns, except `beta_out` of qpat_lsqr_init (see there).
 * - Floating-point arrays are IEEE double (FP64) unless stated otherwise;
 *   index arrays are int32, zero-based.
 * - "[n][m]" means row-major with m fastest.
 * - All device work is enqueued on the HIP stream given to qpat_setup_mesh.
 *   Calls that return host-visible numbers (qpat_info, resnorm_out, status of
 *   iterative solves) synchronise that stream before returning.
 * - Errors never throw across the ABI. Every entry point returns a
 *   qpat_status; qpat_last_error() returns the message of the last failure.
 * - A context is not thread-safe; calls on one context must be serialised.
 *
 * Units: lengths in mm, kappa in mm, mu in 1/mm (Sec. 5).
 */
#ifndef QPAT_H
#define QPAT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qpat_ctx qpat_ctx;

typedef enum {
    QPAT_OK = 0,
    QPAT_ERR_ARG = 1,        /* null pointer, bad size, non-finite or non-positive input   */
    QPAT_ERR_MESH = 2,       /* index out of range, degenerate tetrahedron, row too long    */
    QPAT_ERR_NOCONV = 3,     /* a PCG solve hit pcg_maxit; outputs hold the last iterate   */
    QPAT_ERR_BREAKDOWN = 4,  /* LSQR: p.r <= 0 or non-finite inside a step                  */
    QPAT_ERR_DEVICE = 5,     /* a HIP runtime call failed                                   */
    QPAT_ERR_OOM = 6,        /* device allocation failed                                    */
    QPAT_ERR_STATE = 7       /* call order violated (e.g. qpat_jvp before qpat_forward)     */
} qpat_status;

typedef struct {
    int32_t precision;      /* K solves. 0: FP64 PCG (iterate, residual, direction, operator,
                               dot products). 1: mixed. On the multigrid path's LDS-tiled
                               kernels (lattice meshes, blocks of 16 right-hand sides) the
                               search direction p is stored in FP32; x, r, q = A p (FP64
                               operator), the dot products and the true-residual check stay
                               FP64, and x and r are both updated with the stored p, so the
                               solves meet the same FP64 stopping rule (other multigrid
                               blocks run FP64). On the Jacobi-PCG path (pcg_precond = 0, or
                               meshes without a lattice) the operator, the Jacobi diagonal
                               and the PCG vectors are FP32, with FP64 dot products, FP64
                               true-residual recomputation (reliable updates) and an FP64
                               iterate. In both modes the multigrid V-cycle keeps parts of its
                               own work in FP32 (the finest residual it restricts and, on the
                               tiled path, the last sweep's rows and its output z). M_delta
                               solves and LSQR are FP64 in both modes.                      */
    int32_t max_rhs_block;  /* right-hand sides per block PCG (1, 2, 4, 8 or 16). 1 solves the
                               illuminations one after another ("plain").                    */
    double  pcg_rtol;       /* K solves stop when ||b - K x||_2 <= pcg_rtol ||b||_2 (true
                               residual, FP64).                                                */
    int32_t pcg_maxit;      /* iteration cap per solve -> QPAT_ERR_NOCONV.                    */
    double  prior_rtol;     /* same rule for M_delta solves (default 1e-8). The FP64 result's
                               own rounding bounds the attainable relative residual by about
                               eps ||M_delta|| ||x|| / ||p||, which depends on the problem:
                               on the 128^3 phantom a random p reaches 1e-11 and an LSQR
                               direction stalls near 1.2e-10; on one of the batched 24^3 -
                               96^3 instances a direction stalls at 1.3e-9.                 */
    int32_t prior_deflate;  /* 1: the constant vector of each block (the delta-eigenvector of
                               M_delta) is solved exactly and PCG runs on its complement.    */
    int32_t lsqr_reorth;    /* 1: full reorthogonalisation of both bidiagonalisation bases.
                               0: plain Paige-Saunders recurrences.                           */
    int32_t lsqr_max_steps; /* initial capacity (steps) of the stored bases when lsqr_reorth = 1;
                               a run that fills them doubles the capacity, or -- when the
                               device cannot hold more -- continues with the plain
                               recurrences (qpat_lsqr_basis then reports 0).             */
    double  ru_delta;       /* mixed precision: recompute the FP64 residual whenever the
                               recursive one fell by this factor since the last recompute.   */
    int32_t use_graphs;     /* 1: replay chunks of PCG iterations as captured HIP graphs.     */
    int32_t operator_format;/* 1: on meshes whose node numbering is a lattice (x fastest, every
                               matrix neighbour at most one lattice step away per axis, e.g.
                               the Kuhn voxel meshes of Sec. 5) the PCG products use the
                               stencil form (diagonal + upper offsets, LDS-tiled).
                               0: sliced ELL on every mesh. Same results up to rounding.     */
    int32_t prior_precond;  /* M_delta solves: 1 = PCG with a geometric multigrid V-cycle
                               (lattice meshes with the stencil form; otherwise Jacobi),
                               0 = Jacobi-PCG. Same stopping rule either way.               */
    int32_t pcg_precond;    /* K solves: 1 = PCG with a geometric multigrid V-cycle (lattice
                               meshes with the stencil form; elsewhere Jacobi-PCG); 0 =
                               Jacobi-PCG. `precision` selects the arithmetic of either.
                               Same stopping rule either way.                                */
    int32_t autotune;       /* 1 (default): the z-chunk length of the LDS-tiled finest-level
                               kernels of the multigrid K solves (the PCG direction, update
                               and residual tiles; the fused prolongation + last sweep) is
                               chosen by timing the cost model's lowest-cost candidates on the
                               device at the first solve of a lattice size and block width,
                               and cached for the process. 0: the cost model's choice. The
                               results agree up to the order of the partial sums.            */
} qpat_opts;

/* Solve report of a call (host struct). The first five fields are outputs.
 * The last three are inputs that the call only reads: host arrays of rhs_cap
 * entries that receive, for every linear system the call solved (one per
 * right-hand side, block by block in the order solved; the padding columns
 * of a block of illuminations included, with zero right-hand sides, 0
 * iterations and residual 0), its PCG iteration count and its final true
 * relative residual ||b - A x|| / ||b||. Entries past rhs_cap are dropped;
 * rhs_cap = 0 or NULL arrays ask for none. Zero-initialise the struct when
 * the per-system arrays are not wanted. */
typedef struct {
    int32_t n_solves;       /* linear systems solved by the call                               */
    int32_t iters_max;      /* largest PCG iteration count among them                          */
    int64_t iters_sum;      /* total PCG iterations                                            */
    int32_t updates;        /* FP64 true-residual recomputations (multigrid PCG: restarts     */
                            /* after a failed true-residual check, summed over the systems) */
    double  relres_max;     /* largest final true relative residual                           */
    int32_t rhs_cap;        /* in: capacity of rhs_iters / rhs_relres                          */
    int32_t* rhs_iters;     /* in: host array [rhs_cap] or NULL                                */
    double* rhs_relres;     /* in: host array [rhs_cap] or NULL                                */
} qpat_info;

/* Fill *opts with the defaults: FP64, block 16, rtol 1e-10, maxit 20000,
 * prior_rtol 1e-8, deflation on, reorthogonalisation on with 64 steps,
 * ru_delta 1e-3, graphs on, stencil form on lattice meshes, multigrid for M_delta
 * and K, autotuned tile schedules. */
void qpat_default_opts(qpat_opts* opts);

/* Create a context for a tetrahedral P1 mesh (Sec. 3: piecewise linear
 * basis on a tetrahedral partition; Sec. 5 / Appendix: the FEM system).
 *   N, coords  : nodes, [N][3] FP64 (device).
 *   E, tets    : tetrahedra, [E][4] int32 (device). Either orientation.
 *   F_b, bfaces: boundary triangles, [F_b][3] int32 (device); they carry the
 *                Robin term and the sources.
 *   opts       : NULL for the defaults.
 *   hip_stream : hipStream_t used for all work of this context (NULL = default).
 * Builds on the device: tetrahedron volumes and barycentric gradients,
 * node->element adjacency, the sparsity pattern of K (sorted rows, sliced-ELL
 * layout of 64-row slices) and boundary-triangle areas.
 * Errors: QPAT_ERR_ARG (N < 4, E < 1, null), QPAT_ERR_MESH (index out of
 * range, zero-volume tetrahedron, a row with more than 64 entries). */
qpat_status qpat_setup_mesh(qpat_ctx** ctx, int64_t N, const double* coords,
                            int64_t E, const int32_t* tets,
                            int64_t F_b, const int32_t* bfaces,
                            const qpat_opts* opts, void* hip_stream);

qpat_status qpat_set_opts(qpat_ctx* ctx, const qpat_opts* opts);
qpat_status qpat_get_opts(const qpat_ctx* ctx, qpat_opts* opts);

/* Boundary photon fluxes Phi^(k), k < n_ill (Sec. 2 eq. (2.1); several
 * illuminations: Sec. 4, paragraph after Algorithm 1). phi_src is
 * [n_ill][F_b][3] FP64 (device): Phi at the three vertices of each boundary
 * triangle, linear in between. Computes the load vectors
 * f_k = 2 int Phi_k v dS (Appendix, weak form). 1 <= n_ill <= 64. */
qpat_status qpat_set_sources(qpat_ctx* ctx, int32_t n_ill, const double* phi_src);

/* Linearisation point and forward map (Sec. 2 eqs. (2.1)-(2.2); Appendix).
 * kappa, mu: nodal [N] (device), > 0. Assembles K(kappa, mu) = S(kappa) +
 * Mass(mu) + B/2 with kappa, mu entering as P1 interpolants, solves
 * K phi_k = f_k for every illumination and keeps phi inside the context.
 * phi_out, h_out: [n_ill][N] (device) or NULL; h = mu * phi (nodal product).
 * info: host struct or NULL. */
qpat_status qpat_forward(qpat_ctx* ctx, const double* kappa, const double* mu,
                         double* phi_out, double* h_out, qpat_info* info);

/* Same as qpat_forward at kappa = kappa0 exp(kt), mu = mu0 exp(mt), with
 * beta = [kt; mt] of length 2N (device) (Sec. 3 eq. (3.1)). */
qpat_status qpat_forward_log(qpat_ctx* ctx, double kappa0, double mu0, const double* beta,
                             double* phi_out, double* h_out, qpat_info* info);

/* J s at the last forward point, J the Jacobian of beta -> h w.r.t. the
 * log-parameters (Appendix, formula for J s):
 *   J s = diag(mu) K^{-1} (G1 diag(kappa) s1 + G2 diag(mu) s2) + diag(phi) diag(mu) s2,
 * with G1, G2 applied element by element, never formed.
 * s: [2N] = [s_kt; s_mt] (device). out: [n_ill][N] (device). */
qpat_status qpat_jvp(qpat_ctx* ctx, const double* s, double* out, qpat_info* info);

/* J^T t (Appendix, formula for the transpose): t [n_ill][N] (device),
 * out [2N] (device). */
qpat_status qpat_vjp(qpat_ctx* ctx, const double* t, double* out, qpat_info* info);

/* Lagged-diffusivity Perona-Malik prior (Sec. 3 eq. (3.7); Sec. 4 eqs. (4.3),
 * (4.5), (4.8)): c_T = 1 / (1 + |grad u_T|^2 / T^2) per tetrahedron,
 * M(u) = FEM matrix of -div(c_u grad), M_delta = blockdiag(M(kt),
 * b_over_a M(mt)) + delta I. kt, mt: [N] (device). T, delta > 0. */
qpat_status qpat_prior_setup(qpat_ctx* ctx, const double* kt, const double* mt,
                             double T, double b_over_a, double delta);

/* The same prior with another choice of r in R(u) = int r(|grad u|) (Sec. 3,
 * eq. (3.6) and the remark after eq. (3.7) that smoothed TV and TV^q fit the
 * algorithm unchanged; Sec. 4 eq. (4.3): c_u = r'(|grad u|) / |grad u|).
 *   kind QPAT_PRIOR_PM  : Perona-Malik, exactly qpat_prior_setup (q ignored).
 *   kind QPAT_PRIOR_TVQ : r(t) = T^(2-q) (t^2 + T^2)^(q/2) / q, so
 *                         c_T = (1 + |grad u_T|^2 / T^2)^((q-2)/2); q = 1 is
 *                         smoothed total variation, q = 2 the plain Laplacian.
 *                         The factor T^(2-q) gives c(0) = 1 as for
 *                         Perona-Malik; a constant factor of r is absorbed in
 *                         the prior weights a, b. Needs 0 < q <= 2.
 * Other arguments and errors as qpat_prior_setup; an unknown kind or a q
 * outside (0, 2] returns QPAT_ERR_ARG before any device work. */
#define QPAT_PRIOR_PM 0
#define QPAT_PRIOR_TVQ 1
qpat_status qpat_prior_setup_r(qpat_ctx* ctx, const double* kt, const double* mt, int32_t kind,
                               double T, double q, double b_over_a, double delta);

/* y = M_delta x; x, y: [2N] (device). */
qpat_status qpat_prior_apply(qpat_ctx* ctx, const double* x, double* y);

/* r = M_delta^{-1} p by PCG (prior_rtol); p, r: [2N] (device). */
qpat_status qpat_prior_solve(qpat_ctx* ctx, const double* p, double* r, qpat_info* info);

/* Whitened nonlinear misfit ||W (chi - h)||_2 at the last forward point
 * (Algorithm 1, step 4). chi, w: [n_ill][N] (device), w = Gamma^{-1/2} as a
 * diagonal. The result is written to *out (host). */
qpat_status qpat_misfit(qpat_ctx* ctx, const double* chi, const double* w, double* out);

/* qpat_misfit for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * sum, but it calls no allocating routine and does not synchronise. The
 * partial sums go to a file-scope device array of 1024 doubles, one copy per
 * GPU, whose address qpat_setup_mesh looks up once per device; every size of
 * problem fits it (the reduction's grid is capped at 1024 blocks), so no size
 * is rejected. The result ||W (chi - h)||_2 is written to out_dev[0] (device,
 * 1 double) in stream order on the context's stream.
 * Every call on one GPU shares that array: calls that overlap on one GPU (two
 * contexts on different streams) race and may return wrong sums; serialise
 * them. Errors as qpat_misfit (QPAT_ERR_ARG null pointer, QPAT_ERR_STATE
 * before qpat_forward). */
qpat_status qpat_misfit_noalloc(qpat_ctx* ctx, const double* chi, const double* w, double* out_dev);

/* Initial guess of Algorithm 1 (preamble; several illuminations: Sec. 4 and
 * Sec. 5): call after qpat_forward at the homogeneous (kappa0, mu0).
 * beta_out[0:N] = 0, beta_out[N:2N] = log(mean_k(chi_k / phi_k) / mu0), the
 * ratio clamped below at 1e-12 mu0. chi: [n_ill][N]; beta_out: [2N] (device). */
qpat_status qpat_init_guess(qpat_ctx* ctx, const double* chi, double mu0, double* beta_out);

/* Background values of Algorithm 1's preamble: the homogeneous pair
 * (kappa0, mu0) minimising |W (chi - h(log(kappa) 1, log(mu) 1))| over
 * positive reals (W = Gamma^{-1/2} diagonal), by Gauss-Newton in
 * (log kappa, log mu) with the columns J [1; 0], J [0; 1] of the Jacobian at
 * the current homogeneous point (one forward solve and two J products per
 * iteration). Steps longer than 1 in either log are shortened to 1, then
 * halved up to 30 times until the misfit does not increase. Stops after maxit
 * iterations, when an accepted step is at most tol in both logs, or when no
 * halving decreases the misfit.
 *   chi, w       : [n_ill][N] (device).
 *   kappa0, mu0  : host in/out: the starting pair in, the fitted pair out
 *                  (unchanged, bit for bit, when no step is accepted).
 *   iters        : host out (may be NULL): Gauss-Newton iterations taken.
 * On return the context's forward state (phi, h) is at the fitted pair, so
 * qpat_init_guess may follow directly. Errors: QPAT_ERR_ARG (null pointer,
 * non-positive or non-finite start, maxit < 0, tol < 0), QPAT_ERR_STATE (no
 * sources), QPAT_ERR_NOCONV (a PCG solve), QPAT_ERR_BREAKDOWN (singular 2 x 2
 * normal matrix or an iterate whose exponential overflows). */
qpat_status qpat_fit_background(qpat_ctx* ctx, const double* chi, const double* w, double* kappa0,
                                double* mu0, int32_t maxit, double tol, int32_t* iters,
                                qpat_info* info);

/* Start priorconditioned LSQR (Sec. 4 eq. (4.10); Algorithm 1 steps 1 and 3)
 * at the last forward point with the last prior:
 *   A = W J, yt = W (chi - h + J beta_lin), iterate x = 0.
 * chi, w: [n_ill][N]; beta_lin: [2N] or NULL (then yt = W (chi - h)).
 * beta_out: [2N] device buffer that receives the iterate x (= beta, already
 * mapped back by L^{-1}); it stays registered and is updated in place by each
 * qpat_lsqr_step until the next qpat_lsqr_init or qpat_destroy. */
qpat_status qpat_lsqr_init(qpat_ctx* ctx, const double* chi, const double* w,
                           const double* beta_lin, double* beta_out, qpat_info* info);

/* The zeroth step of Sec. 5: the same priorconditioned LSQR for the diffusion
 * block alone, A = W J_kt (the first N columns of J), prior M_delta's kt
 * block M(kt) + delta I, yt = W (chi - h + J [beta_lin[0:N]; 0]). Arguments
 * as qpat_lsqr_init; beta_out[N:2N] stays 0. qpat_lsqr_step continues it. */
qpat_status qpat_lsqr_init_kappa(qpat_ctx* ctx, const double* chi, const double* w,
                                 const double* beta_lin, double* beta_out, qpat_info* info);

/* One LSQR step: one J v, one J^T u, one M_delta^{-1}, scalar recurrences in
 * FP64 on the device. *resnorm_out (host) = |phibar| = ||A x - yt|| in exact
 * arithmetic. A lucky breakdown (beta or alpha = 0) returns QPAT_OK and
 * freezes the iterate. */
qpat_status qpat_lsqr_step(qpat_ctx* ctx, double* resnorm_out, qpat_info* info);

/* Per-launch timing of the PCG iteration kernels, for roofline
 * measurements. While enabled, the solves run without graph replay and every
 * launch of the kernels below is bracketed by HIP events on the context's
 * stream and its duration accumulated (launches after every right-hand side
 * stopped are not counted). Jacobi-PCG: 0 K direction+SpMV, 1 K update,
 * 2 M_delta direction+SpMV, 3 M_delta update. Multigrid-PCG: 4 K direction
 * + product, 5 K update, 6 K finest-level residual (with the first sweep),
 * 7 K finest-level last sweep (with the dot products); 8-11 the same for
 * M_delta. Where one kernel does the update and the finest-level residual
 * (the LDS-tiled path of 8 or 16 right-hand sides), 5 counts it and 6 stays
 * empty; with 16 right-hand sides 7 then also covers the prolongation to the
 * finest level, which that sweep's kernel forms on the fly.
 * qpat_profile(ctx, 1) clears the counters and starts, 0 stops. */
#define QPAT_NKSTAT 12
typedef struct {
    int64_t launches;       /* launches that did work                                */
    int64_t lanes;          /* sum over those launches of the right-hand sides still
                               iterating (the rest of the block is skipped)         */
    double  total_ms;
    double  min_ms;
    double  max_ms;
} qpat_kstat;
qpat_status qpat_profile(qpat_ctx* ctx, int32_t enable);
qpat_status qpat_profile_read(const qpat_ctx* ctx, qpat_kstat out[QPAT_NKSTAT]);

/* Batched instances (several independent reconstructions, e.g. meshes of
 * different sizes and illumination counts): run one call on n contexts at
 * once and return when all have finished. Each context must own a distinct
 * HIP stream (given at qpat_setup_mesh); the calls run on one host thread per
 * context, so their kernels and graph replays overlap on the device.
 *   QPAT_BATCH_FORWARD  : qpat_forward(ctx, in0 = kappa, in1 = mu, phi = NULL, h = out0 or NULL)
 *   QPAT_BATCH_JVP      : qpat_jvp(ctx, in0 = s, out0)
 *   QPAT_BATCH_VJP      : qpat_vjp(ctx, in0 = t, out0)
 *   QPAT_BATCH_PAIR     : qpat_jvp(ctx, in0, out0) then qpat_vjp(ctx, in1, out1)
 *   QPAT_BATCH_LSQR_STEP: qpat_lsqr_step(ctx, NULL); arrays unused (may be NULL)
 * ctxs, in0, out0, in1, out1: host arrays of n pointers (the pointers device
 * arrays as in the single calls); infos: n entries (host) or NULL, the pair's
 * two calls merged. 1 <= n <= 256. Returns the first failing instance's
 * status (its message in that context's qpat_last_error), or QPAT_OK. */
typedef enum {
    QPAT_BATCH_FORWARD = 0,
    QPAT_BATCH_JVP = 1,
    QPAT_BATCH_VJP = 2,
    QPAT_BATCH_PAIR = 3,
    QPAT_BATCH_LSQR_STEP = 4
} qpat_batch_op;
qpat_status qpat_batch(qpat_ctx* const* ctxs, int32_t n, int32_t op, const double* const* in0, double* const* out0,
                       const double* const* in1, double* const* out1, qpat_info* infos);

/* Storage of the PCG operators. out[0] = 1 when the node numbering was
 * recognised as a lattice (the stencil form exists), out[1..3] = nx, ny, nz,
 * out[4] = stored stencil arrays per operator (diagonal + upper offsets),
 * out[5] = padded sliced-ELL entries. out: 6 int64 (host). */
qpat_status qpat_operator_layout(const qpat_ctx* ctx, int64_t out[6]);

/* The tile schedule of the multigrid K solves for blocks of B right-hand sides
 * (B = 8 or 16), set at the first solve with that B: out[0] = 1 if the finest
 * level is tiled, out[1] / out[2] = the z-chunk length in use / the cost
 * model's for the direction, update and residual tiles, out[3] / out[4] and
 * out[5] / out[6] = the same for the fused prolongation + last sweep in FP64
 * and FP32 staging (0: not in use), out[7] = 1 if the lengths in use were
 * picked by timing (opts.autotune). QPAT_ERR_STATE before that solve. */
qpat_status qpat_tile_schedule(const qpat_ctx* ctx, int32_t B, int32_t out[8]);

/* ---- Learned initial guess of the forward solves (extension; needs a
 * structured node lattice: node (x, y, z) has index x + nx (y + ny z)).
 * A four-layer 3x3x3 convolutional network, channels 3 -> 16 -> 16 -> 16 -> 1,
 * ReLU between layers, zero padding, BF16 weights and activations with FP32
 * accumulation on MFMA. Parameters (15601 FP32 on the device) are ordered
 * layer by layer as w[c_out][c_in][27] (taps (dz, dy, dx), dx fastest) then
 * b[c_out]. For illumination k the inputs are log(mu/mu0), log(kappa/kappa0)
 * and log(phi_hom_k), phi_hom_k the fluence of the homogeneous (kappa0, mu0)
 * medium; the output is the log correction, phi0_k = phi_hom_k exp(net). */
qpat_status qpat_guess_setup(qpat_ctx* ctx, int32_t nx, int32_t ny, int32_t nz);
qpat_status qpat_guess_set_params(qpat_ctx* ctx, const float* params);   /* also resets Adam */
qpat_status qpat_guess_get_params(qpat_ctx* ctx, float* params);
/* raw network: input [3][N] FP32, out [N] FP32 */
qpat_status qpat_guess_eval(qpat_ctx* ctx, const float* input, float* out);
/* mean squared error against target [N] and its gradient [15601] (grad may be NULL) */
qpat_status qpat_guess_grad(qpat_ctx* ctx, const float* input, const float* target, float* grad,
                            double* loss);
/* one Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on a raw sample */
qpat_status qpat_guess_train_step(qpat_ctx* ctx, const float* input, const float* target, float lr,
                                  double* loss);
/* one Adam step on the sample of one illumination: phi_hom, phi [N] FP64 */
qpat_status qpat_guess_train(qpat_ctx* ctx, const double* kappa, const double* mu, double kappa0,
                             double mu0, const double* phi_hom, const double* phi, float lr,
                             double* loss);
/* predicted fluence for every illumination: phi_hom, phi0_out [n_ill][N] FP64 */
qpat_status qpat_guess_fluence(qpat_ctx* ctx, const double* kappa, const double* mu, double kappa0,
                               double mu0, const double* phi_hom, double* phi0_out);
/* qpat_forward with the solves started from x0 [n_ill][N]; the stopping rule
 * is unchanged (true residual relative to ||f_k||). */
qpat_status qpat_forward_x0(qpat_ctx* ctx, const double* kappa, const double* mu, const double* x0,
                            double* phi_out, double* h_out, qpat_info* info);

/* Number of geometry classes the Jacobian's element kernels use: at mesh
 * set-up every tetrahedron's geometry (|T| and the barycentric gradients)
 * is compared bit for bit with the distinct geometries of the first 64
 * tetrahedra; when each matches one of at most 16, the kernels read a class
 * id instead of the per-tetrahedron row (results unchanged). 0: per-
 * tetrahedron rows. A uniform Kuhn lattice whose spacing is exact in binary
 * has 6. Host-only; -1 for a null context. */
int32_t qpat_geometry_classes(const qpat_ctx* ctx);

/* Steps taken since qpat_lsqr_init (0 before any init or for a null context). */
int32_t qpat_lsqr_steps(const qpat_ctx* ctx);

/* Vectors in the stored bases that the reorthogonalisation of the current
 * LSQR run works against (steps + 1 while it is on); 0 when it is off --
 * lsqr_reorth = 0, or the run went on with the plain recurrences because the
 * device could not hold larger bases. */
int32_t qpat_lsqr_basis(const qpat_ctx* ctx);

/* |phibar| after the last qpat_lsqr_init (= ||yt||) or qpat_lsqr_step, from
 * the host copy made when that call returned; -1 before any init. */
double qpat_lsqr_residual(const qpat_ctx* ctx);

const char* qpat_last_error(const qpat_ctx* ctx);
const char* qpat_version(void);
void qpat_destroy(qpat_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* QPAT_H */
