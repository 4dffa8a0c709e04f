/*
 * nce.h -- C ABI of the MI355X narrow capture / narrow escape solver.
 *
 * Problem (Kaye & Greengard, Section 1 and Section 3): N disk-shaped patches of
 * common arclength radius eps on the unit sphere, centres c_i, any two centres
 * at least 3 eps apart in arclength. The narrow escape (interior) problem
 * returns the average mean first passage time mu; the narrow capture
 * (exterior) problem returns the capture rate. Both come from the solution of
 * the preconditioned second-kind multiple scattering system (eq. opinteqnsdisc)
 *
 *     f_i + P sum_{j != i} S_ij B f_j = P 1,   i = 1..N,
 *
 * whose unknowns f_i are K = (M+1)(M+2)/2 Zernike coefficients per patch.
 *
 * Conventions shared by every call
 *   - Coefficient vectors are N x K, row-major (patch-major), FP64. Basis order:
 *     n ascending, then m = -n, -n+2, ..., n; m < 0 is the sin(|m| theta)
 *     function; radial argument t/eps where t is arclength from the centre.
 *     The theta = 0 direction of patch i is e1_i from nce_frames(): the
 *     projection of z-hat onto the tangent plane, or of x-hat when
 *     |c_i . z-hat| > 1/sqrt(2); e2_i = c_i x e1_i.
 *   - Pointers named *_dev are device memory of the current HIP device
 *     (for example a torch tensor's data_ptr()); the library reads and writes
 *     them asynchronously on the context's stream. Pointers named *_host are
 *     host memory. The caller owns every pointer it passes; nce_setup copies
 *     the centres.
 *   - Every call returns an int status: NCE_OK (0), a negative error code, or
 *     NCE_NOTCONVERGED (1) when an iteration limit was reached (outputs are
 *     still written). nce_strerror() describes a code; nce_last_error() gives
 *     the message of the last failure on the calling thread.
 *   - A context may be used by one host thread at a time.
 */
#ifndef NCE_H
#define NCE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NCE_OK 0
#define NCE_NOTCONVERGED 1
#define NCE_EINVAL (-1)   /* bad argument: N < 1, NaN or non-unit centre, eps outside (0, pi/3], ... */
#define NCE_ESEP (-2)     /* two centres closer than 3 eps in arclength */
#define NCE_ENOMEM (-3)   /* host or device allocation failed */
#define NCE_EHIP (-4)     /* a HIP runtime call failed; message in nce_last_error() */
#define NCE_ETABLE (-5)   /* the per-eps precompute failed its self-check */
#define NCE_ESTATE (-6)   /* call not valid in the context's state (e.g. no MLP loaded) */

typedef struct nce_ctx nce_ctx;

/* problem: 0 = interior (narrow escape, mean first passage time),
 *          1 = exterior (narrow capture, capture rate). */
#define NCE_INTERIOR 0
#define NCE_EXTERIOR 1

/* precision of a matrix-vector product or solve */
#define NCE_FP64 0   /* every step in FP64 */
#define NCE_MIXED 1  /* FP32 Green's sums and block applies inside FP64 iterative refinement */

/* far-field method */
#define NCE_FAR_AUTO 0    /* the tree or the direct sum, whichever has the smaller operation count */
#define NCE_FAR_DIRECT 1  /* all pairs of patches summed directly */
#define NCE_FAR_TREE 2    /* hierarchical cube-sphere quadtree (Section 7.2, Section 8 step 2) */

typedef struct nce_opts {
    int problem;        /* NCE_INTERIOR or NCE_EXTERIOR */
    int M;              /* Zernike truncation; K = (M+1)(M+2)/2, 0 <= M <= 15 (the kernels hold at
                           most 2 (M+1)^2 = 512 sampling nodes per patch). Default 15 (K = 136) */
    double tol_id;      /* ID tolerance of the compressed outgoing representation. Default 1e-11 */
    double tol_grid;    /* incoming-grid truncation tolerance (tree only). Default 1e-8 */
    double tol_gmres;   /* relative residual ||b - A x|| / ||b|| to stop at. Default 1e-10 */
    int max_iter;       /* GMRES iteration limit (FP64) or inner limit (mixed). Default 200 */
    int precision;      /* NCE_FP64 or NCE_MIXED for the solves. Default NCE_FP64 */
    int far_field;      /* NCE_FAR_AUTO / NCE_FAR_DIRECT / NCE_FAR_TREE. Default AUTO */
    void *stream;       /* hipStream_t to run on; NULL = the library creates one */
    const char *cache_dir; /* directory for per-eps tables; NULL = $NCE_CACHE or no cache */
    double tol_grid_fp32; /* grid tolerance of the FP32 applies (mixed solves): a second, coarser
                             set of incoming grids when it differs from tol_grid; 0 = tol_grid.
                             Default 3e-4 (FP32 apply errors then measure 2e-5 to 3.4e-5 of the
                             scattered field; the FP64 residuals always use tol_grid, so this
                             only sets how far one refinement step gets) */
    double tol_id_fp32;   /* ID tolerance of the outgoing representation used by the FP32 applies
                             (mixed solves); 0 = tol_id. Default 1e-5 (with tol_grid_fp32, one
                             refinement step from a 5e-4 start still reaches 1e-8 with a margin
                             of 2; the FP64 residuals always use tol_id) */
    double tol_coarse;    /* relative residual to which the coarse (monopole) solve of the initial
                             guess is taken (nce_set_warm_start, nce_coarse_solve); in (0, 0.1).
                             Default 1e-5 (the guess's own residual is set by the monopole
                             model, near 5e-4 at N = 1e5; tighter solves do not improve it) */
    int deflation;        /* 1: the FP32 inner solves of the mixed form are right-preconditioned by
                             coarse-space deflation (not in the paper): the 16 polynomials of degree
                             <= 3 in the patch centres, in every patch's first coefficient, with the
                             coarse (monopole) model of the system on them; built at the first mixed
                             solve or coarse solve of a context with N >= 64, and it also
                             preconditions the coarse solve of the initial guess. 0: off. The FP64
                             solves are never preconditioned. Default 1 */
} nce_opts;

typedef struct nce_info {
    int iters_fp64;       /* FP64 matrix-vector products inside GMRES */
    int iters_fp32;       /* FP32 matrix-vector products (mixed) */
    int outer;            /* outer refinement steps (mixed) */
    int used_fallback;    /* 1 if a learned start or mixed refinement was rejected */
    double rel_residual;  /* final FP64 ||b - A x|| / ||b|| */
    double t_solve_s;     /* wall time of the solve */
    double rel_residual_x0; /* FP64 relative residual of the initial guess */
} nce_info;

/* Fill opts with the defaults listed above. */
void nce_default_opts(nce_opts *opts);

/*
 * Build a context for one patch layout (Section 8, Steps 1 and 2).
 * centers_host: N x 3 row-major unit vectors (|c| = 1 within 1e-12).
 * Computes (or loads from the cache) the per-eps tables -- the one-patch
 * solution operator (Section 9), the compressed outgoing representation T
 * and its skeleton (Section 7.1), the integral vector I (eq. getI) and the
 * Zernike transform P (Section 4) -- builds the tree when the tree is used,
 * and copies everything to the current HIP device.
 * Errors: NCE_EINVAL, NCE_ESEP, NCE_ENOMEM, NCE_EHIP, NCE_ETABLE.
 */
int nce_setup(const double *centers_host, int64_t N, double eps, const nce_opts *opts,
              nce_ctx **out);

/*
 * A configuration of patches of several radii (the paper's Section 11 names
 * patches of different sizes as an extension; the formulation of Sections 3,
 * 6 and 8 holds with one precompute per radius): radius_host[i] is the
 * arclength radius of patch i, at most 8 distinct values in (0, pi/3]; any two
 * patches must satisfy centre arclength >= eps_i + eps_j + max(eps_i, eps_j)
 * (a gap of at least the larger radius; 3 eps for equal radii), so that every
 * patch lies in the far-field region of every other. Every radius gets its
 * own tables; patch j radiates through its radius's outgoing representation
 * and patch i is sampled at its radius's nodes. nce_matvec, nce_solve_*,
 * nce_frames, nce_dims, nce_work, nce_autotune and nce_set_solver work on the
 * context as on any other (coefficient vectors in the caller's patch order),
 * and so do nce_field and nce_patch_residual (each patch by its own radius's
 * densities, skeleton and quadrature), the coarse solve and start and the
 * deflation (every patch's charge chi0 that of its own radius). The learned
 * start (a network in nce_set_warm_start), nce_features and
 * nce_integral_vector (use nce_types) return NCE_ESTATE. One distinct radius
 * is the same as nce_setup.
 * Errors: NCE_EINVAL, NCE_ESEP, NCE_ENOMEM, NCE_EHIP, NCE_ETABLE.
 */
int nce_setup_radii(const double *centers_host, const double *radius_host, int64_t N, const nce_opts *opts,
                    nce_ctx **out);

/* The context's patch radii in ascending order (*ntypes of them, at most 8),
 * each radius's integral vector I (ntypes x K host doubles, may be NULL) and
 * the radius index of every patch (N ints in the caller's order, may be NULL).
 * eps_host may be NULL. */
int nce_types(const nce_ctx *ctx, int *ntypes, double *eps_host, double *I_host, int *type_host);

/* Free every host and device resource of ctx (NULL is allowed). */
void nce_destroy(nce_ctx *ctx);

/* Sizes: K basis functions, K* Zernike sampling nodes, p skeleton points,
 * number of tree levels used (0 for the direct far field). Any pointer may be NULL. */
int nce_dims(const nce_ctx *ctx, int *K, int *Kstar, int *p, int *levels);

/* Patch frames, N x 9 host doubles per patch: c (3), e1 (3), e2 (3). */
int nce_frames(const nce_ctx *ctx, double *frames_host);

/* Work counts of one matrix-vector product at the given precision (NCE_FP64
 * or NCE_MIXED, whose grids may be coarser): Green's function pair evaluations
 * of the far field (P2L or direct), of the near field, and interpolation
 * multiply-adds (tree L2T). Any pointer may be NULL. */
int nce_work(const nce_ctx *ctx, int precision, double *pairs_far, double *pairs_near, double *interp_fma);

/*
 * One application of the system matrix (eq. sysmatapply):
 *   y_i = x_i + P sum_{j != i} G(Z_i, S_j) T x_j
 * x_dev, y_dev: N x K FP64 device arrays (may not alias).
 * precision NCE_FP64 computes every step in FP64; NCE_MIXED computes the
 * block apply T x, the Green's sums and P in FP32 and adds x in FP64.
 * Asynchronous on the context's stream.
 */
int nce_matvec(nce_ctx *ctx, const double *x_dev, double *y_dev, int precision);

/*
 * Same as nce_matvec, but records HIP events between the steps on the
 * context's stream, waits, and writes the elapsed milliseconds of each step:
 * step_ms[0] block apply rho = T x (Step 1), [1] far field (Step 2, or the
 * direct all-pairs sum), [2] near field (Step 3), [3] incoming-grid
 * interpolation (Step 4), [4] P apply and identity (Step 5). Steps the
 * context does not use report 0.
 */
int nce_matvec_profile(nce_ctx *ctx, const double *x_dev, double *y_dev, int precision,
                       double *step_ms_host);

/*
 * Autotuner: times every valid shape of the far-field kernels on this
 * context's own tree at the given precision -- the P2L form (4 or 8 grid
 * points per thread, per-item choice of the two, or matrix-core tiles; see
 * nce_set_shapes) and interpolation nodes per thread (2, 4 or 8 with 256, 128
 * or 64 threads per patch) -- and keeps the fastest for later applies. choice_host
 * (may be NULL): the two chosen values. Synchronises the stream; no effect on
 * a context that sums its far field directly. Results do not depend on the
 * shapes beyond rounding order.
 */
int nce_autotune(nce_ctx *ctx, int precision, int *choice_host);

/*
 * Sets the far-field kernel shapes directly (what nce_autotune chooses):
 * p2l_shape 4 or 8 grid points per thread, 0 = per work item the one of the
 * two that keeps more lanes busy, 16 = the matrix-core form (16 x 16 tiles of
 * pair distances on the MFMA units, Green's function on the vector units);
 * l2t_npt 2, 4 or 8 interpolation nodes per thread. Results differ only in
 * summation order. NCE_EINVAL for other values, or a shape the tree's largest
 * grid does not fit (4 points per thread hold grids of up to 1024 points).
 */
int nce_set_shapes(nce_ctx *ctx, int precision, int p2l_shape, int l2t_npt);

/*
 * Change the solver settings of an existing context (tables and tree are
 * kept): relative residual tolerance, iteration limit, NCE_FP64 or NCE_MIXED.
 * Errors: NCE_EINVAL for values outside the ranges nce_setup accepts.
 */
int nce_set_solver(nce_ctx *ctx, double tol_gmres, int max_iter, int precision);

/*
 * Solve the interior problem (Section 2.3): GMRES (opts.precision FP64), or
 * FP32 inner GMRES inside FP64 iterative refinement (NCE_MIXED), to
 * opts.tol_gmres, optionally from the learned warm start.
 * coeffs_dev: N x K device output (may be NULL); patch_flux_dev: N device
 * output I . f_i (may be NULL); mfpt_host: mu = 1/(3 I_sigma) - 3/5
 * (eq. mufromsigma2); info may be NULL. Synchronises the stream.
 * Returns NCE_ESTATE if the context was built for the exterior problem.
 */
int nce_solve_interior(nce_ctx *ctx, double *coeffs_dev, double *patch_flux_dev,
                       double *mfpt_host, nce_info *info);

/*
 * Solve the exterior problem (Section 2.2). capture_rate_host receives
 * 4 pi I_sigma (the total flux of the concentration; the paper's J is
 * -I_sigma); I_sigma_host receives I_sigma (may be NULL).
 */
int nce_solve_exterior(nce_ctx *ctx, double *coeffs_dev, double *patch_flux_dev,
                       double *capture_rate_host, double *I_sigma_host, nce_info *info);

/* ------------------------------------------------------------------------
 * Learned warm start: a small FP32 multilayer perceptron (SiLU hidden layers,
 * linear output) that maps each patch's local geometry to its coefficient
 * vector f_i, trained on solutions this library computes. It only supplies
 * the initial guess: x0 = gamma m with gamma fitted by one system apply, and
 * GMRES (or the refinement loop) always runs on the true residual; the guess
 * is rejected (info.used_fallback = 1) when it does not reduce the residual.
 * Parameters are flattened per layer as W (row-major, out x in) then b.
 * All *_dev arrays are FP32 device memory; `stream` is a hipStream_t (NULL =
 * the null stream); calls that return host values synchronise it.
 * ------------------------------------------------------------------------ */
typedef struct nce_mlp nce_mlp;

#define NCE_FEATURES 56 /* per patch: 16 nearest neighbours x (u, v, 1/r) in the patch frame
                           (positions / (16 eps), 4 eps / distance), problem flag, 10 x area
                           fraction, neighbour density relative to uniform within 8, 16, 32, 64 eps,
                           10 x (a_i / mean a - 1) and mean a (a: coarse amplitudes, see below) */

/* He-initialised network n_in -> width (x hidden_layers, SiLU) -> n_out. */
int nce_mlp_create(int n_in, int width, int hidden_layers, int n_out, uint64_t seed, nce_mlp **out);
void nce_mlp_destroy(nce_mlp *m);
int nce_mlp_num_params(const nce_mlp *m, int64_t *n);
int nce_mlp_get_params(const nce_mlp *m, float *params_host);
int nce_mlp_set_params(nce_mlp *m, const float *params_host);
/* y (B x n_out) = network(x (B x n_in)). */
int nce_mlp_forward(nce_mlp *m, const float *x_dev, int64_t B, float *y_dev, void *stream);
/*
 * nce_mlp_forward for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops that forbid hipMalloc): the same arguments
 * and results, with no allocation of any kind. The hidden activations live in
 * a fixed 16 MiB device array of the library (one per GPU, held until the
 * process ends); rows are processed in chunks that fit it (8192 rows at width
 * 256) and the output is written straight to y_dev (B x n_out). Nothing in
 * the array needs clearing between calls. Calls that overlap on one GPU (other
 * streams or host threads) share the array and race: serialize them. Runs on
 * the current HIP device, on `stream`.
 * Errors: NCE_EINVAL for a NULL argument, B < 1, or hidden layers so wide that
 * one row (2 x width floats) does not fit the array; NCE_EHIP.
 */
int nce_mlp_forward_noalloc(nce_mlp *m, const float *x_dev, int64_t B, float *y_dev, void *stream);
/* Mean squared error L = sum (y - t)^2 / (B n_out) and its gradient with
 * respect to the parameters (grad_host may be NULL; it is left on the device). */
int nce_mlp_loss_grad(nce_mlp *m, const float *x_dev, const float *t_dev, int64_t B, double *loss_host,
                      float *grad_host, void *stream);
/* One Adam step (beta 0.9 / 0.999, eps 1e-8) on the loss of this batch. */
int nce_mlp_train_step(nce_mlp *m, const float *x_dev, const float *t_dev, int64_t B, float lr, double *loss_host,
                       void *stream);
/* The NCE_FEATURES features of every patch of ctx (N x NCE_FEATURES FP32 device
 * array); runs the coarse solve if it has not run yet. */
int nce_features(nce_ctx *ctx, float *feat_dev);

/*
 * Coarse (monopole) model of the system: with f_i = a_i e_0 and every far
 * field taken as its total charge at the patch centre, row 0 of eq.
 * opinteqnsdisc becomes a_i + chi0 sum_{j != i} G(c_i, c_j) a_j = 1 (chi0 =
 * total charge of e_0 in the outgoing table; with several patch radii, patch
 * j's own radius's chi0_j inside the sum). Solved on the device by GMRES to
 * opts.tol_coarse (FP32 pair sums); once per context. a_dev: N doubles out, in
 * the caller's patch order (may be NULL); iters_host: GMRES iterations (may be
 * NULL); chi0_host: chi0, or with several radii one value per radius in the
 * order of nce_types (ntypes doubles; may be NULL). Not in the paper.
 */
int nce_coarse_solve(nce_ctx *ctx, double *a_dev, int *iters_host, double *chi0_host);

/*
 * The coarse-space deflation of the mixed solves (opts.deflation; not in the
 * paper): *k (<= 16) independent basis columns, the orthonormalized harmonic
 * polynomials of degree <= 3 in the patch centres, and T = I + chi0 Z^T G Z,
 * the coarse model of the system on them (G(c_i, c_j) between centres, i != j;
 * chi0 as for nce_coarse_solve; with several radii T = I + Z^T G D Z, D the
 * diagonal of every patch's chi0_j). T_host: k*k host doubles, row-major (room for
 * 256 suffices), may be NULL. Builds the deflation if the context has not yet;
 * k = 0 for N < 64, where none is used.
 */
int nce_deflation_matrix(nce_ctx *ctx, int *k, double *T_host);

/* Turns the deflation of later mixed solves on (1) or off (0), as opts.deflation. */
int nce_set_deflation(nce_ctx *ctx, int on);

/*
 * Initial guess of later solves (not in the paper): use_coarse = 1 starts from
 * x0_i = a_i e_0 (the coarse solve); with a network m (n_in = NCE_FEATURES,
 * n_out = K) also, x0_i = a_i m_i with m_i the network's output for patch i.
 * GMRES judges the guess: if its FP64 residual is not below 0.99 ||b||, the
 * solve starts from zero (nce_info.used_fallback). The per-layout work (the
 * coarse solve, and the network's features, computed on host threads while
 * the coarse solve runs) is done here, not in the next solve. m = NULL and
 * use_coarse = 0 disable and drop that work, so a later call redoes it; m
 * without use_coarse is NCE_EINVAL; m on a context of several patch radii is
 * NCE_ESTATE (the network's features are those of one radius). The caller
 * keeps m alive while it is set.
 */
int nce_set_warm_start(nce_ctx *ctx, nce_mlp *m, int use_coarse);

/* Integral vector I (K host doubles): I_sigma = I . sum_i f_i (eq. getI). */
int nce_integral_vector(const nce_ctx *ctx, double *I_host);

/*
 * Field of the patch densities at points of the domain (Sections 2.2, 2.3):
 * the single-layer potential u(x) = sum_j int G_E(x, x') sigma_j(x') dS'
 * (exterior, eq. urep) or v(x) with G_I (interior, eq. intBVPansatz), G the
 * off-surface Neumann Green's function (eqs. Gextoffsurface, Gintoffsurface)
 * and sigma_j = B f_j the density of coefficients f_j; with physical = 1 the
 * physical field instead: ubar = 1 - u (exterior; 1 at infinity, 0 on the
 * patches) or the mean first passage time vbar = (v - 1)/(3 D) +
 * (1 - |x|^2)/6, D = -I_sigma (interior, eq. vtilde).
 * coeffs_dev: N x K device coefficients (for example a solve's output);
 * points_dev: n x 3 device doubles, |x| <= 1 (interior) or |x| >= 1
 * (exterior), points on the sphere allowed (on a patch: that patch's term is
 * its data sum_k f_ik Z_k); values_dev: n device doubles out.
 * Patches whose centre lies at arclength >= 3 eps from x/|x| enter through the
 * compressed outgoing representation, nearer ones by quadrature of their
 * density (260 radial nodes x 256 angles): accurate to about the ID tolerance
 * for points at least eps/10 from every patch they do not lie on (with
 * several radii, eps is each patch's own).
 * Synchronises the context's stream. Errors: NCE_EINVAL (NULL pointer, n < 0,
 * non-finite point or one outside the problem's domain), NCE_ESTATE (a
 * context of several configurations), NCE_EHIP.
 */
int nce_field(nce_ctx *ctx, const double *coeffs_dev, const double *points_dev, int64_t n, int physical,
              double *values_dev);

/*
 * L2 residual of the absorbing condition on patches (eq. l2res, normalised
 * as printed): residual_host[a] = (1/|Gamma_i|) ||v - 1||_{L2(Gamma_i)} for
 * patch i = patches_host[a] (0 <= i < N), with v the potential of nce_field
 * for coefficients coeffs_dev, by the rule n_t Gauss-Legendre nodes in
 * arclength on [0, eps] times n_theta equispaced angles offset by half a step
 * (1 <= n_t <= 64, 1 <= n_theta <= 256); |Gamma_i| = 2 pi (1 - cos eps), eps
 * the patch's radius; patch numbers in the caller's order.
 * Synchronises. Errors: NCE_EINVAL, NCE_ESTATE, NCE_EHIP.
 */
int nce_patch_residual(nce_ctx *ctx, const double *coeffs_dev, const int64_t *patches_host, int npatch, int n_t,
                       int n_theta, double *residual_host);

/* ------------------------------------------------------------------------
 * Batched solves: many independent configurations (their own centres, eps and
 * problem) in one set of launches. Not in the paper, whose solver treats one
 * configuration at a time; each configuration's system is the one above
 * (eq. opinteqnsdisc) and its result the scalar of Section 2.
 *
 * Configurations with equal (problem, eps) share tables and are applied by
 * the same launches; each configuration's far field uses its own quadtree or
 * direct all-pairs lists, whichever has the smaller operation count (unless
 * opts.far_field forces one). Batch vectors (device, FP64) hold configuration
 * b's N_b x K coefficients at the element offset nce_batch_offsets() gives.
 */
typedef struct nce_batch nce_batch;

/*
 * centers[b]: host array N[b] x 3 of configuration b (unit vectors, pairwise
 * separation >= 3 eps[b]); problem[b]: NCE_INTERIOR or NCE_EXTERIOR; B >= 1.
 * opts: shared settings (opts.problem is ignored; opts.max_iter <= 120 is the
 * Krylov dimension of the lockstep GMRES; opts.stream as in nce_setup).
 * Errors: NCE_EINVAL / NCE_ESEP (message names the configuration), NCE_ENOMEM,
 * NCE_EHIP, NCE_ETABLE. Release with nce_destroy_batch.
 */
int nce_setup_batch(const double *const *centers_host, const int64_t *N_host, const double *eps_host,
                    const int *problem_host, int B, const nce_opts *opts, nce_batch **out);
void nce_destroy_batch(nce_batch *batch);

/* Total batch vector length, K, and the number of (problem, eps) groups. */
int nce_batch_dims(const nce_batch *batch, int64_t *n_total, int *K, int *ngroups);

/* off_host[b] (B entries): first element of configuration b in batch vectors;
 * far_tree_host[b] (may be NULL): 1 if its far field uses the tree, 0 direct. */
int nce_batch_offsets(const nce_batch *batch, int64_t *off_host, int *far_tree_host);

/* Operation counts of one batched apply at the given precision (as nce_work). */
int nce_batch_work(const nce_batch *batch, int precision, double *pairs_far, double *pairs_near, double *interp_fma);

/* y = A x for every configuration (batch layout, device, FP64 in and out;
 * precision NCE_FP64 or NCE_MIXED = FP32 steps). x and y must not alias. */
int nce_batch_matvec(nce_batch *batch, const double *x_dev, double *y_dev, int precision);

/* Solver settings: relative residual tolerance (per configuration), Krylov
 * dimension (1..120), NCE_FP64 or NCE_MIXED, and whether one Arnoldi step is
 * replayed as a captured HIP graph (1) or launched kernel by kernel (0). */
int nce_batch_set_solver(nce_batch *batch, double tol_gmres, int max_iter, int precision, int use_graph);

/*
 * Solve every configuration from x0 = 0: lockstep GMRES over the batch
 * (NCE_FP64), or FP32 lockstep GMRES inside FP64 iterative refinement
 * (NCE_MIXED); a configuration stops iterating once its own FP64-verified
 * residual meets the tolerance. result_host[b]: mu (interior, eq.
 * mufromsigma2) or the capture rate 4 pi I_sigma (exterior) of configuration
 * b; coeffs_dev (may be NULL): the batch solution vector; infos_host[b] (may
 * be NULL): per configuration, with t_solve_s the whole batch's time.
 * Returns NCE_NOTCONVERGED if any configuration missed the tolerance.
 */
int nce_solve_batch(nce_batch *batch, double *result_host, double *coeffs_dev, nce_info *infos_host);

/* Initial guess of later batched solves, as nce_set_warm_start: a coarse solve
 * per member (use_coarse = 1), refined per patch by network m when given. */
int nce_batch_set_warm_start(nce_batch *batch, nce_mlp *m, int use_coarse);

/* Turns the coarse-space deflation of the batch's mixed inner solves on (1)
 * or off (0) (opts.deflation at setup; not in the paper): per member, as
 * nce_set_deflation, for members of at least 64 patches. Turning it on for a
 * mixed batch builds every member's deflation data now. */
int nce_batch_set_deflation(nce_batch *batch, int on);

/* nce_autotune for every (problem, eps) group of the batch; choice_host (may
 * be NULL): 2 x ngroups values in group order. */
int nce_batch_autotune(nce_batch *batch, int precision, int *choice_host);

/* Short description of a status code. */
const char *nce_strerror(int code);

/* Message of the last error on the calling thread ("" if none). */
const char *nce_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* NCE_H */
