/*
 * mlg.h -- C ABI of the MI355X multilayer-graph Laplacian library (libmlg.so).
 *
 * Operators (Bergermann, Stoll, Volkmer, "Semi-supervised learning for
 * aggregated multilayer graphs using diffuse interface methods and fast
 * matrix-vector products"):
 *
 *   W        layer weight matrix, W_ij = exp(-||x_i - x_j||^2 / sigma^2),
 *            W_ii = 0                                   (Sec. 2, Sec. 4)
 *   D        diag(W 1)                                  (Sec. 2)
 *   L_sym    I - D^-1/2 W D^-1/2                        (Sec. 2)
 *   I - L_1  (1/T) sum_t D_t^-1/2 W_t D_t^-1/2          (Sec. 3, eq. for I - L_1)
 *
 * W v is evaluated either by direct summation (Sec. 2, case (i)) or by NFFT
 * fast summation (Algorithm 1 of Sec. 4; the self term is removed through
 * W = W~ - K(0) I).
 *
 * Conventions shared by every call:
 *  - Status codes are returned; nothing throws across the ABI.  On an error
 *    the outputs are unspecified; mlg_last_error() gives a message
 *    (thread-local, valid until the next call on the same thread).
 *  - Blocks of vectors are column-major n x b FP64 arrays with a leading
 *    dimension ld >= n.
 *  - With MLG_DEVICE_PTRS in `flags`, array arguments are HIP device pointers
 *    (e.g. torch.Tensor.data_ptr() of a CUDA/HIP tensor); otherwise they are
 *    host pointers and the library stages them through device memory.
 *  - The caller owns every array it passes.  The library never frees a
 *    caller pointer and keeps none past the call.  A graph handle owns its
 *    own device memory (points, plans, degrees, workspaces, HIP graphs).
 *  - Work is enqueued on the HIP stream given at creation (NULL = a
 *    non-blocking stream the handle creates and owns) and the call returns
 *    after that stream has drained, so device outputs are ready when it
 *    returns (except mlg_laplacian_matvec with MLG_ASYNC).
 *  - One handle must not be used from two threads at once.
 *  - Same inputs and same parameters give bit-identical outputs: no kernel
 *    accumulates floating point through atomics.
 */
#ifndef MLG_H
#define MLG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MLG_OK = 0,
    MLG_WARN_NOT_CONVERGED = 1, /* Lanczos: best Ritz pairs returned, info filled */
    MLG_ERR_ARG = -1,           /* null pointer, bad size, bad leading dimension  */
    MLG_ERR_RANGE = -2,         /* d outside 1..3 for NFFT, N not a power of two,
                                   sigma <= 0, window not even or too wide, ...    */
    MLG_ERR_ISOLATED = -3,      /* a layer has a node of zero degree               */
    MLG_ERR_NOMEM = -4,         /* device allocation failed                        */
    MLG_ERR_HIP = -5,           /* a HIP runtime call failed                       */
    MLG_ERR_NOT_IMPL = -6       /* valid request the library does not implement    */
} mlg_status;

#define MLG_DEVICE_PTRS 1
/* mlg_graph_create: skip the degree pass; the graph then serves MLG_OP_W
 * products only (degree-normalised operators, degrees and Lanczos return
 * MLG_ERR_ARG). */
#define MLG_SKIP_DEGREES 2
/* mlg_laplacian_matvec with MLG_DEVICE_PTRS: enqueue the product on the
 * graph's stream and return without waiting for it, so that back-to-back
 * products leave no host round trip between them.  Y is ready, and X may be
 * overwritten, once that stream has drained (mlg_graph_synchronize, or the
 * caller's own stream given at creation); a kernel error then surfaces there.
 * Ignored for host pointers. */
#define MLG_ASYNC 4

/* summation method */
#define MLG_METHOD_DIRECT 0 /* O(n^2) tiled direct sum (Sec. 2 case (i))       */
#define MLG_METHOD_NFFT 1   /* NFFT fast summation (Algorithm 1, Sec. 4)       */

/* Kernel functions K of the weight w(x_i, x_j) = K(x_i - x_j) (Sec. 2, Sec. 4). */
#define MLG_KERNEL_GAUSSIAN 0  /* exp(-||y||^2 / sigma^2)                        */
#define MLG_KERNEL_LAPLACIAN 1 /* exp(-||y|| / sigma), direct summation only     */

/* operator selector for mlg_laplacian_matvec */
#define MLG_OP_NADJ 0 /* D^-1/2 W D^-1/2 (one layer) or I - L_1 (layer = -1) */
#define MLG_OP_LSYM 1 /* L_sym (one layer) or L_1 (layer = -1)               */
#define MLG_OP_W 2    /* W itself (one layer only), zero diagonal            */

/*
 * Per-layer summation parameters (Sec. 4; fast-summation parameters of the
 * image and hyperspectral experiments in Sec. 8).
 *   method     MLG_METHOD_DIRECT or MLG_METHOD_NFFT.
 *   precision  32 or 64: arithmetic of the summation itself (spreading, FFT,
 *              interpolation or direct tiles).  Degrees, D^-1/2 scaling and
 *              layer aggregation are always FP64.
 *   N          NFFT bandwidth: frequencies l in {-N/2..N/2}^d are kept; the
 *              FFT grid has 2N points per dimension.  Power of two, 8..256,
 *              or 0: the smallest power of two >= 16 whose dropped Gaussian
 *              tail 2 d sqrt(pi) s exp(-(pi s N / 2)^2) (s = scaled sigma)
 *              is below 1e-8 (precision 32) or 1e-13 (precision 64).
 *   window     window support w in grid points, even, 2..16, with
 *              bin + w/2 <= N/2 (0 = 6 for precision 32, 12 for precision 64).
 *   eps_B      regularisation length of the periodised kernel, 0 < eps_B < 1/4.
 *   p_reg      smoothness degree of the regularisation, 1..12.
 *   bin        bin edge in grid cells used to group points (1, 2 or 4),
 *              or 0: automatic.  For precision 32 the plan starts at 1 and
 *              doubles the edge (up to 4) while the occupied bins hold fewer
 *              than 256 points on average, as long as bin + w/2 <= N/2 and
 *              the patch edge bin + w - 1 stays within the matrix-core
 *              kernels (7 in d = 3, 12 in d = 2, 16 in d = 1); precision 64
 *              takes 1.  The bin only groups points, so the result differs
 *              from another bin's by rounding alone; mlg_graph_layer_info
 *              reports the edge chosen.
 *   kernel     MLG_KERNEL_GAUSSIAN (0) or MLG_KERNEL_LAPLACIAN.  The
 *              Laplacian RBF has a cusp at the origin, so its Fourier
 *              coefficients decay only algebraically and Algorithm 1 (no
 *              near-field correction) cannot reach 1e-4: NFFT layers with it
 *              return MLG_ERR_NOT_IMPL.
 * Ignored for MLG_METHOD_DIRECT except `precision` and `kernel`.
 */
typedef struct {
    int method;
    int precision;
    int N;
    int window;
    double eps_B;
    int p_reg;
    int bin;
    int kernel;
} mlg_kparams;

typedef struct mlg_graph mlg_graph;

/* Message describing the last error on this thread ("" if none). */
const char *mlg_last_error(void);

/* Library version string. */
const char *mlg_version(void);

/*
 * Build a multilayer graph (Sec. 2 multilayer graph; Sec. 7 feature
 * grouping gives one layer per feature group).
 *   n        nodes shared by all layers, n >= 2.
 *   T        layers, 1..1024.
 *   d        T layer dimensions (1..3 for NFFT, 1..16 for direct).
 *   points   T pointers, layer t is n x d[t] row-major FP64 (host or device
 *            per flags; only read during the call).
 *   sigma    T kernel widths, > 0.
 *   kp       T parameter records.
 *   flags    MLG_DEVICE_PTRS and/or MLG_SKIP_DEGREES, or 0.
 *   stream   hipStream_t for all work on this graph (NULL = a non-blocking
 *            stream owned by the handle).
 * Plans every layer (torus scaling, kernel Fourier coefficients, bin sort)
 * and, unless MLG_SKIP_DEGREES is given, computes each layer's degrees in
 * FP64: direct layers by the direct sum, NFFT layers by one FP64 fast
 * summation of the ones vector with a plan of its own (bandwidth from the
 * FP64 tail rule, at least the layer's N; window 14, or 12 when a bin of 4
 * is needed to keep its patches below 2 GiB).  The NFFT degree pass's error
 * is measured on 64 evenly spaced rows against the FP64 direct sum.
 * Returns MLG_ERR_ISOLATED if a degree is zero (direct layers) or at most 64
 * times that measured error (NFFT layers: the pass cannot tell it from
 * zero), and MLG_ERR_ARG if a coordinate is not finite.
 */
mlg_status mlg_graph_create(mlg_graph **out, int64_t n, int T, const int *d,
                            const double *const *points, const double *sigma,
                            const mlg_kparams *kp, int flags, void *stream);

/*
 * Feature grouping (Sec. 7): a multilayer graph whose layer t uses the
 * feature columns of group t of one n x D feature matrix, so that data with
 * D >= 4 features can use layers of dimension <= 3 (NFFT) that are merged
 * again by the power mean (Sec. 2).
 *   features    n x D row-major FP64 (host or device per flags; only read
 *               during the call).
 *   T           groups (layers), 1..1024.
 *   group_dim   T group sizes d_t (1..3 for NFFT layers, 1..16 for direct).
 *   group_cols  the groups' feature indices (0..D-1), concatenated in layer
 *               order: sum_t d_t entries, host memory.
 *   sigma, kp, flags, stream   as for mlg_graph_create.
 * The layers are exactly those mlg_graph_create builds from the gathered
 * columns.
 */
mlg_status mlg_graph_create_grouped(mlg_graph **out, int64_t n, int D, const double *features,
                                    int T, const int *group_dim, const int *group_cols,
                                    const double *sigma, const mlg_kparams *kp, int flags,
                                    void *stream);

/*
 * Kernel width from the data: the median of the pairwise Euclidean distances
 * ||x_a - x_b||_2 (a < b) between s sampled nodes, over the d feature columns
 * cols (NULL: 0..d-1) of the n x D row-major feature matrix; for an even
 * number of pairs, the mean of the two middle values.  The paper tunes sigma
 * by a grid search (Sec. 6); this is the data-driven choice the synthetic
 * workloads use.  Each squared distance is summed over the columns in order
 * without fused multiply-add, then rounded to its square root.
 *   sample   s distinct node indices (host memory), 2 <= s <= min(n, 8192).
 *   sigma    out (host).
 */
mlg_status mlg_median_pairwise_distance(int64_t n, int D, const double *features, int d,
                                        const int *cols, int s, const int64_t *sample,
                                        double *sigma, int flags, void *stream);

mlg_status mlg_graph_destroy(mlg_graph *g);

/* Wait until all work enqueued on the graph's stream has finished (for
 * products enqueued with MLG_ASYNC); reports a failed kernel of that work as
 * MLG_ERR_HIP. */
mlg_status mlg_graph_synchronize(mlg_graph *g);

/* Copy layer `layer`'s degrees deg(x_i) (Sec. 2) into deg (n FP64). */
mlg_status mlg_graph_degrees(mlg_graph *g, int layer, double *deg, int flags);

/*
 * Y = W X for one point set, zero diagonal (Sec. 4: W v = W~ v - K(0) v).
 * Stateless: plans, applies and frees.  points n x d row-major FP64.
 */
mlg_status mlg_kernel_matvec(int64_t n, int d, const double *points, double sigma,
                             const mlg_kparams *kp, int b, const double *X, int64_t ldx,
                             double *Y, int64_t ldy, int flags, void *stream);

/*
 * Y = op X with op one of MLG_OP_* for layer `layer` (0..T-1), or for the
 * layer mean (layer = -1, p = 1 power mean of Sec. 2 eq. (1) and Sec. 3).
 * b: 1..64 vectors.  X and Y must not overlap.  The first call for a given
 * (layer, op, b) captures the whole launch sequence (entry kernel, the
 * layers' summations, exit kernel) into one HIP graph; later calls replay
 * it, re-pointing its entry and exit kernels when X, Y or their leading
 * dimensions differ from the previous call's (launches already enqueued keep
 * the buffers they were given).  With device pointers the call only
 * enqueues on the graph's stream.
 */
mlg_status mlg_laplacian_matvec(mlg_graph *g, int layer, int op, int b, const double *X,
                                int64_t ldx, double *Y, int64_t ldy, int flags);

typedef struct {
    int iters;        /* block expansion steps taken                       */
    int restarts;     /* thick restarts                                    */
    int matvecs;      /* p = 1: operator applications to single vectors;  */
                      /* p < 0: single-vector layer matvecs (all inner     */
                      /* Krylov steps), saturating at INT32_MAX            */
    int nconv;        /* wanted pairs whose residual is <= tol             */
    double max_resid; /* max residual norm ||A phi - mu phi|| over the k   */
    int inner_steps;  /* p < 0: longest inner Krylov dimension used        */
    int inner_unconverged; /* p < 0: inner runs stopped at max_steps       */
} mlg_eig_info;

/*
 * Inner iteration of the matrix power for p < 0 (polynomial Krylov method,
 * Sec. 3).  Per column of a block, the Lanczos coefficient vector
 * c_m = f(T_m) e_1 (normalised so that |c| <= 1) is recomputed every 4 steps;
 * the iteration stops when every column changed by <= tol since the last
 * check, which bounds the error relative to ||x|| delta^p, delta^p being the
 * norm of (L_sym + delta I)^p.
 *   tol        <= 0: default (1e-2 x the eigensolver tol; 1e-12 for
 *              mlg_power_mean_matvec).
 *   max_steps  Krylov dimension limit, >= 4; 0: default 128.  The device
 *              caps it where the per-column tridiagonal eigensolve
 *              (max_steps^2 doubles of LDS) would not fit one workgroup.
 */
typedef struct {
    double tol;
    int max_steps;
} mlg_pksm_params;

/*
 * k smallest eigenpairs of a graph Laplacian by FP64 block thick-restart
 * Lanczos with full reorthogonalisation (CGS2) (Sec. 3; Algorithm 2 step 1).
 *   p = 1:  L_sym of one layer (layer >= 0) or L_1 (layer = -1), as the k
 *           largest eigenpairs of D^-1/2 W D^-1/2 resp. I - L_1,
 *           lambda = 1 - mu.
 *   p < 0:  the shifted power mean L_{p,delta}, delta = log(1 + |p|)
 *           (Sec. 2), as the k largest eigenpairs of its p-th power
 *           (1/T) sum_t (L_sym^(t) + delta I)^p (order reversed by
 *           lambda^p), every product through the polynomial Krylov method
 *           (see mlg_power_mean_matvec); the operator is scaled by delta^-p
 *           so that its spectrum lies in (0, 1], and lambda = delta mu^(1/p).
 *           layer >= 0 gives L_sym^(t) + delta I.  The eigenvalues include
 *           the shift (they are >= delta).
 *   p            1.0 or < 0; anything else returns MLG_ERR_NOT_IMPL.
 *   k            1..n/2 wanted pairs.
 *   block        vectors per Lanczos block, 1..32.
 *   tol          stop when every residual ||A phi - mu phi||_2 <= tol.
 *   max_restarts restarts allowed (0 = expand once, no restart).  The
 *                basis grows to max(4k, k + 6 block) columns (rounded up to
 *                whole blocks; at most 256 - block and n - block) before
 *                each restart keeps the k + block best Ritz vectors; the
 *                first expansion also stops for a convergence check every
 *                ~16 columns from max(2k, k + 3 block) columns on.
 *   seed         start block: counter-based N(0,1) draws (SplitMix64 +
 *                Box-Muller) unless V0 is given.
 *   V0           optional n x block start block (same pointer kind as the
 *                outputs), or NULL.
 *   evals        k eigenvalues lambda, ascending.
 *   evecs        n x k column-major, leading dim ldv; unit 2-norm, sign
 *                chosen so that the largest-magnitude entry is positive.
 * Returns MLG_WARN_NOT_CONVERGED if the restarts ran out.
 */
mlg_status mlg_lanczos_eigs(mlg_graph *g, int layer, double p, int k, int block, double tol,
                            int max_restarts, uint64_t seed, const double *V0, double *evals,
                            double *evecs, int64_t ldv, mlg_eig_info *info,
                            const mlg_pksm_params *pk, int flags);

/*
 * Y = (L_sym^(t) + delta I)^p X for layer t >= 0, or
 * Y = L_{p,delta}^p X = (1/T) sum_t (L_sym^(t) + delta I)^p X for layer = -1,
 * with p < 0 and delta = log(1 + |p|) (Sec. 2 shifted power mean; Sec. 3 p-th
 * power), by the polynomial Krylov method of Sec. 3: per layer and column,
 * Lanczos on L_sym^(t) started from x (no reorthogonalisation), then
 * y = ||x|| V_m f(T_m + delta I) e_1 with f(lambda) = lambda^p; f(T_m) e_1
 * comes from an implicit-QL eigensolve of the tridiagonal T_m on the device.
 * FP64 recurrences over the layers' matvecs (NFFT or direct, each in its own
 * precision); every reduction has one fixed order, so results are
 * reproducible bit for bit.
 *   b      1..64 vectors; X and Y n x b column-major (ldx, ldy >= n), not
 *          overlapping.  A zero column gives a zero column.
 *   pk     stopping rule (NULL: defaults, see mlg_pksm_params).
 *   steps  optional out: longest Krylov dimension used.
 * Returns MLG_ERR_ARG for p >= 0 and MLG_WARN_NOT_CONVERGED (Y still
 * written) if some layer stopped at max_steps.  Allocates (max_steps + 1) n b
 * doubles of device workspace for the call.
 */
mlg_status mlg_power_mean_matvec(mlg_graph *g, int layer, double p, int b, const double *X,
                                 int64_t ldx, double *Y, int64_t ldy, const mlg_pksm_params *pk,
                                 int *steps, int flags);

/* Allen--Cahn parameters (Algorithm 2): epsilon, omega_0, c, dt, tolerance,
 * max_iter. */
typedef struct {
    double eps, omega0, c, dt, tol;
    int max_iter;
} mlg_ac_params;

/*
 * Multiclass Allen--Cahn scores in the truncated eigenbasis (Algorithm 2,
 * steps 2-4; Sec. 5-6; Appendix B), FP64.
 *   evals   k eigenvalues lambda_r of the Laplacian.
 *   evecs   n x k column-major, leading dim ldv.
 *   labels  n int32: -1 unlabelled, 0..m-1 class.
 *   U       n x m row-major output scores (rows in the Gibbs simplex).
 *   pred    n int32 output: row argmax, lowest class id on ties (Sec. 6).
 *   iters   iterations run (the loop body runs at least once).
 * The arithmetic follows one fixed FP64 operation order (documented with the
 * kernels), so results are reproducible bit for bit.
 */
mlg_status mlg_allen_cahn_ssl(int64_t n, int k, int m, const double *evals,
                              const double *evecs, int64_t ldv, const int32_t *labels,
                              const mlg_ac_params *prm, double *U, int32_t *pred, int *iters,
                              int flags, void *stream);

/* ---- parameter selection ------------------------------------------------ */

/* Result of mlg_autotune_layer. */
typedef struct {
    int window;    /* chosen window width w (even)                               */
    int N;         /* chosen bandwidth N                                         */
    int bin;       /* chosen bin edge (grid cells per bin and dimension)         */
    int tried;     /* candidates planned and measured                            */
    int passed;    /* candidates within the error budget                         */
    double err;    /* sampled relative error of the choice: max over the b test  */
                   /* vectors of ||Y_s - R_s|| / ||R_s|| over the sampled rows   */
    double ms;     /* wall milliseconds of one b-vector product with the choice  */
                   /* (-1 when no candidate met the budget)                      */
} mlg_tune_info;

/*
 * Choose the NFFT window width w, bandwidth N and bin edge of one
 * Gaussian-kernel layer (Algorithm 1, Sec. 4) for an error budget: the
 * fastest measured candidate
 * whose error on a seeded sample of rows, against the FP64 direct sum of
 * those rows (zero diagonal), is <= tol for a seeded block of b test vectors
 * uniform in [-1, 1).
 *   Candidates: N in {N0/2, N0, 2 N0} (powers of two in 8..256; N0 = the
 *   automatic bandwidth of mlg_graph_create with N = 0) and w in {4, 6, 8, 10}
 *   (FP32) or {4, 6, ..., 16} (FP64), bin in {1, 2, 4}, eps_B = 1/16,
 *   p_reg = 5.  For each (N, bin) the windows are tried in increasing order
 *   and the first within the budget is timed (the fastest of three rounds
 *   of 5 products, after one warm-up);
 *   a later candidate (larger N or bin) replaces the current choice only if
 *   it is at least 5 % faster.
 *   Larger bins give fewer, fuller tasks when points are sparse on the grid;
 *   the d = 3 matrix-core kernels take bin + w - 1 <= 7 (bins of 1 or 2 at
 *   w = 6), wider patches run on the vector ALUs.
 *   points     n x d row-major FP64 (device pointer with MLG_DEVICE_PTRS, else
 *              host), d in 1..3; 2 <= n < 2^31.
 *   precision  32 or 64 (the summation precision of the candidates).
 *   b          test vectors, 1..64;  tol in (0, 1);  nrows sampled rows,
 *              1..min(n, 4096);  seed selects the rows and the test block.
 *   kp         out: the chosen parameters, ready for mlg_graph_create.
 *   info       out: the choice and the counts (always filled when the
 *              arguments are valid).
 * Returns MLG_ERR_RANGE when no candidate meets tol; kp and info then hold
 * the candidate with the smallest sampled error.  The reference rows cost
 * O(nrows n d) on the device.
 */
mlg_status mlg_autotune_layer(int64_t n, int d, const double *points, double sigma,
                              int precision, int b, double tol, int nrows, uint64_t seed,
                              int flags, void *stream, mlg_kparams *kp, mlg_tune_info *info);

/* ---- allocation-free product ------------------------------------------- */

/* Bytes of device scratch the library holds per device (from the first
 * mlg_kernel_matvec_noalloc call on it until the process ends). */
#define MLG_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/*
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, serving loops with a fixed memory budget, harnesses that forbid
 * hipMalloc.  Y = W X as mlg_kernel_matvec computes it with
 * MLG_METHOD_DIRECT (same kernels, same column split, same bits), without
 * any device allocation, host synchronisation or library call that
 * allocates.
 *   points   n x d row-major FP64, device pointer, d in 1..16, n >= 2.
 *   kp       method must be MLG_METHOD_DIRECT (else MLG_ERR_NOT_IMPL);
 *            precision 32 or 64; kernel MLG_KERNEL_GAUSSIAN or
 *            MLG_KERNEL_LAPLACIAN; other fields ignored.
 *   X, Y     n x b column-major FP64 device blocks (ldx, ldy >= n), b in
 *            1..64, not overlapping.
 *   stream   hipStream_t of the current device (NULL = its null stream).
 * Every intermediate (coordinates, summation slices, column partials) lives
 * in one library-owned array of MLG_NOALLOC_SCRATCH_BYTES per device, so the
 * size is limited: with bs = the next power of two >= b, e = 8 (precision
 * 64) or 4 (32), and S column splits (S = 1 for n >= 131072, about
 * 1024 / (n / 128) below), it needs about n (12 d + (2 + S) bs e) bytes;
 * larger requests return MLG_ERR_RANGE and enqueue nothing.
 * The call only enqueues work on `stream` and returns: Y is ready once the
 * stream has reached that point.  Non-finite coordinates are not rejected
 * (they make the outputs NaN).  All calls on one device share the array, so
 * calls that can overlap on one device (other streams, other threads) race;
 * calls on one stream are ordered and safe.
 */
mlg_status mlg_kernel_matvec_noalloc(int64_t n, int d, const double *points, double sigma,
                                     const mlg_kparams *kp, int b, const double *X, int64_t ldx,
                                     double *Y, int64_t ldy, void *stream);

/* ---- measurement helpers ------------------------------------------------ */

/* Stages of one matvec, for mlg_profile_stages. */
#define MLG_STAGE_PRE 0     /* scatter-in: z_t = D_t^-1/2 x, sorted, cast (Sec. 2) */
#define MLG_STAGE_SPREAD 1  /* window spreading into bin patches, Alg. 1 step 1 */
#define MLG_STAGE_GATHER 2  /* patch sums onto the grid (part of spreading)     */
#define MLG_STAGE_FFT 3     /* forward FFT, multiply, inverse FFT (Alg. 1)      */
#define MLG_STAGE_INTERP 4  /* interpolation, Alg. 1 step 3 (part)              */
#define MLG_STAGE_POST 5    /* gather-out: self term, D^-1/2, layer mean, y     */
#define MLG_STAGE_DIRECT 6  /* direct tiled summation                          */
#define MLG_STAGE_IO 7      /* unused (kept for layout stability)               */
#define MLG_NSTAGES 8

/*
 * Run the matvec of mlg_laplacian_matvec `reps` times without a HIP graph,
 * with HIP events around every kernel on the graph's stream, and return the
 * average milliseconds per matvec spent in each stage (stage_ms has
 * MLG_NSTAGES entries, summed over layers).
 */
mlg_status mlg_profile_stages(mlg_graph *g, int layer, int op, int b, const double *X,
                              int64_t ldx, double *Y, int64_t ldy, int reps, double *stage_ms,
                              int flags);

/* Parameters each layer ended up with: 6 ints per layer
 * (d, N, window, bin, precision, method) and 2 doubles per layer
 * (scaled sigma, scale factor). */
mlg_status mlg_graph_layer_info(mlg_graph *g, int layer, int *iparams, double *dparams);

#ifdef __cplusplus
}
#endif
#endif /* MLG_H */
