// Internal data structures and launcher declarations of libmlg.so.
#pragma once

#include "common.h"

namespace mlg {

// Point-chunk capacity of one spreading task.
constexpr int kMaxTaskPoints = 256;

// NFFT plan of one layer (Algorithm 1 of Sec. 4): torus scaling, bin-sorted
// points, per-bin tasks, and the Fourier multipliers on the 2N grid.
struct NfftPlan {
    int d = 0, N = 0, nos = 0;  // bandwidth N, grid nos = 2N per dimension
    int B = 1;                  // bin edge (cells)
    int nb = 0;                 // bins per dimension = nos / B
    int64_t nbins = 0;
    double eps_B = 1.0 / 16, sigma_s = 0, scale = 1, center[3] = {0, 0, 0};
    int p_reg = 5;
    int64_t n = 0;
    DevBuf<int> perm;       // sorted position -> original index
    DevBuf<double> u64;     // d x n grid coordinates in sorted order, FP64
    DevBuf<int> c32;        // d x n grid cell of each sorted point
    DevBuf<float> f32;      // d x n offset inside that cell, FP32
    int nruns = 0;          // occupied bins
    int ntasks = 0;         // tasks (runs cut into chunks of <= kMaxTaskPoints)
    int nscratch = 0;       // task patches of runs with more than one task
    int nmulti = 0;         // runs with more than one task
    DevBuf<int4> tasks;     // (bin key, first point, count, destination patch slot)
    DevBuf<int4> multi;     // (run, first scratch slot, task count, 0)
    DevBuf<int> bin_run;    // per bin: run index or -1
    DevBuf<unsigned> run_key;   // per run: its bin key
    int nred1 = 0, nred2 = 0;
    DevBuf<int4> red1;      // level-1 groups (first slot, count <= 32, destination slot, 0)
    DevBuf<int4> red2;      // level-2, runs of > 1 group (run, first scratch slot, groups, 0)
    // Spreading schedule of the d = 3 matrix-core kernel: runs cut into tasks
    // of at most seg_chunks 64-point chunks (chosen per plan so the tasks
    // fill the device's slots evenly), larger tasks first.  Runs cut into
    // several tasks accumulate in scratch slots after the task list's
    // nscratch, summed by sred1/sred2 like red1/red2.
    int nseg = 0, seg_chunks = 0, nsscr = 0, nsred1 = 0, nsred2 = 0;
    DevBuf<int4> seg;       // (bin key, first point, count, destination patch slot)
    DevBuf<int4> sred1, sred2;
    // Interpolation schedule of the same kernel family: runs cut into tasks
    // of at most iseg_chunks chunks for three wavefronts per SIMD, larger
    // first; one workgroup per task.
    int niseg = 0, iseg_chunks = 0;
    DevBuf<int4> iseg;
    int SB = 8, nsb = 0;    // superbin edge (bins) and superbins per dimension
    DevBuf<unsigned char> occ;  // per superbin: 1 if occupied
    DevBuf<double> bhat;    // kernel Fourier coefficients b^_l, l in [0,N)^d (index l mod N)
    DevBuf<float2> tw32;    // exp(-2 pi i j / nos), j < nos/2
    DevBuf<double2> tw64;
};

// Multiplier set for one (window, precision) choice.
struct NfftWindow {
    int w = 0;           // window support, even
    double beta = 0;     // exponential-of-semicircle shape
    int prec = 32;
    DevBuf<float> M32;   // nos^d real multipliers
    DevBuf<double> M64;
    // grid cell -> patch entries (run * PD + cell offset), sorted; empty
    // when the table would be too large (the gather then walks the bins)
    bool csr = false;
    DevBuf<int> cell_ptr;   // nos^d + 1
    DevBuf<int> cell_ent;
};

struct Layer {
    int d = 0;
    double sigma = 0;
    mlg_kparams kp{};
    int64_t n = 0;
    // direct path: coordinates centred on the bounding box and scaled by
    // 1/sigma (x64) or sqrt(log2 e)/sigma (x32), SoA d x n
    DevBuf<double> x64;
    DevBuf<float> x32;
    NfftPlan nf;
    NfftWindow win;          // matvec window
    DevBuf<double> deg;      // degrees, original order
    DevBuf<double> dinv;     // D^-1/2, original order
    DevBuf<float> zsc;       // NFFT: D^-1/2 rounded to FP32, in bin order
    double deg_err = 0;      // NFFT: largest sampled absolute error of the degree pass
    double iso_thresh = 0;   // degrees <= this are isolated (MLG_ERR_ISOLATED)
};

// What the block entry/exit kernels need to know about one layer.
struct LayerIO {
    void *Z;                 // n x bs input of the summation (node order), float or double
    const void *F;           // n x bs output of the summation (node order)
    const double *dinv;      // D^-1/2, original order
    double K0;               // self term removed after the summation (0 for direct)
    int is64;
    // 1: the summation reads the shared FP32 slice of x and multiplies each
    // row by D^-1/2 rounded to FP32 itself (its input value is the FP32
    // product fl(x) fl(D^-1/2)); the entry kernel writes no slice for it
    int shared;
};

// ---- layer_ops.hip ----------------------------------------------------------
// X32: the shared FP32 slice of x (n x bs, node order) written once, or null.
void launch_scatter_in(int64_t n, int b, int bs, const double *X, int64_t ldx, const LayerIO *L,
                       int nl, int use_dinv, hipStream_t s, float *X32 = nullptr);
void launch_gather_out(int64_t n, int b, int bs, const double *X, int64_t ldx, double *Y,
                       int64_t ldy, const LayerIO *L, int nl, int use_dinv, int lsym, double coef,
                       hipStream_t s);
// Graph nodes captured from the two launches above: whether a kernel node is
// one of them, and re-pointing it at other X (and Y) blocks in an
// instantiated graph (same shapes and layer tables as when captured).
bool is_scatter_in_node(hipGraphNode_t node);
bool is_gather_out_node(hipGraphNode_t node);
void set_scatter_in_node(hipGraphExec_t e, hipGraphNode_t node, int64_t n, int b, int bs,
                         const double *X, int64_t ldx, const LayerIO *L, int nl, int use_dinv,
                         float *X32);
void set_gather_out_node(hipGraphExec_t e, hipGraphNode_t node, int64_t n, int b, int bs,
                         const double *X, int64_t ldx, double *Y, int64_t ldy, const LayerIO *L,
                         int nl, int use_dinv, int lsym, double coef);
void launch_fill_ones(int64_t n, double *Xr, hipStream_t s);
void launch_check_degrees(int64_t n, const double *deg, double thresh, int *flag, hipStream_t s);
void launch_dinv(int64_t n, const double *deg, double *dinv, hipStream_t s);
// dst[p] = (float)src[perm[p]].
void launch_sorted_f32(int64_t n, const int *perm, const double *src, float *dst, hipStream_t s);

// ---- direct.hip ---------------------------------------------------------------
// Scaled, centred coordinates of a direct layer (d x n SoA): x64 for the
// FP64 kernels, x32 for the FP32 kernels; kernel = MLG_KERNEL_*.
// Returns MLG_ERR_ARG if a coordinate is not finite.
void direct_coords(int64_t n, int d, const double *pts_dev, double sigma, int kernel,
                   DevBuf<double> &x64, DevBuf<float> &x32, hipStream_t s);
// The same into caller-provided buffers (mid: d doubles; x64, x32: n x d),
// enqueued only: no allocation, no wait.  A non-finite coordinate makes its
// dimension's midpoint NaN, and with it every coordinate of that dimension.
void direct_coords_into(int64_t n, int d, const double *pts_dev, double sigma, int kernel,
                        double *mid, double *x64, float *x32, hipStream_t s);
// Fs = W Zs (zero diagonal) for n points with coordinates from direct_coords;
// part: S x n x bs column-split partials (direct_part_size elements).
template <class T>
void launch_direct(int64_t n, int d, int kernel, const T *x, int bs, const T *Zs, T *Fs, T *part,
                   size_t part_cap, hipStream_t s);
template <class T>
size_t direct_part_size(int64_t n, int bs);

// ---- nfft.hip -----------------------------------------------------------------
void nfft_plan_layer(Layer &L, const double *pts_dev, hipStream_t s);
// Bandwidth of the automatic rule (N = 0) for a scaled sigma and precision.
int nfft_auto_bandwidth(double sigma_s, int d, int prec);
void nfft_make_window(const Layer &L, NfftWindow &W, int w, int prec, int bs, hipStream_t s);
size_t nfft_patch_elems(const NfftPlan &P, const NfftWindow &W, int bs);
size_t nfft_grid_elems(const NfftPlan &P, int bs);
// W~ applied to Zs (node order, T, stride bs) -> Fs; uses patch and grid
// workspaces.  With zsc (FP32 matrix-core path only, see
// nfft_scaled_input_ok), the summation input of point p (bin order) is row
// perm[p] of Zs times zsc[p], as an FP32 product.
template <class T>
void nfft_apply(const NfftPlan &P, const NfftWindow &W, int bs, const T *Zs, T *Fs, T *patch,
                T *grid, hipStream_t s, hipEvent_t *ev /* 5 events or null */,
                const float *zsc = nullptr);
bool nfft_scaled_input_ok(const NfftPlan &P, const NfftWindow &W, int bs);

// Several FP32 matrix-core NFFT layers of one dimension and patch edge run
// as one launch per stage (spreading, split-bin reductions, cell-table
// gather, interpolation; the FFT once per group of equal N): the layers'
// task lists are concatenated with a task -> layer map, patch slots and grid
// regions laid out one layer after another in buffers the batch owns.  Each
// layer's arithmetic is the per-layer path's, so results are the same bits.
struct NfftBatch {
    int D = 0, Pside = 0, bs = 0, bg = 0, nl = 0;
    std::vector<int> layers;       // graph layer of each batch layer (sorted by N)
    DevBuf<char> args, args_n;     // nl device LayerArgs: with D^-1/2 scaling, without
    DevBuf<int4> stasks;           // spreading tasks, destination slots global
    DevBuf<int> slayer;
    int nst = 0;
    DevBuf<int4> itasks;           // interpolation tasks
    DevBuf<int> ilayer;
    int nit = 0, isplit = 1, iper = 0;
    DevBuf<int4> red1, red2;
    int nred1 = 0, nred2 = 0;
    DevBuf<int> cptr, cent;        // concatenated cell tables
    DevBuf<int64_t> coff, goff;    // flat cell offsets (nl + 1), grid offsets (elements)
    std::vector<int64_t> goff_h;
    int64_t ncell = 0;
    struct Sub {                   // layers first .. first + count - 1 share N
        const NfftPlan *plan = nullptr;   // the first one's plan (N, grid, twiddles)
        int first = 0, count = 0;
        int64_t mstr = 0;
        DevBuf<float> M;           // their multipliers, one after another
    };
    std::vector<Sub> subs;
    DevBuf<float> patch, grid;
    size_t patch_elems = 0, grid_elems = 0;
};
// Build a batch of the given layers (all FP32 NFFT on the matrix-core path
// with a cell table, one D and patch edge) for block stride bs; Zs[i] / Fs[i]
// are layer i's summation slices.
// The batch reads the shared FP32 slice X32 and scales it by each layer's
// zsc (use_dinv) or not (two argument tables).
void nfft_batch_build(NfftBatch &B, const std::vector<const Layer *> &layers,
                      const std::vector<int> &ids, const float *X32,
                      const std::vector<float *> &Fs, int bs, hipStream_t s);
// Whether a layer can join a batch for block stride bs, and its (D, patch
// edge) key.
bool nfft_batchable(const Layer &L, int bs, int *key);
void nfft_batch_apply(const NfftBatch &B, int use_dinv, hipStream_t s);

// ---- lanczos.hip ----------------------------------------------------------------
struct Graph;
// Operator of the block eigensolver: Y = A X for b columns (device pointers,
// enqueued on the graph's stream), and the map from an eigenvalue mu of A to
// the Laplacian eigenvalue lambda it stands for.  The solver finds the
// largest mu.
struct LanczosOp {
    virtual ~LanczosOp() = default;
    virtual void apply(int b, const double *X, int64_t ldx, double *Y, int64_t ldy) = 0;
    virtual double lambda(double mu) const = 0;
};
mlg_status lanczos_run(Graph &g, LanczosOp &op, int k, int block, double tol, int max_restarts,
                       uint64_t seed, const double *V0_dev, double *evals_host,
                       double *evecs_dev, int64_t ldv, mlg_eig_info *info);

// ---- autotune.hip -------------------------------------------------------------
// out[r + v nrow] = sum_{j != rows[r]} exp(-||x_i - x_j||^2 / sigma^2) X[j + v ldx]
// in FP64 (one workgroup per row, fixed-order tree), d <= 3, device pointers.
void launch_ref_rows(int64_t n, int d, const double *pts, double sigma, const int64_t *rows,
                     int nrow, int b, const double *X, int64_t ldx, double *out, hipStream_t s);

// ---- pksm.hip -------------------------------------------------------------------
constexpr int kPksmMaxSteps = 128;      // Krylov dimension limit of the matrix power
constexpr int kPksmDefaultSteps = 128;
// Largest Krylov dimension whose tridiagonal eigensolve fits the LDS of one
// workgroup on the current device (<= kPksmMaxSteps).
int pksm_max_steps_device();
// Y = (L_sym^(t) + delta I)^p X (one layer) or the layer mean of these terms,
// p < 0, delta = log(1+|p|), by the polynomial Krylov method (Sec. 3).
// Workspace for b columns is allocated once per lane and reused by every
// apply; the Krylov basis grows on demand up to `max_steps` vectors.  The
// layers of different graph branches run side by side.
struct PowerMeanOp {
    Graph &g;
    int b;
    double p, delta = 0.0;
    double tol = 1e-12;        // stopping threshold on the change of f(T_m) e_1 / delta^p
    int mcap = 0;              // Krylov dimension limit
    int nrow = 0;              // blocks of the row-per-thread kernels
    // One Krylov run in flight: basis (grown on demand), work vectors,
    // coefficients, and the stream it runs on (one lane per graph branch).
    struct Lane {
        DevBuf<double> V, W, part, xn, al, be, C[2], chg;
        DevBuf<int> fail;
        int vcap = 0;          // basis slots allocated in V
        hipStream_t s = nullptr;
        hipEvent_t done = nullptr;
        std::vector<double> ch;
        std::vector<int> bad;
        int t = -1, m = 0, last = 1;
        bool conv = false, active = false;
    };
    std::vector<Lane> lanes;
    hipEvent_t free_ev = nullptr;
    int max_used = 0;          // longest Krylov dimension used so far
    int unconverged = 0;       // layer applications stopped at mcap
    int64_t layer_matvecs = 0; // single-vector layer matvecs
    PowerMeanOp(Graph &g, int b, double p, int max_steps);
    ~PowerMeanOp();
    PowerMeanOp(const PowerMeanOp &) = delete;
    PowerMeanOp &operator=(const PowerMeanOp &) = delete;
    bool fuse = false;         // next vector and the layer's summation input in one pass
    void scale_next(Lane &L, const double *X, int64_t ldx, const double *Q, const double *alpha,
                    const double *den, int dstride, double *Vnext);
    void prepare(Lane &L);
    void ensure_slots(Lane &L, int need);
    void start(Lane &L, int t, const double *X, int64_t ldx);
    void step(Lane &L, int j);
    void run(const std::vector<int> &ts, const double *X, int64_t ldx);
    void combine(Lane &L, double *Y, int64_t ldy, bool accumulate, double coef);
    void apply_layer(int t, const double *X, int64_t ldx, double *Y, int64_t ldy, bool accumulate,
                     double coef);
    // normalised: f / delta^p (spectrum in (0, 1]) instead of f.
    void apply(int layer, const double *X, int64_t ldx, double *Y, int64_t ldy, bool normalised);
};

// ---- ac.hip -------------------------------------------------------------------
void ac_run(int64_t n, int k, int m, const double *evals_dev, const double *evecs_dev,
            int64_t ldv, const int32_t *labels_dev, const mlg_ac_params &prm, double *U_dev,
            int32_t *pred_dev, int *iters, hipStream_t s);

// ---- features.hip ---------------------------------------------------------------
// Layer point arrays (device, n x d_t row-major) of T feature groups of the
// n x D row-major feature matrix (host or device): group t takes the columns
// group_cols[off_t .. off_t + d_t).
void gather_feature_groups(int64_t n, int D, const double *features, bool dev, int T,
                           const int *group_dim, const int *group_cols,
                           std::vector<DevBuf<double>> &pts);
// Median of the s (s - 1) / 2 pairwise distances of the sample rows over the
// columns cols (NULL: 0..d-1); even counts give the mean of the middle two.
double median_pair_distance(int64_t n, int D, const double *features, bool dev, int d,
                            const int *cols_host, int s, const int64_t *sample_host,
                            hipStream_t stream);

// ---- graph.hip ----------------------------------------------------------------
struct Graph {
    int64_t n = 0;
    int T = 0;
    bool has_degrees = true;
    hipStream_t stream = nullptr;
    std::vector<Layer> layers;
    // workspaces: per-layer slices of Zs/Fs (n x bs, the layer's precision);
    // summation scratch per branch: layer t uses branch t mod br.size(), and
    // the branches of an all-layer product run side by side (the main
    // stream and side[r - 1] for branch r), so each has its own patch, grid
    // and direct-path partials
    DevBuf<char> Zs, Fs;
    struct Scratch {
        DevBuf<char> patch, grid, part;
    };
    std::vector<Scratch> br;
    std::vector<hipStream_t> side;
    std::vector<hipEvent_t> fork_join;   // [0]: fork, [r]: join of branch r
    int ws_bs = 0;                 // block stride the slices are laid out for
    std::vector<size_t> slice;     // byte offset of layer t's slice
    DevBuf<LayerIO> io;            // device copy of the T layer descriptors (own slices)
    // the API's products: FP32 matrix-core NFFT layers read one shared FP32
    // slice of x (X32) and scale it per point themselves (shared[t]);
    // io_sh marks them.  The Krylov power keeps own slices (its layers run
    // different vectors at once).
    DevBuf<float> X32;
    std::vector<char> shared;
    DevBuf<LayerIO> io_sh;
    // all-layer products: batches of FP32 matrix-core layers (built for
    // block stride batch_bs) and the layers that run alone
    std::vector<NfftBatch> batches;
    std::vector<int> unbatched;
    int batch_bs = 0;
    // captured graphs keyed by (layer, op, b)
    struct Cap {
        int layer, op, b;
        hipGraphExec_t exec;
    };
    std::vector<Cap> caps;
    // whole products (entry kernel, layer summations, exit kernel) as one
    // captured graph per (layer, op, b); the entry and exit nodes are
    // re-pointed in the instantiated graph when X or Y change
    struct WholeCap {
        int layer, op, b;
        hipGraph_t graph;
        hipGraphExec_t exec;
        hipGraphNode_t in_node, out_node;
        const double *X;
        int64_t ldx;
        double *Y;
        int64_t ldy;
    };
    std::vector<WholeCap> whole;
    ~Graph();
};

// Enqueue Y = op X (device pointers) on g.stream.  With `ev` non-null,
// records stage events (see mlg_profile_stages).
void graph_matvec_enqueue(Graph &g, int layer, int op, int b, const double *X, int64_t ldx,
                          double *Y, int64_t ldy, double *stage_ms);
// The entry and summation part of that: scatter-in of X (with D^-1/2 when
// use_dinv) and the layers' summations, leaving F_t in the workspace slices
// described by the returned device descriptors (one for layer >= 0, T for
// -1; block stride = the next power of two >= b).  The caller enqueues its
// own exit kernel on the same stream: `stream`, or g.stream if null.  Two
// layers may be enqueued on different streams at once only if they belong
// to different branches (t mod graph_branches(g)).
// With scatter = false the entry kernel is skipped: the caller has written
// the layers' summation inputs itself (see graph_layer_io).
// With own = false the layers marked shared read the shared FP32 slice
// (the API's products); own = true keeps every layer on its own slice.
const LayerIO *graph_core_enqueue(Graph &g, int layer, int use_dinv, int b, const double *X,
                                  int64_t ldx, hipStream_t stream = nullptr, bool scatter = true,
                                  bool own = false);
// Device descriptor of layer t's slices for blocks of b vectors (workspace
// laid out for that block stride first).
const LayerIO *graph_layer_io(Graph &g, int b, int t);
// Stream of branch r (g.stream for r = 0; side streams created on demand).
hipStream_t graph_branch_stream(Graph &g, int r);
// Number of branches (layers t and t' share scratch iff t = t' mod this).
int graph_branches(const Graph &g);

}  // namespace mlg
