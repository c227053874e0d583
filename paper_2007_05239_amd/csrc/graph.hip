// The mlg_graph handle and the C ABI entry points (declared in include/mlg.h).
//
// A matvec with the layer mean (Sec. 3, eq. for I - L_1) or one layer's
// operator (Sec. 2) runs as
//   scatter-in: z_t = D_t^-1/2 x for every layer, in node order
//               and summation precision;
//   per layer:  F_t = W~_t z_t (NFFT, Algorithm 1) or W_t z_t (direct);
//   gather-out: y = coef sum_t D_t^-1/2 (F_t - K(0) z_t) in FP64 (y = x - that
//               for L_sym / L_1), written column-major.
// The per-layer part is captured once into a HIP graph and replayed.
#include <algorithm>
#include <cmath>
#include <memory>

#include "internal.h"

namespace mlg {

static thread_local std::string g_last_error;
void set_last_error(const std::string &msg) { g_last_error = msg; }

// Instantiated graphs refer to the workspaces; they go whenever those move.
static void drop_captures(Graph &g) {
    for (auto &c : g.caps) (void)hipGraphExecDestroy(c.exec);
    g.caps.clear();
    for (auto &w : g.whole) {
        (void)hipGraphExecDestroy(w.exec);
        (void)hipGraphDestroy(w.graph);
    }
    g.whole.clear();
}

Graph::~Graph() {
    drop_captures(*this);
    if (stream) (void)hipStreamSynchronize(stream);
    for (hipStream_t q : side) {
        (void)hipStreamSynchronize(q);
        (void)hipStreamDestroy(q);
    }
    for (hipEvent_t e : fork_join) (void)hipEventDestroy(e);
}

// Concurrent branches of an all-layer product (at most this many layers'
// summations in flight).
constexpr int kMaxBranches = 3;

static int block_stride(int b) {
    int bs = 1;
    while (bs < b) bs <<= 1;
    return bs;
}

static int default_window(const Layer &L) {
    if (L.kp.window > 0) return L.kp.window;
    return L.kp.precision == 64 ? 12 : 6;
}

// Widest even window the plan admits (bin + w/2 <= N/2, bin + w - 1 <= 20).
static int max_window(const NfftPlan &P) {
    int w = 2 * (P.N / 2 - P.B);
    w = std::min(w, 21 - P.B);
    w = std::min(w, 16);
    return w & ~1;
}

// Per-layer workspace slices: Zs/Fs hold n x bs values of each layer's
// precision; patch, grid and partials per branch, sized for its layers.
static void ensure_ws(Graph &g, int bs) {
    const int nb = std::min(g.T, kMaxBranches);
    size_t zs = 0;
    std::vector<size_t> patch(nb, 0), grid(nb, 0), part(nb, 0);
    std::vector<size_t> slice(g.T);
    for (int t = 0; t < g.T; ++t) {
        const Layer &L = g.layers[t];
        const int r = t % nb;
        const size_t esz = L.kp.precision == 64 ? 8 : 4;
        slice[t] = zs;
        zs += ((size_t)g.n * bs * esz + 255) / 256 * 256;
        if (L.kp.method == MLG_METHOD_NFFT) {
            patch[r] = std::max(patch[r], nfft_patch_elems(L.nf, L.win, bs) * esz);
            grid[r] = std::max(grid[r], nfft_grid_elems(L.nf, bs) * esz);
        } else {
            size_t ps = esz == 8 ? direct_part_size<double>(g.n, bs) : direct_part_size<float>(g.n, bs);
            part[r] = std::max(part[r], ps * esz);
        }
    }
    if ((int)g.br.size() != nb) {
        drop_captures(g);
        g.br.clear();
        g.br.resize(nb);
        g.ws_bs = 0;
    }
    // layers that read the shared FP32 slice of x in the API's products
    std::vector<char> shared(g.T, 0);
    bool any_shared = false;
    for (int t = 0; t < g.T; ++t) {
        const Layer &L = g.layers[t];
        shared[t] = L.kp.method == MLG_METHOD_NFFT && L.kp.precision == 32 &&
                    nfft_scaled_input_ok(L.nf, L.win, bs) && (!g.has_degrees || L.zsc.p);
        any_shared |= shared[t] != 0;
    }
    std::vector<void *> before{g.Zs.p, g.Fs.p, g.X32.p};
    for (auto &w : g.br) before.insert(before.end(), {w.patch.p, w.grid.p, w.part.p});
    g.Zs.ensure(zs);
    g.Fs.ensure(zs);
    if (any_shared) g.X32.ensure((size_t)g.n * bs);
    for (int r = 0; r < nb; ++r) {
        g.br[r].patch.ensure(patch[r]);
        g.br[r].grid.ensure(grid[r]);
        g.br[r].part.ensure(part[r]);
    }
    std::vector<void *> after{g.Zs.p, g.Fs.p, g.X32.p};
    for (auto &w : g.br) after.insert(after.end(), {w.patch.p, w.grid.p, w.part.p});
    const bool moved = g.ws_bs != bs || before != after;
    if (!moved) return;
    drop_captures(g);
    g.batches.clear();
    g.unbatched.clear();
    g.batch_bs = 0;
    g.slice = slice;
    g.ws_bs = bs;
    std::vector<LayerIO> io(g.T);
    for (int t = 0; t < g.T; ++t) {
        const Layer &L = g.layers[t];
        io[t].Z = g.Zs.p + slice[t];
        io[t].F = g.Fs.p + slice[t];
        io[t].dinv = L.dinv.p;
        io[t].K0 = L.kp.method == MLG_METHOD_NFFT ? 1.0 : 0.0;
        io[t].is64 = L.kp.precision == 64;
        io[t].shared = 0;
    }
    g.io.alloc(g.T);
    MLG_HIP(hipMemcpyAsync(g.io.p, io.data(), sizeof(LayerIO) * g.T, hipMemcpyHostToDevice, g.stream));
    g.shared = shared;
    for (int t = 0; t < g.T; ++t) io[t].shared = shared[t];
    g.io_sh.alloc(g.T);
    MLG_HIP(hipMemcpyAsync(g.io_sh.p, io.data(), sizeof(LayerIO) * g.T, hipMemcpyHostToDevice,
                           g.stream));
    MLG_HIP(hipStreamSynchronize(g.stream));
}

struct StageTimer {
    hipEvent_t ev[8];
    double *acc;
};

// F_t = W~ z_t (NFFT) or W z_t (direct) for one layer, in its slices, on
// stream s with the scratch of the layer's branch.
// How the summations read their input: own slices, or (sh) the shared FP32
// slice for the layers marked shared, scaled by D^-1/2 when use_dinv.
struct InMode {
    bool sh = false;
    int use_dinv = 1;
};

template <class T>
static void layer_core(Graph &g, int t, int bs, StageTimer *tm, hipStream_t s, InMode md) {
    Layer &L = g.layers[t];
    Graph::Scratch &w = g.br[t % g.br.size()];
    const bool sh = md.sh && g.shared[t];
    T *Zs = sh ? reinterpret_cast<T *>(g.X32.p) : reinterpret_cast<T *>(g.Zs.p + g.slice[t]);
    T *Fs = reinterpret_cast<T *>(g.Fs.p + g.slice[t]);
    float ms = 0.f;
    if (tm) MLG_HIP(hipEventRecord(tm->ev[5], s));
    if (L.kp.method == MLG_METHOD_NFFT) {
        nfft_apply<T>(L.nf, L.win, bs, Zs, Fs, reinterpret_cast<T *>(w.patch.p),
                      reinterpret_cast<T *>(w.grid.p), s, tm ? tm->ev : nullptr,
                      sh && md.use_dinv ? L.zsc.p : nullptr);
    } else {
        const T *x = nullptr;
        if constexpr (sizeof(T) == 8) x = L.x64.p; else x = L.x32.p;
        launch_direct<T>(g.n, L.d, L.kp.kernel, x, bs, Zs, Fs,
                         reinterpret_cast<T *>(w.part.p), w.part.n / sizeof(T), s);
        if (tm) MLG_HIP(hipEventRecord(tm->ev[4], s));
    }
    if (tm) {
        MLG_HIP(hipStreamSynchronize(s));
        if (L.kp.method == MLG_METHOD_NFFT) {
            MLG_HIP(hipEventElapsedTime(&ms, tm->ev[5], tm->ev[1]));
            tm->acc[MLG_STAGE_SPREAD] += ms;
            MLG_HIP(hipEventElapsedTime(&ms, tm->ev[1], tm->ev[2]));
            tm->acc[MLG_STAGE_GATHER] += ms;
            MLG_HIP(hipEventElapsedTime(&ms, tm->ev[2], tm->ev[3]));
            tm->acc[MLG_STAGE_FFT] += ms;
            MLG_HIP(hipEventElapsedTime(&ms, tm->ev[3], tm->ev[4]));
            tm->acc[MLG_STAGE_INTERP] += ms;
        } else {
            MLG_HIP(hipEventElapsedTime(&ms, tm->ev[5], tm->ev[4]));
            tm->acc[MLG_STAGE_DIRECT] += ms;
        }
    }
}

static void core_layer(Graph &g, int t, int bs, StageTimer *tm, hipStream_t s, InMode md) {
    if (g.layers[t].kp.precision == 64)
        layer_core<double>(g, t, bs, tm, s, md);
    else
        layer_core<float>(g, t, bs, tm, s, md);
}

int graph_branches(const Graph &g) { return std::min(g.T, kMaxBranches); }

// Largest patch buffer of a layer that may join a batch (a batch holds the
// patches of all its layers at once).
constexpr size_t kBatchPatchBytes = (size_t)512 << 20;

// Batches of the all-layer product for block stride bs: layers with the
// same batch key (FP32 matrix-core NFFT, one dimension and patch edge) run
// together when more of them share it than there are branches.  (A few
// large layers do better as parallel branches, where one layer's short
// gather, reduction and FFT kernels overlap another's matrix-core kernels;
// many small layers do better as one launch per stage.)  Built outside any
// stream capture.
static void ensure_batches(Graph &g, int bs) {
    if (g.batch_bs == bs) return;
    g.batches.clear();
    g.unbatched.clear();
    std::vector<int> key(g.T, -1);
    for (int t = 0; t < g.T; ++t) {
        const Layer &L = g.layers[t];
        int k = -1;
        if (g.shared[t] && nfft_batchable(L, bs, &k) &&
            nfft_patch_elems(L.nf, L.win, bs) * 4 <= kBatchPatchBytes)
            key[t] = k;
    }
    std::vector<bool> done(g.T, false);
    for (int t = 0; t < g.T; ++t) {
        if (done[t]) continue;
        std::vector<int> members;
        if (key[t] >= 0)
            for (int u = t; u < g.T; ++u)
                if (!done[u] && key[u] == key[t]) members.push_back(u);
        if ((int)members.size() <= kMaxBranches) {
            g.unbatched.push_back(t);
            done[t] = true;
            continue;
        }
        std::vector<const Layer *> ls;
        std::vector<float *> fs;
        for (int u : members) {
            done[u] = true;
            ls.push_back(&g.layers[u]);
            fs.push_back(reinterpret_cast<float *>(g.Fs.p + g.slice[u]));
        }
        g.batches.emplace_back();
        nfft_batch_build(g.batches.back(), ls, members, g.X32.p, fs, bs, g.stream);
    }
    std::sort(g.unbatched.begin(), g.unbatched.end());
    g.batch_bs = bs;
}

// Stream of branch r: g.stream for r = 0, else side stream r - 1 (created
// on first use, default priority).
hipStream_t graph_branch_stream(Graph &g, int r) {
    if (r == 0) return g.stream;
    while ((int)g.side.size() < r) {
        hipStream_t q;
        MLG_HIP(hipStreamCreateWithFlags(&q, hipStreamNonBlocking));
        g.side.push_back(q);
    }
    return g.side[r - 1];
}

// All layers (layer = -1) or one.  With `fork`, the branches of an
// all-layer product are enqueued on their own streams after an event on
// g.stream and joined back into it (used under stream capture, where this
// makes parallel branches of the captured graph); otherwise in layer order
// on stream s (g.stream if null).
static void core(Graph &g, int layer, int bs, StageTimer *tm, InMode md, bool fork = false,
                 hipStream_t s = nullptr) {
    const int nb = (int)g.br.size();
    // all-layer products on the shared slice (not stage-timed) run their
    // batches, one launch per stage for all of a batch's layers; stage
    // timing walks the layers
    const bool batched = layer < 0 && md.sh && !tm && g.batch_bs == bs && !g.batches.empty();
    if (batched && (!fork || nb < 2)) {
        hipStream_t q = s ? s : g.stream;
        for (const NfftBatch &B : g.batches) nfft_batch_apply(B, md.use_dinv, q);
        for (int t : g.unbatched) core_layer(g, t, bs, nullptr, q, md);
        return;
    }
    if (!fork || layer >= 0 || nb < 2) {
        for (int t = 0; t < g.T; ++t)
            if (layer < 0 || t == layer) core_layer(g, t, bs, tm, s ? s : g.stream, md);
        return;
    }
    for (int r = 1; r < nb; ++r) graph_branch_stream(g, r);
    while ((int)g.fork_join.size() < nb) {
        hipEvent_t e;
        MLG_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        g.fork_join.push_back(e);
    }
    MLG_HIP(hipEventRecord(g.fork_join[0], g.stream));
    for (int r = 1; r < nb; ++r) MLG_HIP(hipStreamWaitEvent(g.side[r - 1], g.fork_join[0], 0));
    if (batched) {
        // batch k on branch k mod nb; a layer alone on branch t mod nb, whose
        // scratch it uses (the batches own theirs)
        for (size_t k = 0; k < g.batches.size(); ++k) {
            const int r = (int)(k % nb);
            nfft_batch_apply(g.batches[k], md.use_dinv, r == 0 ? g.stream : g.side[r - 1]);
        }
        for (int t : g.unbatched) {
            const int r = t % nb;
            core_layer(g, t, bs, nullptr, r == 0 ? g.stream : g.side[r - 1], md);
        }
    } else {
        for (int t = 0; t < g.T; ++t) {
            const int r = t % nb;
            core_layer(g, t, bs, tm, r == 0 ? g.stream : g.side[r - 1], md);
        }
    }
    for (int r = 1; r < nb; ++r) {
        MLG_HIP(hipEventRecord(g.fork_join[r], g.side[r - 1]));
        MLG_HIP(hipStreamWaitEvent(g.stream, g.fork_join[r], 0));
    }
}

static void check_op(const Graph &g, int layer, int op, int b) {
    MLG_REQUIRE(layer >= -1 && layer < g.T, MLG_ERR_ARG, "layer out of range");
    MLG_REQUIRE(op == MLG_OP_NADJ || op == MLG_OP_LSYM || op == MLG_OP_W, MLG_ERR_ARG, "bad op");
    MLG_REQUIRE(op == MLG_OP_W || g.has_degrees, MLG_ERR_ARG,
                "graph created with MLG_SKIP_DEGREES serves MLG_OP_W only");
    MLG_REQUIRE(!(op == MLG_OP_W && layer < 0), MLG_ERR_ARG, "MLG_OP_W needs one layer");
    MLG_REQUIRE(b >= 1 && b <= 64, MLG_ERR_ARG, "b must be in 1..64");
}

void graph_matvec_enqueue(Graph &g, int layer, int op, int b, const double *X, int64_t ldx,
                          double *Y, int64_t ldy, double *stage_ms) {
    check_op(g, layer, op, b);
    const int bs = block_stride(b);
    ensure_ws(g, bs);
    hipStream_t s = g.stream;
    const LayerIO *io = layer >= 0 ? g.io_sh.p + layer : g.io_sh.p;
    const int nl = layer >= 0 ? 1 : g.T;
    const int use_dinv = op != MLG_OP_W;
    const double coef = layer < 0 ? 1.0 / g.T : 1.0;
    bool need32 = false;
    for (int t = 0; t < g.T; ++t) need32 |= (layer < 0 || t == layer) && g.shared[t];
    float *X32 = need32 ? g.X32.p : nullptr;
    InMode md;
    md.sh = true;
    md.use_dinv = use_dinv;
    if (stage_ms) {
        StageTimer tm;
        tm.acc = stage_ms;
        for (auto &e : tm.ev) MLG_HIP(hipEventCreate(&e));
        float ms;
        MLG_HIP(hipEventRecord(tm.ev[6], s));
        launch_scatter_in(g.n, b, bs, X, ldx, io, nl, use_dinv, s, X32);
        MLG_HIP(hipEventRecord(tm.ev[7], s));
        MLG_HIP(hipStreamSynchronize(s));
        MLG_HIP(hipEventElapsedTime(&ms, tm.ev[6], tm.ev[7]));
        stage_ms[MLG_STAGE_PRE] += ms;
        core(g, layer, bs, &tm, md);
        MLG_HIP(hipEventRecord(tm.ev[6], s));
        launch_gather_out(g.n, b, bs, X, ldx, Y, ldy, io, nl, use_dinv, op == MLG_OP_LSYM, coef, s);
        MLG_HIP(hipEventRecord(tm.ev[7], s));
        MLG_HIP(hipStreamSynchronize(s));
        MLG_HIP(hipEventElapsedTime(&ms, tm.ev[6], tm.ev[7]));
        stage_ms[MLG_STAGE_POST] += ms;
        for (auto &e : tm.ev) (void)hipEventDestroy(e);
        return;
    }
    // entry kernel, layer summations and exit kernel as one graph launch
    if (layer < 0) ensure_batches(g, bs);
    Graph::WholeCap *w = nullptr;
    for (auto &c : g.whole)
        if (c.layer == layer && c.op == op && c.b == b) w = &c;
    if (!w) {
        hipGraph_t graph;
        MLG_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        try {
            launch_scatter_in(g.n, b, bs, X, ldx, io, nl, use_dinv, s, X32);
            core(g, layer, bs, nullptr, md, true, s);
            launch_gather_out(g.n, b, bs, X, ldx, Y, ldy, io, nl, use_dinv, op == MLG_OP_LSYM, coef, s);
        } catch (...) {
            hipGraph_t junk = nullptr;
            (void)hipStreamEndCapture(s, &junk);
            if (junk) (void)hipGraphDestroy(junk);
            throw;
        }
        MLG_HIP(hipStreamEndCapture(s, &graph));
        size_t cnt = 0;
        hipError_t e = hipGraphGetNodes(graph, nullptr, &cnt);
        std::vector<hipGraphNode_t> nodes(cnt);
        if (e == hipSuccess) e = hipGraphGetNodes(graph, nodes.data(), &cnt);
        hipGraphNode_t in = nullptr, out = nullptr;
        for (size_t i = 0; e == hipSuccess && i < cnt; ++i) {
            if (is_scatter_in_node(nodes[i])) in = nodes[i];
            if (is_gather_out_node(nodes[i])) out = nodes[i];
        }
        hipGraphExec_t exec = nullptr;
        if (e == hipSuccess && (!in || !out)) e = hipErrorInvalidValue;
        if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(graph);
            MLG_HIP(e);
        }
        g.whole.push_back({layer, op, b, graph, exec, in, out, X, ldx, Y, ldy});
        w = &g.whole.back();
    } else if (w->X != X || w->ldx != ldx || w->Y != Y || w->ldy != ldy) {
        set_scatter_in_node(w->exec, w->in_node, g.n, b, bs, X, ldx, io, nl, use_dinv, X32);
        set_gather_out_node(w->exec, w->out_node, g.n, b, bs, X, ldx, Y, ldy, io, nl, use_dinv,
                            op == MLG_OP_LSYM, coef);
        w->X = X;
        w->ldx = ldx;
        w->Y = Y;
        w->ldy = ldy;
    }
    MLG_HIP(hipGraphLaunch(w->exec, s));
}

const LayerIO *graph_layer_io(Graph &g, int b, int t) {
    MLG_REQUIRE(t >= 0 && t < g.T && b >= 1 && b <= 64, MLG_ERR_ARG, "layer or block out of range");
    ensure_ws(g, block_stride(b));
    return g.io.p + t;
}

const LayerIO *graph_core_enqueue(Graph &g, int layer, int use_dinv, int b, const double *X,
                                  int64_t ldx, hipStream_t stream, bool scatter, bool own) {
    MLG_REQUIRE(layer >= -1 && layer < g.T, MLG_ERR_ARG, "layer out of range");
    MLG_REQUIRE(b >= 1 && b <= 64, MLG_ERR_ARG, "b must be in 1..64");
    const int bs = block_stride(b);
    ensure_ws(g, bs);
    hipStream_t s = stream ? stream : g.stream;
    const LayerIO *iob = own ? g.io.p : g.io_sh.p;
    const LayerIO *io = layer >= 0 ? iob + layer : iob;
    const int nl = layer >= 0 ? 1 : g.T;
    InMode md;
    md.sh = !own;
    md.use_dinv = use_dinv;
    bool need32 = false;
    for (int t = 0; t < g.T; ++t) need32 |= !own && (layer < 0 || t == layer) && g.shared[t];
    if (layer < 0 && !own) ensure_batches(g, bs);
    if (scatter) launch_scatter_in(g.n, b, bs, X, ldx, io, nl, use_dinv, s, need32 ? g.X32.p : nullptr);
    // captured launch sequences keyed by (layer, input mode, b)
    const int mode = (own ? 0 : 2) + (use_dinv ? 1 : 0);
    hipGraphExec_t exec = nullptr;
    for (auto &c : g.caps)
        if (c.layer == layer && c.op == mode && c.b == bs) exec = c.exec;
    if (!exec) {
        hipGraph_t graph;
        MLG_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        try {
            core(g, layer, bs, nullptr, md, s == g.stream, s);
        } catch (...) {
            hipGraph_t junk = nullptr;
            (void)hipStreamEndCapture(s, &junk);
            if (junk) (void)hipGraphDestroy(junk);
            throw;
        }
        MLG_HIP(hipStreamEndCapture(s, &graph));
        hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        MLG_HIP(e);
        g.caps.push_back({layer, mode, bs, exec});
    }
    MLG_HIP(hipGraphLaunch(exec, s));
    return io;
}

// Patch bytes above which the degree pass takes a larger bin.
constexpr double kDegPatchBytes = 2.0 * (1 << 30);
// Rows sampled to measure the degree pass's error, and the margin of the
// isolation threshold over the largest sampled error.
constexpr int kDegSampleRows = 64;
constexpr double kDegMargin = 64.0;

// Degrees deg = W 1 in FP64 (Sec. 2).  NFFT layers take a plan of their own
// for this one product: bandwidth from the FP64 tail rule (at least the
// layer's own), FP64 window of width 14, the smallest bin whose patches fit
// kDegPatchBytes.  Its error is then measured on kDegSampleRows rows against
// the FP64 direct sum of those rows, and a degree at or below kDegMargin times
// that error (the pass cannot tell it from zero) is MLG_ERR_ISOLATED.  Direct
// layers sum exactly up to rounding; there only a zero degree is isolated.
static void compute_degrees(Graph &g, Layer &L, const double *pts) {
    hipStream_t s = g.stream;
    const int64_t n = g.n;
    DevBuf<double> ones(n), Z(n), F(n);
    launch_fill_ones(n, ones.p, s);
    L.deg.alloc(n);
    LayerIO io{};
    io.Z = Z.p;
    io.F = F.p;
    io.dinv = nullptr;
    io.is64 = 1;
    DevBuf<LayerIO> dio(1);
    double thresh = 0.0;
    if (L.kp.method == MLG_METHOD_NFFT) {
        Layer Ld;
        Ld.d = L.d;
        Ld.sigma = L.sigma;
        Ld.n = n;
        Ld.kp = L.kp;
        Ld.kp.precision = 64;
        Ld.kp.N = std::max(L.nf.N, nfft_auto_bandwidth(L.nf.sigma_s, L.d, 64));
        // bin 1 unless its patches are too large and a larger bin still admits
        // a window of at least 10
        auto deg_window = [&](int B) {
            int w = std::min(14, max_window(Ld.nf));
            // the one-vector spreading holds a patch of at most 4096 cells
            // (16^3 in d = 3): bin + w - 1 <= 16
            if (L.d == 3) w = std::min(w, (16 - B + 1) & ~1);
            return w;
        };
        auto patch_bytes = [&](int B, int w) {
            double cells = 1.0;
            for (int t = 0; t < L.d; ++t) cells *= (double)(B + w - 1);
            return cells * 8.0 * (double)(Ld.nf.nruns + Ld.nf.nscratch);
        };
        Ld.kp.bin = 1;
        nfft_plan_layer(Ld, pts, s);
        int wdeg = deg_window(1);
        for (int B = 2; B <= 4 && patch_bytes(Ld.nf.B, wdeg) > kDegPatchBytes; B *= 2) {
            if (B / 2 + 5 > Ld.nf.N / 2) break;   // bin + 10/2 <= N/2 needed
            Ld.kp.bin = B;
            nfft_plan_layer(Ld, pts, s);
            wdeg = deg_window(B);
        }
        NfftWindow Wd;
        nfft_make_window(Ld, Wd, wdeg, 64, 1, s);
        io.K0 = 1.0;
        MLG_HIP(hipMemcpyAsync(dio.p, &io, sizeof(io), hipMemcpyHostToDevice, s));
        launch_scatter_in(n, 1, 1, ones.p, n, dio.p, 1, 0, s);
        DevBuf<double> patch(nfft_patch_elems(Ld.nf, Wd, 1)), grid(nfft_grid_elems(Ld.nf, 1));
        nfft_apply<double>(Ld.nf, Wd, 1, Z.p, F.p, patch.p, grid.p, s, nullptr);
        launch_gather_out(n, 1, 1, ones.p, n, L.deg.p, n, dio.p, 1, 0, 0, 1.0, s);
        // measured error on evenly spaced rows
        const int ns = (int)std::min<int64_t>(n, kDegSampleRows);
        std::vector<int64_t> rows(ns);
        for (int k = 0; k < ns; ++k) rows[k] = (int64_t)((double)k * (double)n / ns);
        DevBuf<int64_t> drows;
        upload(drows, rows.data(), rows.size(), false, s);
        DevBuf<double> ref(ns);
        launch_ref_rows(n, L.d, pts, L.sigma, drows.p, ns, 1, ones.p, n, ref.p, s);
        std::vector<double> href(ns);
        MLG_HIP(hipMemcpyAsync(href.data(), ref.p, sizeof(double) * ns, hipMemcpyDeviceToHost, s));
        std::vector<double> got(ns);
        for (int k = 0; k < ns; ++k)
            MLG_HIP(hipMemcpyAsync(&got[k], L.deg.p + rows[k], 8, hipMemcpyDeviceToHost, s));
        MLG_HIP(hipStreamSynchronize(s));
        double err = 0.0, typ = 0.0;
        for (int k = 0; k < ns; ++k) {
            err = std::max(err, std::fabs(got[k] - href[k]));
            typ = std::max(typ, href[k]);
        }
        L.deg_err = err;
        // FP64 rounding floor of an n-term sum of weights <= 1
        thresh = kDegMargin * std::max(err, 1e-16 * std::max(typ, 1.0));
    } else {
        io.K0 = 0.0;
        MLG_HIP(hipMemcpyAsync(dio.p, &io, sizeof(io), hipMemcpyHostToDevice, s));
        launch_scatter_in(n, 1, 1, ones.p, n, dio.p, 1, 0, s);
        DevBuf<double> part(direct_part_size<double>(n, 1));
        launch_direct<double>(n, L.d, L.kp.kernel, L.x64.p, 1, Z.p, F.p, part.p,
                              part.n, s);
        launch_gather_out(n, 1, 1, ones.p, n, L.deg.p, n, dio.p, 1, 0, 0, 1.0, s);
        MLG_HIP(hipStreamSynchronize(s));
        L.deg_err = 0.0;
    }
    L.iso_thresh = thresh;
    DevBuf<int> flag(1);
    MLG_HIP(hipMemsetAsync(flag.p, 0, 4, s));
    launch_check_degrees(n, L.deg.p, thresh, flag.p, s);
    int hf = 0;
    MLG_HIP(hipMemcpyAsync(&hf, flag.p, 4, hipMemcpyDeviceToHost, s));
    MLG_HIP(hipStreamSynchronize(s));
    MLG_REQUIRE(hf == 0, MLG_ERR_ISOLATED,
                "a node has zero degree (isolated) in some layer: degree <= " +
                    std::to_string(thresh) + (L.kp.method == MLG_METHOD_NFFT
                                                  ? " (the degree pass's measured error margin)"
                                                  : ""));
    L.dinv.alloc(n);
    launch_dinv(n, L.deg.p, L.dinv.p, s);
    if (L.kp.method == MLG_METHOD_NFFT) {
        // D^-1/2 in the layer's bin order, FP32: the factor its matrix-core
        // spreading applies to the shared slice of x
        L.zsc.alloc(n);
        launch_sorted_f32(n, L.nf.perm.p, L.dinv.p, L.zsc.p, s);
    }
    MLG_HIP(hipStreamSynchronize(s));
}

static void build_layer(Graph &g, Layer &L, const double *pts, bool dev, bool degrees) {
    hipStream_t s = g.stream;
    const int64_t n = g.n;
    DevBuf<double> pd;
    const double *p = pts;
    if (!dev) {
        upload(pd, pts, (size_t)n * L.d, false, s);
        p = pd.p;
    }
    L.n = n;
    if (L.kp.method == MLG_METHOD_DIRECT) direct_coords(n, L.d, p, L.sigma, L.kp.kernel, L.x64, L.x32, s);
    if (L.kp.method == MLG_METHOD_NFFT) {
        nfft_plan_layer(L, p, s);
        int w = default_window(L);
        nfft_make_window(L, L.win, w, L.kp.precision, 1, s);
    }
    MLG_HIP(hipStreamSynchronize(s));
    if (degrees) compute_degrees(g, L, p);
}

static hipStream_t make_stream(void *user) {
    if (user) return (hipStream_t)user;
    hipStream_t s;
    MLG_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    return s;
}

}  // namespace mlg

using namespace mlg;

struct mlg_graph {
    mlg::Graph g;
    bool own_stream = false;
};

template <class F>
static mlg_status guard(F f) {
    try {
        set_last_error("");
        f();
        return MLG_OK;
    } catch (const mlg::Error &e) {
        set_last_error(e.what());
        return e.code;
    } catch (const std::exception &e) {
        set_last_error(e.what());
        return MLG_ERR_HIP;
    }
}

extern "C" {

const char *mlg_last_error(void) { return mlg::g_last_error.c_str(); }

const char *mlg_version(void) { return "mlg 0.1 (gfx950)"; }

static mlg_status create_graph(mlg_graph **out, int64_t n, int T, const int *d,
                               const double *const *points, const double *sigma,
                               const mlg_kparams *kp, int flags, void *stream, bool degrees) {
    return guard([&] {
        MLG_REQUIRE(out && d && points && sigma && kp, MLG_ERR_ARG, "null argument");
        *out = nullptr;
        MLG_REQUIRE(n >= 2, MLG_ERR_ARG, "n must be >= 2");
        MLG_REQUIRE(T >= 1 && T <= 1024, MLG_ERR_ARG, "T must be in 1..1024");
        for (int t = 0; t < T; ++t) {
            MLG_REQUIRE(points[t], MLG_ERR_ARG, "null point array");
            MLG_REQUIRE(sigma[t] > 0 && std::isfinite(sigma[t]), MLG_ERR_RANGE, "sigma must be > 0");
            MLG_REQUIRE(kp[t].method == MLG_METHOD_DIRECT || kp[t].method == MLG_METHOD_NFFT,
                        MLG_ERR_ARG, "bad method");
            MLG_REQUIRE(kp[t].precision == 32 || kp[t].precision == 64, MLG_ERR_ARG,
                        "precision must be 32 or 64");
            MLG_REQUIRE(kp[t].kernel == MLG_KERNEL_GAUSSIAN || kp[t].kernel == MLG_KERNEL_LAPLACIAN,
                        MLG_ERR_ARG, "bad kernel");
            MLG_REQUIRE(kp[t].method == MLG_METHOD_DIRECT || kp[t].kernel == MLG_KERNEL_GAUSSIAN,
                        MLG_ERR_NOT_IMPL,
                        "the Laplacian RBF kernel runs on the direct path only (its cusp at the "
                        "origin needs a near-field correction that Algorithm 1 does not have)");
            if (kp[t].method == MLG_METHOD_NFFT)
                MLG_REQUIRE(d[t] >= 1 && d[t] <= 3, MLG_ERR_RANGE, "NFFT layers need d in 1..3");
            else
                MLG_REQUIRE(d[t] >= 1 && d[t] <= 16, MLG_ERR_RANGE, "direct layers need d in 1..16");
        }
        std::unique_ptr<mlg_graph> h(new mlg_graph());
        h->own_stream = stream == nullptr;
        h->g.stream = make_stream(stream);
        h->g.n = n;
        h->g.T = T;
        h->g.has_degrees = degrees;
        h->g.layers.resize(T);
        try {
            for (int t = 0; t < T; ++t) {
                Layer &L = h->g.layers[t];
                L.d = d[t];
                L.sigma = sigma[t];
                L.kp = kp[t];
                build_layer(h->g, L, points[t], (flags & MLG_DEVICE_PTRS) != 0, degrees);
            }
        } catch (...) {
            hipStream_t s = h->g.stream;
            bool own = h->own_stream;
            h.reset();
            if (own) (void)hipStreamDestroy(s);
            throw;
        }
        *out = h.release();
    });
}

mlg_status mlg_graph_create(mlg_graph **out, int64_t n, int T, const int *d,
                            const double *const *points, const double *sigma,
                            const mlg_kparams *kp, int flags, void *stream) {
    return create_graph(out, n, T, d, points, sigma, kp, flags, stream,
                        (flags & MLG_SKIP_DEGREES) == 0);
}

mlg_status mlg_graph_create_grouped(mlg_graph **out, int64_t n, int D, const double *features,
                                    int T, const int *group_dim, const int *group_cols,
                                    const double *sigma, const mlg_kparams *kp, int flags,
                                    void *stream) {
    std::vector<DevBuf<double>> pts;
    mlg_status st = guard([&] {
        MLG_REQUIRE(out, MLG_ERR_ARG, "null argument");
        *out = nullptr;
        gather_feature_groups(n, D, features, (flags & MLG_DEVICE_PTRS) != 0, T, group_dim,
                              group_cols, pts);
    });
    if (st != MLG_OK) return st;
    std::vector<const double *> ptrs(T);
    for (int t = 0; t < T; ++t) ptrs[t] = pts[t].p;
    return create_graph(out, n, T, group_dim, ptrs.data(), sigma, kp, flags | MLG_DEVICE_PTRS,
                        stream, (flags & MLG_SKIP_DEGREES) == 0);
}

mlg_status mlg_median_pairwise_distance(int64_t n, int D, const double *features, int d,
                                        const int *cols, int s, const int64_t *sample,
                                        double *sigma, int flags, void *stream) {
    return guard([&] {
        MLG_REQUIRE(sigma, MLG_ERR_ARG, "null argument");
        hipStream_t st = make_stream(stream);
        struct SD {
            hipStream_t s;
            bool own;
            ~SD() { if (own) (void)hipStreamDestroy(s); }
        } sd{st, stream == nullptr};
        *sigma = median_pair_distance(n, D, features, (flags & MLG_DEVICE_PTRS) != 0, d, cols, s,
                                      sample, st);
    });
}

mlg_status mlg_graph_destroy(mlg_graph *g) {
    return guard([&] {
        if (!g) return;
        hipStream_t s = g->g.stream;
        bool own = g->own_stream;
        (void)hipStreamSynchronize(s);
        delete g;
        if (own) (void)hipStreamDestroy(s);
    });
}

mlg_status mlg_graph_degrees(mlg_graph *h, int layer, double *deg, int flags) {
    return guard([&] {
        MLG_REQUIRE(h && deg, MLG_ERR_ARG, "null argument");
        Graph &g = h->g;
        MLG_REQUIRE(layer >= 0 && layer < g.T, MLG_ERR_ARG, "layer out of range");
        MLG_REQUIRE(g.has_degrees, MLG_ERR_ARG, "graph created with MLG_SKIP_DEGREES has no degrees");
        MLG_HIP(hipMemcpyAsync(deg, g.layers[layer].deg.p, sizeof(double) * g.n,
                               (flags & MLG_DEVICE_PTRS) ? hipMemcpyDeviceToDevice
                                                         : hipMemcpyDeviceToHost,
                               g.stream));
        MLG_HIP(hipStreamSynchronize(g.stream));
    });
}

mlg_status mlg_graph_layer_info(mlg_graph *h, int layer, int *ip, double *dp) {
    return guard([&] {
        MLG_REQUIRE(h && ip && dp, MLG_ERR_ARG, "null argument");
        Graph &g = h->g;
        MLG_REQUIRE(layer >= 0 && layer < g.T, MLG_ERR_ARG, "layer out of range");
        const Layer &L = g.layers[layer];
        ip[0] = L.d;
        ip[1] = L.kp.method == MLG_METHOD_NFFT ? L.nf.N : 0;
        ip[2] = L.kp.method == MLG_METHOD_NFFT ? L.win.w : 0;
        ip[3] = L.kp.method == MLG_METHOD_NFFT ? L.nf.B : 0;
        ip[4] = L.kp.precision;
        ip[5] = L.kp.method;
        dp[0] = L.kp.method == MLG_METHOD_NFFT ? L.nf.sigma_s : L.sigma;
        dp[1] = L.kp.method == MLG_METHOD_NFFT ? L.nf.scale : 1.0;
    });
}

mlg_status mlg_laplacian_matvec(mlg_graph *h, int layer, int op, int b, const double *X,
                                int64_t ldx, double *Y, int64_t ldy, int flags) {
    return guard([&] {
        MLG_REQUIRE(h && X && Y, MLG_ERR_ARG, "null argument");
        Graph &g = h->g;
        check_op(g, layer, op, b);
        MLG_REQUIRE(ldx >= g.n && ldy >= g.n, MLG_ERR_ARG, "leading dimension < n");
        if (flags & MLG_DEVICE_PTRS) {
            graph_matvec_enqueue(g, layer, op, b, X, ldx, Y, ldy, nullptr);
            if (!(flags & MLG_ASYNC)) MLG_HIP(hipStreamSynchronize(g.stream));
            return;
        }
        DevBuf<double> dX((size_t)g.n * b), dY((size_t)g.n * b);
        copy_cols(dX.p, g.n, X, ldx, g.n, b, hipMemcpyHostToDevice, g.stream);
        graph_matvec_enqueue(g, layer, op, b, dX.p, g.n, dY.p, g.n, nullptr);
        copy_cols(Y, ldy, dY.p, g.n, g.n, b, hipMemcpyDeviceToHost, g.stream);
        MLG_HIP(hipStreamSynchronize(g.stream));
    });
}

mlg_status mlg_graph_synchronize(mlg_graph *h) {
    return guard([&] {
        MLG_REQUIRE(h, MLG_ERR_ARG, "null argument");
        MLG_HIP(hipStreamSynchronize(h->g.stream));
    });
}

mlg_status mlg_profile_stages(mlg_graph *h, int layer, int op, int b, const double *X, int64_t ldx,
                              double *Y, int64_t ldy, int reps, double *stage_ms, int flags) {
    return guard([&] {
        MLG_REQUIRE(h && X && Y && stage_ms, MLG_ERR_ARG, "null argument");
        MLG_REQUIRE(flags & MLG_DEVICE_PTRS, MLG_ERR_ARG, "profiling needs device pointers");
        MLG_REQUIRE(reps >= 1, MLG_ERR_ARG, "reps must be >= 1");
        Graph &g = h->g;
        MLG_REQUIRE(ldx >= g.n && ldy >= g.n, MLG_ERR_ARG, "leading dimension < n");
        for (int i = 0; i < MLG_NSTAGES; ++i) stage_ms[i] = 0.0;
        for (int r = 0; r < reps; ++r)
            graph_matvec_enqueue(g, layer, op, b, X, ldx, Y, ldy, stage_ms);
        for (int i = 0; i < MLG_NSTAGES; ++i) stage_ms[i] /= reps;
    });
}

mlg_status mlg_kernel_matvec(int64_t n, int d, const double *points, double sigma,
                             const mlg_kparams *kp, int b, const double *X, int64_t ldx, double *Y,
                             int64_t ldy, int flags, void *stream) {
    mlg_graph *h = nullptr;
    const double *pp[1] = {points};
    mlg_status st = create_graph(&h, n, 1, &d, pp, &sigma, kp, flags, stream, false);
    if (st != MLG_OK) return st;
    st = guard([&] {
        MLG_REQUIRE(X && Y, MLG_ERR_ARG, "null argument");
    });
    if (st == MLG_OK) st = mlg_laplacian_matvec(h, 0, MLG_OP_W, b, X, ldx, Y, ldy, flags);
    std::string keep = mlg::g_last_error;
    mlg_graph_destroy(h);
    mlg::set_last_error(keep);
    return st;
}

// Operators of the eigensolver.
namespace {
struct NadjOp : LanczosOp {
    Graph &g;
    int layer;
    NadjOp(Graph &g_, int l) : g(g_), layer(l) {}
    void apply(int b, const double *X, int64_t ldx, double *Y, int64_t ldy) override {
        graph_matvec_enqueue(g, layer, MLG_OP_NADJ, b, X, ldx, Y, ldy, nullptr);
    }
    double lambda(double mu) const override { return 1.0 - mu; }
};

// delta^-p L_{p,delta}^p, spectrum in (0, 1]; lambda = delta mu^(1/p).
struct PowerLanczosOp : LanczosOp {
    PowerMeanOp pw;
    int layer;
    PowerLanczosOp(Graph &g, int l, int b, double p, int max_steps) : pw(g, b, p, max_steps), layer(l) {}
    void apply(int b, const double *X, int64_t ldx, double *Y, int64_t ldy) override {
        MLG_REQUIRE(b == pw.b, MLG_ERR_ARG, "block size mismatch in the Krylov power");
        pw.apply(layer, X, ldx, Y, ldy, true);
    }
    double lambda(double mu) const override {
        return pw.delta * std::pow(std::max(mu, 1e-300), 1.0 / pw.p);
    }
};

void pksm_defaults(const mlg_pksm_params *pk, double outer_tol, double *tol, int *steps) {
    *tol = (pk && pk->tol > 0) ? pk->tol : 0.01 * outer_tol;
    *steps = (pk && pk->max_steps > 0) ? pk->max_steps : kPksmDefaultSteps;
}
}  // namespace

mlg_status mlg_lanczos_eigs(mlg_graph *h, int layer, double p, int k, int block, double tol,
                            int max_restarts, uint64_t seed, const double *V0, double *evals,
                            double *evecs, int64_t ldv, mlg_eig_info *info,
                            const mlg_pksm_params *pk, int flags) {
    mlg_status rc = MLG_OK;
    mlg_status st = guard([&] {
        MLG_REQUIRE(h && evals && evecs, MLG_ERR_ARG, "null argument");
        Graph &g = h->g;
        MLG_REQUIRE(layer >= -1 && layer < g.T, MLG_ERR_ARG, "layer out of range");
        MLG_REQUIRE(g.has_degrees, MLG_ERR_ARG, "graph created with MLG_SKIP_DEGREES has no Laplacian");
        MLG_REQUIRE(p == 1.0 || p < 0.0, MLG_ERR_NOT_IMPL,
                    "power means are implemented for p = 1 and p < 0");
        MLG_REQUIRE(k >= 1 && 2 * (int64_t)k <= g.n, MLG_ERR_ARG, "k must be in 1..n/2");
        MLG_REQUIRE(block >= 1 && block <= 32, MLG_ERR_ARG, "block must be in 1..32");
        MLG_REQUIRE(tol > 0, MLG_ERR_ARG, "tol must be > 0");
        MLG_REQUIRE(max_restarts >= 0, MLG_ERR_ARG, "max_restarts must be >= 0");
        MLG_REQUIRE(ldv >= g.n, MLG_ERR_ARG, "ldv < n");
        if (pk) MLG_REQUIRE(pk->max_steps == 0 || pk->max_steps >= 4, MLG_ERR_ARG,
                            "pksm max_steps must be 0 or >= 4");
        const bool dev = (flags & MLG_DEVICE_PTRS) != 0;
        DevBuf<double> dV0, dE;
        const double *v0 = V0;
        if (V0 && !dev) {
            upload(dV0, V0, (size_t)g.n * block, false, g.stream);
            v0 = dV0.p;
        }
        double *E = evecs;
        int64_t lde = ldv;
        if (!dev) {
            dE.alloc((size_t)g.n * k);
            E = dE.p;
            lde = g.n;
        }
        std::vector<double> ev(k);
        if (p == 1.0) {
            NadjOp op(g, layer);
            rc = lanczos_run(g, op, k, block, tol, max_restarts, seed, v0, ev.data(), E, lde, info);
            if (info) {
                info->inner_steps = 0;
                info->inner_unconverged = 0;
            }
        } else {
            double itol;
            int isteps;
            pksm_defaults(pk, tol, &itol, &isteps);
            PowerLanczosOp op(g, layer, block, p, isteps);
            op.pw.tol = itol;
            rc = lanczos_run(g, op, k, block, tol, max_restarts, seed, v0, ev.data(), E, lde, info);
            if (info) {
                info->inner_steps = op.pw.max_used;
                info->inner_unconverged = op.pw.unconverged;
                info->matvecs = (int)std::min<int64_t>(op.pw.layer_matvecs, INT32_MAX);
            }
            if (rc == MLG_OK && op.pw.unconverged) rc = MLG_WARN_NOT_CONVERGED;
        }
        if (dev) {
            MLG_HIP(hipMemcpyAsync(evals, ev.data(), 8 * k, hipMemcpyHostToDevice, g.stream));
        } else {
            std::copy(ev.begin(), ev.end(), evals);
            copy_cols(evecs, ldv, E, g.n, g.n, k, hipMemcpyDeviceToHost, g.stream);
        }
        MLG_HIP(hipStreamSynchronize(g.stream));
    });
    return st != MLG_OK ? st : rc;
}

mlg_status mlg_power_mean_matvec(mlg_graph *h, int layer, double p, int b, const double *X,
                                 int64_t ldx, double *Y, int64_t ldy, const mlg_pksm_params *pk,
                                 int *steps, int flags) {
    mlg_status rc = MLG_OK;
    mlg_status st = guard([&] {
        MLG_REQUIRE(h && X && Y, MLG_ERR_ARG, "null argument");
        Graph &g = h->g;
        MLG_REQUIRE(layer >= -1 && layer < g.T, MLG_ERR_ARG, "layer out of range");
        MLG_REQUIRE(g.has_degrees, MLG_ERR_ARG, "graph created with MLG_SKIP_DEGREES has no Laplacian");
        MLG_REQUIRE(p < 0.0, MLG_ERR_ARG, "p must be negative");
        MLG_REQUIRE(b >= 1 && b <= 64, MLG_ERR_ARG, "b must be in 1..64");
        MLG_REQUIRE(ldx >= g.n && ldy >= g.n, MLG_ERR_ARG, "leading dimension < n");
        if (pk) MLG_REQUIRE(pk->max_steps == 0 || pk->max_steps >= 4, MLG_ERR_ARG,
                            "pksm max_steps must be 0 or >= 4");
        double itol;
        int isteps;
        pksm_defaults(pk, 1e-10, &itol, &isteps);
        PowerMeanOp op(g, b, p, isteps);
        op.tol = itol;
        if (flags & MLG_DEVICE_PTRS) {
            op.apply(layer, X, ldx, Y, ldy, false);
        } else {
            DevBuf<double> dX((size_t)g.n * b), dY((size_t)g.n * b);
            copy_cols(dX.p, g.n, X, ldx, g.n, b, hipMemcpyHostToDevice, g.stream);
            op.apply(layer, dX.p, g.n, dY.p, g.n, false);
            copy_cols(Y, ldy, dY.p, g.n, g.n, b, hipMemcpyDeviceToHost, g.stream);
        }
        MLG_HIP(hipStreamSynchronize(g.stream));
        if (steps) *steps = op.max_used;
        if (op.unconverged) rc = MLG_WARN_NOT_CONVERGED;
    });
    return st != MLG_OK ? st : rc;
}

mlg_status mlg_allen_cahn_ssl(int64_t n, int k, int m, const double *evals, const double *evecs,
                              int64_t ldv, const int32_t *labels, const mlg_ac_params *prm,
                              double *U, int32_t *pred, int *iters, int flags, void *stream) {
    return guard([&] {
        MLG_REQUIRE(evals && evecs && labels && prm && U && pred, MLG_ERR_ARG, "null argument");
        MLG_REQUIRE(n >= 1 && k >= 1 && m >= 2 && m <= 64 && ldv >= n, MLG_ERR_ARG,
                    "need n >= 1, k >= 1, 2 <= m <= 64, ldv >= n");
        MLG_REQUIRE(prm->eps > 0 && prm->dt > 0 && prm->max_iter >= 1, MLG_ERR_ARG,
                    "need eps > 0, dt > 0, max_iter >= 1");
        hipStream_t s = make_stream(stream);
        struct SD {
            hipStream_t s;
            bool own;
            ~SD() { if (own) (void)hipStreamDestroy(s); }
        } sd{s, stream == nullptr};
        const bool dev = (flags & MLG_DEVICE_PTRS) != 0;
        DevBuf<double> dE, dV, dU;
        DevBuf<int32_t> dL, dP;
        const double *E = evals, *V = evecs;
        const int32_t *Lb = labels;
        double *Uo = U;
        int32_t *Po = pred;
        int64_t ld = ldv;
        if (!dev) {
            upload(dE, evals, k, false, s);
            dV.alloc((size_t)n * k);
            copy_cols(dV.p, n, evecs, ldv, n, k, hipMemcpyHostToDevice, s);
            upload(dL, labels, n, false, s);
            dU.alloc((size_t)n * m);
            dP.alloc(n);
            E = dE.p;
            V = dV.p;
            Lb = dL.p;
            Uo = dU.p;
            Po = dP.p;
            ld = n;
        }
        int it = 0;
        ac_run(n, k, m, E, V, ld, Lb, *prm, Uo, Po, &it, s);
        if (!dev) {
            MLG_HIP(hipMemcpyAsync(U, Uo, sizeof(double) * n * m, hipMemcpyDeviceToHost, s));
            MLG_HIP(hipMemcpyAsync(pred, Po, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s));
        }
        MLG_HIP(hipStreamSynchronize(s));
        if (iters) *iters = it;
    });
}

}  // extern "C"
