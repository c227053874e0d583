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
};

struct Layer {
    int d = 0;
    double sigma = 0;
    mlg_kparams kp{};
    int64_t n = 0;
    // direct path: centred coordinates, SoA d x n
    DevBuf<double> x64;
    DevBuf<float> x32;
    double center[64];
    NfftPlan nf;
    NfftWindow win;          // matvec window
    DevBuf<double> deg;      // degrees, original order
    DevBuf<double> dinv_s;   // D^-1/2 in sorted (NFFT) or original (direct) order
    int sorted = 0;          // 1 if perm applies
};

// ---- layer_ops.hip ----------------------------------------------------------
void launch_to_rowmajor(int64_t n, int b, const double *X, int64_t ldx, double *Xr, hipStream_t s);
void launch_finish(int64_t n, int b, const double *Yr, const double *X, int64_t ldx, double *Y,
                   int64_t ldy, int lsym, hipStream_t s);
template <class T>
void launch_pre(int64_t n, int b, int bs, const int *perm, const double *dinv, const double *Xr,
                T *Zs, hipStream_t s);
template <class T>
void launch_post(int64_t n, int b, int bs, const int *perm, const double *dinv, double coef,
                 double K0, const T *Fs, const T *Zs, double *Yr, int accumulate, hipStream_t s);
void launch_fill_ones(int64_t n, double *Xr, hipStream_t s);
void launch_check_degrees(int64_t n, const double *deg, double thresh, int *flag, hipStream_t s);
void launch_dinv(int64_t n, const double *deg, const int *perm, double *dinv_s, hipStream_t s);

// ---- direct.hip ---------------------------------------------------------------
template <class T>
void launch_direct(int64_t n, int d, const T *x, double inv_s2, int bs, const T *Zs, T *Fs,
                   T *part, size_t part_cap, hipStream_t s);
template <class T>
size_t direct_part_size(int64_t n, int bs);

// ---- nfft.hip -----------------------------------------------------------------
void nfft_plan_layer(Layer &L, const double *pts_dev, hipStream_t s);
void nfft_make_window(const Layer &L, NfftWindow &W, int w, int prec, int bs, hipStream_t s);
size_t nfft_patch_elems(const NfftPlan &P, const NfftWindow &W, int bs);
size_t nfft_grid_elems(const NfftPlan &P, int bs);
// W~ applied to Zs (sorted, T, stride bs) -> Fs; uses patch and grid workspaces.
template <class T>
void nfft_apply(const NfftPlan &P, const NfftWindow &W, int bs, const T *Zs, T *Fs, T *patch,
                T *grid, hipStream_t s, hipEvent_t *ev /* 5 events or null */);

// ---- lanczos.hip ----------------------------------------------------------------
struct Graph;
mlg_status lanczos_run(Graph &g, int layer, int k, int block, double tol, int max_restarts,
                       uint64_t seed, const double *V0_dev, double *evals_host,
                       double *evecs_dev, int64_t ldv, mlg_eig_info *info);

// ---- ac.hip -------------------------------------------------------------------
void ac_run(int64_t n, int k, int m, const double *evals_dev, const double *evecs_dev,
            int64_t ldv, const int32_t *labels_dev, const mlg_ac_params &prm, double *U_dev,
            int32_t *pred_dev, int *iters, hipStream_t s);

// ---- graph.hip ----------------------------------------------------------------
struct Graph {
    int64_t n = 0;
    int T = 0;
    hipStream_t stream = nullptr;
    std::vector<Layer> layers;
    // workspaces
    DevBuf<double> Xr, Yr;         // n x b point-major FP64
    DevBuf<char> Zs, Fs;           // n x bs, T
    DevBuf<char> patch, grid, part;
    // captured graphs keyed by (layer, op, b)
    struct Cap {
        int layer, op, b;
        hipGraphExec_t exec;
    };
    std::vector<Cap> caps;
    DevBuf<void *> argbuf;         // device copy of (X, Y) pointers for replays
    DevBuf<int64_t> argld;
    ~Graph();
};

// Enqueue Y = op X (device pointers) on g.stream.  With `ev` non-null,
// records stage events (see mlg_profile_stages).
void graph_matvec_enqueue(Graph &g, int layer, int op, int b, const double *X, int64_t ldx,
                          double *Y, int64_t ldy, double *stage_ms);

}  // namespace mlg
