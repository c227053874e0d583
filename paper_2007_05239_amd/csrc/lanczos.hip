// FP64 block thick-restart Lanczos for the k largest eigenpairs of a
// symmetric operator A given as a LanczosOp (Sec. 3; Algorithm 2 step 1):
//   p = 1:  A = D^-1/2 W D^-1/2 (one layer) or I - L_1 =
//           (1/T) sum_t D_t^-1/2 W_t D_t^-1/2, lambda = 1 - mu;
//   p < 0:  A = delta^-p L_{p,delta}^p through the polynomial Krylov power,
//           lambda = delta mu^(1/p).
// The paper used MATLAB's Krylov-Schur; for a symmetric operator, thick
// restart with Ritz vectors is the same method.
//
// State kept between steps:  A V_m = V_m H_m + Q S,  V_m^T Q = 0,
//   V_m  n x m orthonormal basis, H_m = V_m^T A V_m (m x m),
//   Q    n x b next block, S (b x m) its coupling.
// Expansion:  W = A Q; two passes of classical Gram-Schmidt against [V_m, Q]
//   (CGS2, full reorthogonalisation) give the new column block of H; a
//   Cholesky QR (twice) of W gives the next Q and its coupling R.
// Restart:  H = Y Theta Y^T (one-workgroup Jacobi); residual of Ritz pair i is
//   ||S y_i||; the k+b largest Ritz pairs are kept: V <- V Y_keep,
//   H <- Theta_keep, S <- S Y_keep.
// Every reduction runs in a fixed order (chunk partials, then a sequential
// sum), so results are reproducible bit for bit.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "internal.h"

namespace mlg {

constexpr int kTnMaxP = 256;   // rows of C = A^T B
constexpr int kTnMaxQ = 32;    // columns of C
constexpr int kRB = 16;        // rows per LDS batch

// ---- C = A^T B, partials per row chunk --------------------------------------
// Rows pass through LDS 16 at a time (element e = tid + 256 u of a batch:
// row e mod 16, column e / 16, so each column's 16 rows are one 128-byte
// load); the next batch's loads are issued before the current batch is
// multiplied, so each workgroup keeps a batch of rows in flight.  The
// products run on the FP64 matrix cores (v_mfma_f64_16x16x4f64, K = 4 rows
// per instruction): wavefront w owns the 16 x 16 tiles a = w, w + 4, ... of C
// (rows i of A^T) for every column tile c, over all rows of the chunk.
// Operand layout: A[i][k] in lane i + 16 k, B[k][v] in lane v + 16 k; the
// result D[i][v] in lane v + 16 qq, element m, with i = qq + 4 m.
typedef double f64x4_t __attribute__((ext_vector_type(4)));

template <int NA, int NQ>
__global__ __launch_bounds__(256) void k_gemm_tn_part(int64_t n, int p, int q,
                                                      const double *__restrict__ A, int64_t lda,
                                                      const double *__restrict__ B, int64_t ldb,
                                                      int64_t rc, double *__restrict__ part) {
    constexpr int AS = NA * 16 + 1, BS = NQ * 16 + 1;   // padded LDS rows
    constexpr int NT = (NA + 3) / 4;                    // tiles per wavefront
    __shared__ double As[kRB * AS];
    __shared__ double Bs[kRB * BS];
    const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
    const int li = lane & 15, lk = lane >> 4;
    const int64_t r0 = (int64_t)blockIdx.x * rc;
    const int64_t r1 = (r0 + rc < n) ? r0 + rc : n;
    f64x4_t acc[NT][NQ];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int c = 0; c < NQ; ++c) acc[t][c] = f64x4_t{0.0, 0.0, 0.0, 0.0};
    static_assert(kRB == 16, "batch layout");
    double ra[NA], rb_[NQ];
    auto fetch = [&](int64_t rb) {
        const int cnt = (int)((r1 - rb) < kRB ? (r1 - rb) : kRB);
#pragma unroll
        for (int u = 0; u < NA; ++u) {
            const int e = tid + 256 * u, rr = e % kRB, i = e / kRB;
            ra[u] = (rr < cnt && i < p) ? A[rb + rr + (int64_t)i * lda] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < NQ; ++u) {
            const int e = tid + 256 * u, rr = e % kRB, j = e / kRB;
            rb_[u] = (rr < cnt && j < q) ? B[rb + rr + (int64_t)j * ldb] : 0.0;
        }
    };
    if (r0 < r1) fetch(r0);
    for (int64_t rb = r0; rb < r1; rb += kRB) {
        __syncthreads();
#pragma unroll
        for (int u = 0; u < NA; ++u) {
            const int e = tid + 256 * u;
            As[(e % kRB) * AS + e / kRB] = ra[u];
        }
#pragma unroll
        for (int u = 0; u < NQ; ++u) {
            const int e = tid + 256 * u;
            Bs[(e % kRB) * BS + e / kRB] = rb_[u];
        }
        __syncthreads();
        if (rb + kRB < r1) fetch(rb + kRB);
        // four K steps of four rows; rows past the chunk's end are zero
#pragma unroll
        for (int s4 = 0; s4 < kRB / 4; ++s4) {
            const int row = 4 * s4 + lk;
            double bop[NQ];
#pragma unroll
            for (int c = 0; c < NQ; ++c) bop[c] = Bs[row * BS + 16 * c + li];
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const int a = wv + 4 * t;
                if (a < NA) {
                    const double aop = As[row * AS + 16 * a + li];
#pragma unroll
                    for (int c = 0; c < NQ; ++c)
                        acc[t][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(aop, bop[c], acc[t][c], 0, 0, 0);
                }
            }
        }
    }
    double *o = part + (int64_t)blockIdx.x * p * q;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int a = wv + 4 * t;
        if (a >= NA) continue;
#pragma unroll
        for (int c = 0; c < NQ; ++c)
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const int i = 16 * a + lk + 4 * m, j = 16 * c + li;
                if (i < p && j < q) o[i * q + j] = acc[t][c][m];
            }
    }
}

__device__ inline double wave_sum64(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// C[e] = sum_c part[c][e]: one wavefront per e; lane l adds c = l, l + 64, ...
// in order, then a fixed butterfly over the lanes.
__global__ __launch_bounds__(256) void k_sum_parts(int nparts, int total,
                                                   const double *__restrict__ part,
                                                   double *__restrict__ C) {
    const int e = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (e >= total) return;
    double s = 0.0;
    for (int c = lane; c < nparts; c += 64) s += part[(int64_t)c * total + e];
    s = wave_sum64(s);
    if (lane == 0) C[e] = s;
}

// Out[:, j] (=, -=) sum_i A[:, i] C[i][j] for the column group of QG
// columns in blockIdx.y (C row-major p x q; its p x QG slice in dynamic LDS).
// mode 0: =, 1: -=.  A thread reads its whole row of A before it writes its
// row of Out, so with a single column group (q <= QG) Out may be A itself.
template <int QG>
__global__ __launch_bounds__(256) void k_gemm_nn(int64_t n, int p, int q, const double *A,
                                                 int64_t lda, const double *__restrict__ C,
                                                 double *Out, int64_t ldo, int mode) {
    extern __shared__ double Cs[];
    const int j0 = blockIdx.y * QG;
    const int qq = (q - j0) < QG ? (q - j0) : QG;
    for (int e = threadIdx.x; e < p * QG; e += 256) {
        int i = e / QG, j = e % QG;
        Cs[e] = j < qq ? C[i * q + j0 + j] : 0.0;
    }
    __syncthreads();
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r >= n) return;
    double acc[QG];
#pragma unroll
    for (int j = 0; j < QG; ++j) acc[j] = 0.0;
    // the next PF entries of the row are loaded while the current PF are
    // used, so each thread keeps PF loads in flight; the sums still run over
    // i in ascending order
    constexpr int PF = 8;
    double cur[PF], nxt[PF];
#pragma unroll
    for (int u = 0; u < PF; ++u) cur[u] = u < p ? A[r + (int64_t)u * lda] : 0.0;
    for (int i0 = 0; i0 < p; i0 += PF) {
#pragma unroll
        for (int u = 0; u < PF; ++u) nxt[u] = i0 + PF + u < p ? A[r + (int64_t)(i0 + PF + u) * lda] : 0.0;
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            if (i0 + u < p) {
#pragma unroll
                for (int j = 0; j < QG; ++j) acc[j] += cur[u] * Cs[(i0 + u) * QG + j];
            }
        }
#pragma unroll
        for (int u = 0; u < PF; ++u) cur[u] = nxt[u];
    }
#pragma unroll
    for (int j = 0; j < QG; ++j) {
        if (j < qq) {
            double *o = Out + r + (int64_t)(j0 + j) * ldo;
            *o = mode ? *o - acc[j] : acc[j];
        }
    }
}

// W[r, :] <- W[r, :] M (q x q row-major, q <= QB), in place per row: the row
// is held in registers, each output column is formed and stored in turn.
template <int QB>
__global__ __launch_bounds__(256) void k_rowmul(int64_t n, int q, double *__restrict__ W,
                                                int64_t ldw, const double *__restrict__ M) {
    __shared__ double Ms[QB * QB];
    for (int e = threadIdx.x; e < q * q; e += blockDim.x) Ms[(e / q) * QB + e % q] = M[e];
    __syncthreads();
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    double w[QB];
#pragma unroll
    for (int i = 0; i < QB; ++i) w[i] = i < q ? W[r + (int64_t)i * ldw] : 0.0;
    for (int j = 0; j < q; ++j) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < QB; ++i)
            if (i < q) s += w[i] * Ms[i * QB + j];
        W[r + (int64_t)j * ldw] = s;
    }
}

// Cholesky G = R^T R (G q x q row-major, symmetric); writes Rinv (q x q
// row-major, upper) into out[0..q*q) and R into out[q*q..2q*q); flag = 1 if a
// pivot is not positive relative to the largest diagonal.  One wavefront:
// right-looking elimination in LDS (each entry receives its updates in the
// order k = 0, 1, ...), then one lane per column of the inverse (back
// substitution).
__global__ __launch_bounds__(64) void k_chol_inv(int q, const double *__restrict__ G,
                                                 double *__restrict__ out, int *flag) {
    __shared__ double A[kTnMaxQ][kTnMaxQ + 1];
    __shared__ double Ri[kTnMaxQ][kTnMaxQ + 1];
    __shared__ int bad_s;
    __shared__ double dmax_s;
    const int lane = threadIdx.x;
    for (int e = lane; e < q * q; e += 64) {
        A[e / q][e % q] = G[e];
        Ri[e / q][e % q] = 0.0;
    }
    __syncthreads();
    if (lane == 0) {
        double dmax = 0.0;
        for (int i = 0; i < q; ++i) dmax = fmax(dmax, A[i][i]);
        dmax_s = dmax;
        bad_s = !(dmax > 0.0);
    }
    __syncthreads();
    const double dmax = dmax_s;
    for (int j = 0; j < q && !bad_s; ++j) {
        if (lane == 0) {
            const double sv = A[j][j];
            if (!(sv > 1e-28 * dmax)) bad_s = 1;
            else A[j][j] = sqrt(sv);
        }
        __syncthreads();
        if (bad_s) break;
        const double rjj = A[j][j];
        for (int i = j + 1 + lane; i < q; i += 64) A[j][i] = A[j][i] / rjj;
        __syncthreads();
        const int w = q - j - 1;
        for (int e = lane; e < w * w; e += 64) {
            const int i = j + 1 + e / w, l = j + 1 + e % w;
            if (l >= i) A[i][l] -= A[j][i] * A[j][l];
        }
        __syncthreads();
    }
    const int bad = bad_s;
    if (!bad) {
        for (int j = lane; j < q; j += 64) {
            Ri[j][j] = 1.0 / A[j][j];
            for (int i = j - 1; i >= 0; --i) {
                double sv = 0.0;
                for (int k = i + 1; k <= j; ++k) sv += A[i][k] * Ri[k][j];
                Ri[i][j] = -sv / A[i][i];
            }
        }
    }
    __syncthreads();
    for (int e = lane; e < q * q; e += 64) {
        const int i = e / q, j = e % q;
        const bool up = !bad && i <= j;
        out[e] = up ? Ri[i][j] : 0.0;
        out[q * q + e] = up ? A[i][j] : 0.0;
    }
    if (lane == 0) flag[0] = bad;
}

// C (m+b) x b row-major from CGS -> H columns [m, m+b) and rows; the diagonal
// block is symmetrised.
__global__ void k_store_H(int mtot, int m, int b, const double *__restrict__ C,
                          double *__restrict__ H, int ldh) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= mtot * b) return;
    const int i = e / b, j = e % b;
    double v = C[i * b + j];
    if (i >= m) v = 0.5 * (v + C[(m + j) * b + (i - m)]);
    H[(int64_t)i * ldh + m + j] = v;
    H[(int64_t)(m + j) * ldh + i] = v;
}

// R (b x b, upper, row-major) -> coupling rows H[m+b.., m..] = R, and the
// transpose.
__global__ void k_store_R(int m, int b, const double *__restrict__ R, double *__restrict__ H,
                          int ldh) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= b * b) return;
    const int i = e / b, j = e % b;
    const double v = R[i * b + j];
    H[(int64_t)(m + b + i) * ldh + m + j] = v;
    H[(int64_t)(m + j) * ldh + m + b + i] = v;
}

// Parallel cyclic Jacobi (round-robin pairing) for a symmetric m x m matrix
// in one workgroup.  A (ldh) is overwritten: diag = eigenvalues; Y (m x m,
// row-major, column c = eigenvector c).  AL / YL: A / Y are worked on in LDS
// (dynamic shared memory, A first, rows padded to m + 1 doubles so that the
// column rotations' rows fall in different banks) and written back at the
// end.  A Y kept in global memory is worked on transposed (the column
// rotations then touch consecutive addresses) and transposed in place at
// the end.
template <bool AL, bool YL>
__global__ __launch_bounds__(256) void k_jacobi(int m, double *__restrict__ Ag, int ldag,
                                                double *__restrict__ Yg, int max_sweeps) {
    __shared__ double cs[kTnMaxP / 2 + 1], sn[kTnMaxP / 2 + 1];
    __shared__ int pp[kTnMaxP / 2 + 1], qq[kTnMaxP / 2 + 1];
    __shared__ int rotated;
    extern __shared__ double jsm[];
    double *A = AL ? jsm : Ag;
    const int lda = AL ? m + 1 : ldag;
    double *Y = YL ? (AL ? jsm + m * (m + 1) : jsm) : Yg;
    // element (r, c) of Y at Y[r * yr + c * yc]
    const int yr = YL ? m + 1 : 1, yc = YL ? 1 : m;
    const int tid = threadIdx.x;
    const int me = m + (m & 1);  // even, with a dummy index m if odd
    if (AL)
        for (int e = tid; e < m * m; e += 256) A[(e / m) * lda + e % m] = Ag[(e / m) * ldag + e % m];
    for (int e = tid; e < m * m; e += 256)
        Y[(e / m) * yr + (e % m) * yc] = (e / m == e % m) ? 1.0 : 0.0;
    __syncthreads();
    for (int sweep = 0; sweep < max_sweeps; ++sweep) {
        if (tid == 0) rotated = 0;
        __syncthreads();
        for (int round = 0; round < me - 1; ++round) {
            // pairs of the round-robin schedule: index me-1 fixed, others rotate
            for (int k = tid; k < me / 2; k += 256) {
                int a, b;
                if (k == 0) {
                    a = me - 1;
                    b = round;
                } else {
                    a = (round + k) % (me - 1);
                    b = (round - k + (me - 1)) % (me - 1);
                }
                int p = a < b ? a : b, q = a < b ? b : a;
                double c = 1.0, s = 0.0;
                if (q < m) {
                    const double apq = A[p * lda + q];
                    const double app = A[p * lda + p], aqq = A[q * lda + q];
                    if (fabs(apq) > 1e-300 && fabs(apq) > 1e-17 * sqrt(fabs(app * aqq))) {
                        const double th = (aqq - app) / (2.0 * apq);
                        const double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                        c = 1.0 / sqrt(t * t + 1.0);
                        s = t * c;
                        rotated = 1;
                    }
                }
                pp[k] = p;
                qq[k] = q;
                cs[k] = c;
                sn[k] = s;
            }
            __syncthreads();
            // columns: A <- A J.  The elements of one round are disjoint, so
            // each thread loads kJacB of them before it stores any (a Y in
            // global memory otherwise costs one memory latency per element).
            constexpr int kJacB = 4;
            const int ncol = (me / 2) * m;
            for (int e0 = tid; e0 < ncol; e0 += 256 * kJacB) {
                int ia[kJacB], ib[kJacB], ja[kJacB], jb[kJacB];
                bool act[kJacB];
                double c[kJacB], sv[kJacB], ap[kJacB], aq[kJacB], yp[kJacB], yq[kJacB];
#pragma unroll
                for (int u = 0; u < kJacB; ++u) {
                    const int e = e0 + u * 256;
                    act[u] = false;
                    if (e < ncol) {
                        const int k = e / m, r = e % m;
                        const int p = pp[k], q = qq[k];
                        act[u] = q < m && sn[k] != 0.0;
                        c[u] = cs[k];
                        sv[u] = sn[k];
                        ia[u] = r * lda + p;
                        ib[u] = r * lda + q;
                        ja[u] = r * yr + p * yc;
                        jb[u] = r * yr + q * yc;
                    }
                    if (act[u]) {
                        ap[u] = A[ia[u]];
                        aq[u] = A[ib[u]];
                        yp[u] = Y[ja[u]];
                        yq[u] = Y[jb[u]];
                    }
                }
#pragma unroll
                for (int u = 0; u < kJacB; ++u) {
                    if (act[u]) {
                        A[ia[u]] = c[u] * ap[u] - sv[u] * aq[u];
                        A[ib[u]] = sv[u] * ap[u] + c[u] * aq[u];
                        Y[ja[u]] = c[u] * yp[u] - sv[u] * yq[u];
                        Y[jb[u]] = sv[u] * yp[u] + c[u] * yq[u];
                    }
                }
            }
            __syncthreads();
            // rows: A <- J^T A
            for (int e = tid; e < (me / 2) * m; e += 256) {
                int k = e / m, cidx = e % m;
                int p = pp[k], q = qq[k];
                if (q >= m || sn[k] == 0.0) continue;
                double c = cs[k], s = sn[k];
                double ap = A[p * lda + cidx], aq = A[q * lda + cidx];
                A[p * lda + cidx] = c * ap - s * aq;
                A[q * lda + cidx] = s * ap + c * aq;
            }
            __syncthreads();
        }
        if (!rotated) break;
        __syncthreads();
    }
    __syncthreads();
    if (AL)
        for (int e = tid; e < m * m; e += 256) Ag[(e / m) * ldag + e % m] = A[(e / m) * lda + e % m];
    if (YL) {
        for (int e = tid; e < m * m; e += 256) Yg[e] = Y[(e / m) * yr + e % m];
    } else {
        // back to row-major: each pair (i < j) swapped by one thread
        for (int e = tid; e < m * m; e += 256) {
            const int i = e / m, j = e % m;
            if (i < j) {
                const double t = Yg[i * m + j];
                Yg[i * m + j] = Yg[j * m + i];
                Yg[j * m + i] = t;
            }
        }
    }
}

// Residual norms ||S y_c|| for the selected Ritz columns sel[0..ns).
__global__ void k_ritz_resid(int m, int b, const double *__restrict__ S, int lds,
                             const double *__restrict__ Y, const int *__restrict__ sel, int ns,
                             double *__restrict__ res) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ns) return;
    const int col = sel[c];
    double acc = 0.0;
    for (int r = 0; r < b; ++r) {
        double s = 0.0;
        for (int i = 0; i < m; ++i) s += S[r * lds + i] * Y[i * m + col];
        acc += s * s;
    }
    res[c] = sqrt(acc);
}

// Ysel (m x ns row-major) = Y[:, sel].
__global__ void k_select_cols(int m, const double *__restrict__ Y, const int *__restrict__ sel,
                              int ns, double *__restrict__ Ys) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m * ns) return;
    const int i = e / ns, c = e % ns;
    Ys[e] = Y[i * m + sel[c]];
}

// S_new (b x ns) = S (b x m) Ysel; H <- diag(theta_sel).
__global__ void k_restart_small(int m, int b, const double *__restrict__ S, int lds,
                                const double *__restrict__ Ys, int ns,
                                const double *__restrict__ theta, double *__restrict__ Snew,
                                double *__restrict__ H, int ldh) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < b * ns) {
        const int r = e / ns, c = e % ns;
        double s = 0.0;
        for (int i = 0; i < m; ++i) s += S[r * lds + i] * Ys[i * ns + c];
        Snew[r * lds + c] = s;
    }
    if (e < ldh * ldh) {
        const int i = e / ldh, j = e % ldh;
        H[e] = (i == j && i < ns) ? theta[i] : 0.0;
    }
}

// Coupling after an expansion: S = [0 ... 0 R] with R at columns [m, m+b).
__global__ void k_set_S(int mnew, int b, const double *__restrict__ R, double *__restrict__ S,
                        int lds) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= b * mnew) return;
    const int r = e / mnew, c = e % mnew;
    const int m = mnew - b;
    S[r * lds + c] = (c >= m) ? R[r * b + (c - m)] : 0.0;
}

__device__ inline uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// N(0,1) draws by Box-Muller from two SplitMix64 outputs per element.
__global__ void k_randn(uint64_t seed, int64_t n, int b, double *__restrict__ X, int64_t ldx,
                        int64_t offset) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * b) return;
    const int64_t c = offset + e;
    const uint64_t z1 = splitmix64(seed + 2ull * (uint64_t)c * 0x9E3779B97F4A7C15ull);
    const uint64_t z2 = splitmix64(seed + (2ull * (uint64_t)c + 1ull) * 0x9E3779B97F4A7C15ull);
    const double u1 = ((double)(z1 >> 11) + 1.0) * 0x1.0p-53;
    const double u2 = (double)(z2 >> 11) * 0x1.0p-53;
    const int64_t i = e % n, j = e / n;
    X[i + j * ldx] = sqrt(-2.0 * log(u1)) * cospi(2.0 * u2);
}

// Sign convention: the largest-magnitude entry of each column is positive
// (lowest index on ties).
// Sign of each eigenvector: the entry of largest magnitude (lowest index on
// ties) is made positive.  Two passes over kSignChunks row chunks per column:
// chunk maxima (magnitude, index, value), then every chunk's workgroup
// reduces its column's maxima in chunk order (all reach the same entry) and
// negates its chunk if that entry is negative.  The value travels with the
// maximum, so no workgroup reads an entry another one may be negating.
constexpr int kSignChunks = 64;

__global__ __launch_bounds__(256) void k_sign_part(int64_t n, const double *__restrict__ V,
                                                   int64_t ldv, double *__restrict__ pa,
                                                   int64_t *__restrict__ pi,
                                                   double *__restrict__ pv) {
    __shared__ double sa[256], sv[256];
    __shared__ int64_t si[256];
    const double *col = V + (int64_t)blockIdx.x * ldv;
    const int64_t len = (n + kSignChunks - 1) / kSignChunks;
    const int64_t lo = (int64_t)blockIdx.y * len;
    const int64_t hi = lo + len < n ? lo + len : n;
    double best = -1.0, val = 0.0;
    int64_t bi = 0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += 256) {
        const double v = col[i];
        const double a = fabs(v);
        if (a > best) { best = a; bi = i; val = v; }
    }
    sa[threadIdx.x] = best;
    si[threadIdx.x] = bi;
    sv[threadIdx.x] = val;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            const double a = sa[threadIdx.x + off];
            const int64_t ai = si[threadIdx.x + off];
            if (a > sa[threadIdx.x] || (a == sa[threadIdx.x] && ai < si[threadIdx.x])) {
                sa[threadIdx.x] = a;
                si[threadIdx.x] = ai;
                sv[threadIdx.x] = sv[threadIdx.x + off];
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int64_t o = (int64_t)blockIdx.x * kSignChunks + blockIdx.y;
        pa[o] = sa[0];
        pi[o] = si[0];
        pv[o] = sv[0];
    }
}

__global__ __launch_bounds__(256) void k_sign_apply(int64_t n, double *__restrict__ V, int64_t ldv,
                                                    const double *__restrict__ pa,
                                                    const int64_t *__restrict__ pi,
                                                    const double *__restrict__ pv) {
    __shared__ int flip;
    if (threadIdx.x == 0) {
        const int64_t o = (int64_t)blockIdx.x * kSignChunks;
        double best = -1.0, val = 0.0;
        int64_t bi = 0;
        for (int j = 0; j < kSignChunks; ++j) {
            const double a = pa[o + j];
            const int64_t ai = pi[o + j];
            if (a > best || (a == best && ai < bi)) { best = a; bi = ai; val = pv[o + j]; }
        }
        flip = val < 0.0;
    }
    __syncthreads();
    if (!flip) return;
    double *col = V + (int64_t)blockIdx.x * ldv;
    const int64_t len = (n + kSignChunks - 1) / kSignChunks;
    const int64_t lo = (int64_t)blockIdx.y * len;
    const int64_t hi = lo + len < n ? lo + len : n;
    for (int64_t i = lo + threadIdx.x; i < hi; i += 256) col[i] = -col[i];
}

__global__ void k_add(int cnt, double *a, const double *b) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < cnt) a[e] += b[e];
}

// ------------------------------------------------------------------------------
struct Lz {
    hipStream_t s;
    int64_t n;
    DevBuf<double> part, C, C2, G, RR;
    DevBuf<int> flag;
    int nchunks = 0;
    int64_t rc = 0;
    void setup(int64_t n_, hipStream_t s_) {
        n = n_;
        s = s_;
        // about 2048 row chunks at large n (eight workgroups per CU, all
        // resident), at least 1024 rows each
        rc = std::max<int64_t>(1024, (n + 2047) / 2048);
        rc = (rc + kRB - 1) / kRB * kRB;
        nchunks = ceil_div(n, rc);
        part.alloc((size_t)nchunks * kTnMaxP * kTnMaxQ);
        C.alloc(kTnMaxP * kTnMaxQ);
        C2.alloc(kTnMaxP * kTnMaxQ);
        G.alloc(kTnMaxQ * kTnMaxQ);
        RR.alloc(2 * kTnMaxQ * kTnMaxQ);
        flag.alloc(1);
    }
    // Cout (p x q row-major) = A^T B
    void tn(int p, int q, const double *A, int64_t lda, const double *B, int64_t ldb, double *Cout) {
        MLG_REQUIRE(p >= 1 && p <= kTnMaxP && q >= 1 && q <= kTnMaxQ, MLG_ERR_ARG, "tn shape");
        const int na = ceil_div(p, 16), nq = ceil_div(q, 16);
        const dim3 g(nchunks), t(256);
#define MLG_TN(NA)                                                                              \
    case NA:                                                                                    \
        if (nq == 1)                                                                            \
            hipLaunchKernelGGL((k_gemm_tn_part<NA, 1>), g, t, 0, s, n, p, q, A, lda, B, ldb, rc, \
                               part.p);                                                         \
        else                                                                                    \
            hipLaunchKernelGGL((k_gemm_tn_part<NA, 2>), g, t, 0, s, n, p, q, A, lda, B, ldb, rc, \
                               part.p);                                                         \
        break;
        switch (na) {
            MLG_TN(1) MLG_TN(2) MLG_TN(3) MLG_TN(4) MLG_TN(5) MLG_TN(6) MLG_TN(7) MLG_TN(8)
            MLG_TN(9) MLG_TN(10) MLG_TN(11) MLG_TN(12) MLG_TN(13) MLG_TN(14) MLG_TN(15) MLG_TN(16)
        }
#undef MLG_TN
        MLG_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_sum_parts, dim3(ceil_div(p * q, 4)), dim3(256), 0, s, nchunks, p * q,
                           part.p, Cout);
        MLG_LAUNCH_CHECK();
    }
    // Whether nn(p, q, ...) runs as one column group, so that Out may be A
    // (the product written over the first q columns of A in place).
    static bool nn_single(int p, int q) { return q <= 32 || (q <= 64 && (size_t)p * 64 * 8 <= 65536); }
    void nn(int p, int q, const double *A, int64_t lda, const double *Cm, double *Out, int64_t ldo,
            int mode) {
        MLG_REQUIRE(p >= 1 && p <= kTnMaxP && q >= 1, MLG_ERR_ARG, "nn shape");
        MLG_REQUIRE(Out != A || nn_single(p, q), MLG_ERR_ARG, "nn in place needs one column group");
        const dim3 t(256);
        if (q <= 16)
            hipLaunchKernelGGL(k_gemm_nn<16>, dim3(ceil_div(n, 256), 1), t, (size_t)p * 16 * 8, s, n, p,
                               q, A, lda, Cm, Out, ldo, mode);
        else if (q <= 32 || !nn_single(p, q))
            hipLaunchKernelGGL(k_gemm_nn<32>, dim3(ceil_div(n, 256), ceil_div(q, 32)), t,
                               (size_t)p * 32 * 8, s, n, p, q, A, lda, Cm, Out, ldo, mode);
        else
            hipLaunchKernelGGL(k_gemm_nn<64>, dim3(ceil_div(n, 256), 1), t, (size_t)p * 64 * 8, s, n, p,
                               q, A, lda, Cm, Out, ldo, mode);
        MLG_LAUNCH_CHECK();
    }
    void rowmul(int q, double *W, int64_t ldw, const double *M) {
        const dim3 g(ceil_div(n, 256)), t(256);
        if (q <= 4) hipLaunchKernelGGL(k_rowmul<4>, g, t, 0, s, n, q, W, ldw, M);
        else if (q <= 8) hipLaunchKernelGGL(k_rowmul<8>, g, t, 0, s, n, q, W, ldw, M);
        else if (q <= 16) hipLaunchKernelGGL(k_rowmul<16>, g, t, 0, s, n, q, W, ldw, M);
        else hipLaunchKernelGGL(k_rowmul<32>, g, t, 0, s, n, q, W, ldw, M);
        MLG_LAUNCH_CHECK();
    }
    // W (n x q) -> orthonormal, R (q x q upper) with W_in = W_out R.  Returns
    // false if W is numerically rank deficient.
    bool cholqr2(int q, double *W, int64_t ldw, std::vector<double> &Rhost) {
        std::vector<double> R1(q * q), R2(q * q);
        for (int pass = 0; pass < 2; ++pass) {
            tn(q, q, W, ldw, W, ldw, G.p);
            hipLaunchKernelGGL(k_chol_inv, dim3(1), dim3(64), 0, s, q, G.p, RR.p, flag.p);
            MLG_LAUNCH_CHECK();
            int bad = 0;
            MLG_HIP(hipMemcpyAsync(&bad, flag.p, 4, hipMemcpyDeviceToHost, s));
            MLG_HIP(hipMemcpyAsync(pass == 0 ? R1.data() : R2.data(), RR.p + q * q, 8 * q * q,
                                   hipMemcpyDeviceToHost, s));
            MLG_HIP(hipStreamSynchronize(s));
            if (bad) return false;
            rowmul(q, W, ldw, RR.p);
        }
        // R = R2 R1 (upper triangular)
        Rhost.assign(q * q, 0.0);
        for (int i = 0; i < q; ++i)
            for (int j = i; j < q; ++j) {
                double acc = 0.0;
                for (int k = i; k <= j; ++k) acc += R2[i * q + k] * R1[k * q + j];
                Rhost[i * q + j] = acc;
            }
        return true;
    }
    // CGS2 of W (n x b) against V (n x p): W -= V (V^T W), twice; Csum = total.
    void cgs2(int p, int b, const double *V, int64_t ldv, double *W, int64_t ldw) {
        tn(p, b, V, ldv, W, ldw, C.p);
        nn(p, b, V, ldv, C.p, W, ldw, 1);
        tn(p, b, V, ldv, W, ldw, C2.p);
        nn(p, b, V, ldv, C2.p, W, ldw, 1);
        hipLaunchKernelGGL(k_add, dim3(ceil_div(p * b, 256)), dim3(256), 0, s, p * b, C.p, C2.p);
        MLG_LAUNCH_CHECK();
    }
};

// Dynamic LDS the Jacobi kernel may take: the device's limit per workgroup
// (160 KB on gfx950) less 4 KB for the kernel's static rotation tables;
// 60 KB if the device does not report one.  With it the projected matrix
// of a 128-column basis (128 KB) is rotated in LDS.
static int64_t jacobi_lds_budget() {
    static int64_t budget = -1;
    if (budget < 0) {
        int dev = 0, lim = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
            lim < 64 * 1024)
            lim = 64 * 1024;
        budget = (int64_t)lim - 4 * 1024;
    }
    return budget;
}

mlg_status lanczos_run(Graph &g, LanczosOp &op, int k, int b, double tol, int max_restarts,
                       uint64_t seed, const double *V0, double *evals, double *evecs, int64_t ldv,
                       mlg_eig_info *info) {
    const int64_t n = g.n;
    hipStream_t s = g.stream;
    // Basis of up to mmax columns before a thick restart: wide enough that a
    // restart adds about five blocks to the k + b kept Ritz vectors (fewer
    // restarts and fewer products; the basis is small next to HBM), capped
    // by the projected-matrix limit and by n.  30 pairs of a 10^7-node graph
    // with blocks of 16: 128 columns take 63 block products and 11 restarts,
    // 80 columns (max(2k, k + 3b)) took 115 and 55.
    int mmax = std::max(4 * k, k + 6 * b);
    mmax = (mmax + b - 1) / b * b;
    while (mmax + b > kTnMaxP) mmax -= b;
    while (mmax > k + b && (int64_t)mmax + b > n) mmax -= b;
    // The first expansion also checks convergence every ~16 columns from
    // max(2k, k + 3b) columns on, so that a problem which converges early
    // does not run to the full basis (a few extra Rayleigh-Ritz steps once).
    int mfirst = std::max(2 * k, k + 3 * b);
    mfirst = (mfirst + b - 1) / b * b;
    if (mfirst > mmax) mfirst = mmax;
    MLG_REQUIRE(mmax >= k + b, MLG_ERR_ARG, "k + 2 block exceeds the basis limit of 256 columns");
    MLG_REQUIRE((int64_t)mmax + b <= n, MLG_ERR_ARG, "basis larger than n");
    Lz z;
    z.setup(n, s);
    DevBuf<double> V((size_t)n * (mmax + b)), W((size_t)n * b), Hd((size_t)kTnMaxP * kTnMaxP),
        Ad((size_t)kTnMaxP * kTnMaxP), Yd((size_t)kTnMaxP * kTnMaxP), Sd((size_t)kTnMaxQ * kTnMaxP),
        S2((size_t)kTnMaxQ * kTnMaxP), Ysel((size_t)kTnMaxP * kTnMaxP), theta(kTnMaxP),
        res(kTnMaxP), Rd(kTnMaxQ * kTnMaxQ);
    DevBuf<int> seld(kTnMaxP);
    const int ldh = kTnMaxP;
    MLG_HIP(hipMemsetAsync(Hd.p, 0, sizeof(double) * ldh * ldh, s));
    MLG_HIP(hipMemsetAsync(Sd.p, 0, sizeof(double) * kTnMaxQ * kTnMaxP, s));
    // start block
    if (V0)
        MLG_HIP(hipMemcpyAsync(V.p, V0, sizeof(double) * n * b, hipMemcpyDeviceToDevice, s));
    else {
        hipLaunchKernelGGL(k_randn, dim3(ceil_div(n * b, 256)), dim3(256), 0, s, seed, n, b, V.p, n,
                           (int64_t)0);
        MLG_LAUNCH_CHECK();
    }
    std::vector<double> Rh;
    int64_t rnd_off = n * b;
    auto orthonormalize_new = [&](double *blk, int m_before) {
        // blk (n x b) against V[:, :m_before], then CholQR2; random refill on
        // breakdown (coupling of the refilled block is zero).
        for (int attempt = 0; attempt < 4; ++attempt) {
            if (m_before > 0) z.cgs2(m_before, b, V.p, n, blk, n);
            if (z.cholqr2(b, blk, n, Rh)) return attempt == 0;
            hipLaunchKernelGGL(k_randn, dim3(ceil_div(n * b, 256)), dim3(256), 0, s, seed, n, b, blk,
                               n, rnd_off);
            MLG_LAUNCH_CHECK();
            rnd_off += n * b;
        }
        throw Error(MLG_ERR_HIP, "Lanczos: could not extend the basis (rank deficiency)");
    };
    orthonormalize_new(V.p, 0);
    int m = 0;  // basis columns with complete H; Q = V[:, m : m+b]
    int iters = 0, restarts = 0, matvecs = 0;
    std::vector<double> th(kTnMaxP), rs(kTnMaxP);
    std::vector<int> order(kTnMaxP);
    mlg_status st = MLG_WARN_NOT_CONVERGED;
    int nconv = 0;
    double maxres = 0.0;
    int mstop = mfirst;   // columns at which the next Rayleigh-Ritz step runs
    for (;;) {
        // ---- expand to mstop columns ----
        while (m + b <= mstop) {
            double *Q = V.p + (int64_t)m * n;
            op.apply(b, Q, n, W.p, n);
            matvecs += b;
            ++iters;
            const int mt = m + b;
            z.cgs2(mt, b, V.p, n, W.p, n);
            hipLaunchKernelGGL(k_store_H, dim3(ceil_div(mt * b, 256)), dim3(256), 0, s, mt, m, b, z.C.p,
                               Hd.p, ldh);
            MLG_LAUNCH_CHECK();
            // next block
            double *Qn = V.p + (int64_t)mt * n;
            MLG_HIP(hipMemcpyAsync(Qn, W.p, sizeof(double) * n * b, hipMemcpyDeviceToDevice, s));
            bool clean = false;
            if (z.cholqr2(b, Qn, n, Rh)) {
                clean = true;
            } else {
                orthonormalize_new(Qn, mt);
                std::fill(Rh.begin(), Rh.end(), 0.0);
                Rh.resize(b * b, 0.0);
            }
            (void)clean;
            MLG_HIP(hipMemcpyAsync(Rd.p, Rh.data(), 8 * b * b, hipMemcpyHostToDevice, s));
            if (mt + b <= mmax) {
                hipLaunchKernelGGL(k_store_R, dim3(ceil_div(b * b, 256)), dim3(256), 0, s, m, b, Rd.p,
                                   Hd.p, ldh);
                MLG_LAUNCH_CHECK();
            }
            hipLaunchKernelGGL(k_set_S, dim3(ceil_div(b * mt, 256)), dim3(256), 0, s, mt, b, Rd.p, Sd.p,
                               kTnMaxP);
            MLG_LAUNCH_CHECK();
            m = mt;
            MLG_HIP(hipStreamSynchronize(s));
        }
        // ---- Rayleigh-Ritz on H (m x m) ----
        MLG_HIP(hipMemcpyAsync(Ad.p, Hd.p, sizeof(double) * m * ldh, hipMemcpyDeviceToDevice, s));
        const int64_t jlds = jacobi_lds_budget();
        const int64_t jmat = (int64_t)m * (m + 1) * 8;   // one padded m x m matrix
        if (2 * jmat <= jlds)
            hipLaunchKernelGGL((k_jacobi<true, true>), dim3(1), dim3(256), 2 * jmat, s, m, Ad.p, ldh,
                               Yd.p, 40);
        else if (jmat <= jlds)
            hipLaunchKernelGGL((k_jacobi<true, false>), dim3(1), dim3(256), jmat, s, m, Ad.p, ldh,
                               Yd.p, 40);
        else
            hipLaunchKernelGGL((k_jacobi<false, false>), dim3(1), dim3(256), 0, s, m, Ad.p, ldh, Yd.p,
                               40);
        MLG_LAUNCH_CHECK();
        std::vector<double> Ah((size_t)m * ldh);
        MLG_HIP(hipMemcpyAsync(Ah.data(), Ad.p, sizeof(double) * m * ldh, hipMemcpyDeviceToHost, s));
        MLG_HIP(hipStreamSynchronize(s));
        for (int i = 0; i < m; ++i) th[i] = Ah[(size_t)i * ldh + i];
        std::iota(order.begin(), order.begin() + m, 0);
        std::stable_sort(order.begin(), order.begin() + m,
                         [&](int a, int c) { return th[a] > th[c]; });
        const int keep = std::min(m - b, k + b);
        MLG_HIP(hipMemcpyAsync(seld.p, order.data(), 4 * keep, hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_ritz_resid, dim3(ceil_div(keep, 64)), dim3(64), 0, s, m, b, Sd.p, kTnMaxP,
                           Yd.p, seld.p, keep, res.p);
        MLG_LAUNCH_CHECK();
        MLG_HIP(hipMemcpyAsync(rs.data(), res.p, 8 * keep, hipMemcpyDeviceToHost, s));
        MLG_HIP(hipStreamSynchronize(s));
        nconv = 0;
        maxres = 0.0;
        for (int i = 0; i < k; ++i) {
            if (rs[i] <= tol) ++nconv;
            maxres = std::max(maxres, rs[i]);
        }
        const bool full = m + b > mmax;
        const bool done = nconv == k || (full && restarts >= max_restarts);
        if (!done && !full) {
            // an early check of the first expansion: the next one after
            // about 16 more columns (one block of 16, four of 4)
            mstop = std::min(mmax, m + b * std::max(1, 16 / b));
            continue;
        }
        if (done) {
            // Ritz vectors of the k wanted pairs, in descending mu
            hipLaunchKernelGGL(k_select_cols, dim3(ceil_div(m * k, 256)), dim3(256), 0, s, m, Yd.p, seld.p,
                               k, Ysel.p);
            MLG_LAUNCH_CHECK();
            z.nn(m, k, V.p, n, Ysel.p, evecs, ldv, 0);
            {
                DevBuf<double> pa((size_t)k * kSignChunks), pv((size_t)k * kSignChunks);
                DevBuf<int64_t> pi((size_t)k * kSignChunks);
                hipLaunchKernelGGL(k_sign_part, dim3(k, kSignChunks), dim3(256), 0, s, n, evecs, ldv,
                                   pa.p, pi.p, pv.p);
                MLG_LAUNCH_CHECK();
                hipLaunchKernelGGL(k_sign_apply, dim3(k, kSignChunks), dim3(256), 0, s, n, evecs, ldv,
                                   pa.p, pi.p, pv.p);
                MLG_LAUNCH_CHECK();
                MLG_HIP(hipStreamSynchronize(s));
            }
            for (int i = 0; i < k; ++i) evals[i] = op.lambda(th[order[i]]);
            st = nconv == k ? MLG_OK : MLG_WARN_NOT_CONVERGED;
            MLG_HIP(hipStreamSynchronize(s));
            break;
        }
        // ---- thick restart: keep the `keep` largest Ritz pairs ----
        ++restarts;
        std::vector<double> thk(keep);
        for (int i = 0; i < keep; ++i) thk[i] = th[order[i]];
        MLG_HIP(hipMemcpyAsync(theta.p, thk.data(), 8 * keep, hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_select_cols, dim3(ceil_div(m * keep, 256)), dim3(256), 0, s, m, Yd.p,
                           seld.p, keep, Ysel.p);
        MLG_LAUNCH_CHECK();
        // V[:, :keep] = V[:, :m] Ysel: in place when one column group covers
        // keep (each row is read whole before it is written), else via a temp
        if (Lz::nn_single(m, keep)) {
            z.nn(m, keep, V.p, n, Ysel.p, V.p, n, 0);
        } else {
            DevBuf<double> tmp((size_t)n * keep);
            z.nn(m, keep, V.p, n, Ysel.p, tmp.p, n, 0);
            MLG_HIP(hipMemcpyAsync(V.p, tmp.p, sizeof(double) * n * keep, hipMemcpyDeviceToDevice, s));
        }
        // move Q = V[:, m : m+b] to V[:, keep : keep+b]
        MLG_HIP(hipMemcpyAsync(V.p + (int64_t)keep * n, V.p + (int64_t)m * n, sizeof(double) * n * b,
                               hipMemcpyDeviceToDevice, s));
        const int tot = std::max(b * keep, ldh * ldh);
        hipLaunchKernelGGL(k_restart_small, dim3(ceil_div(tot, 256)), dim3(256), 0, s, m, b, Sd.p,
                           kTnMaxP, Ysel.p, keep, theta.p, S2.p, Hd.p, ldh);
        MLG_LAUNCH_CHECK();
        // H's arrow: rows/cols [keep, keep+b) couple through S^T; written on
        // the next expansion by CGS (C[0:keep] = S^T up to rounding).
        MLG_HIP(hipMemcpyAsync(Sd.p, S2.p, sizeof(double) * kTnMaxQ * kTnMaxP, hipMemcpyDeviceToDevice,
                               s));
        m = keep;
        mstop = mmax;
        MLG_HIP(hipStreamSynchronize(s));
    }
    if (info) {
        info->iters = iters;
        info->restarts = restarts;
        info->matvecs = matvecs;
        info->nconv = nconv;
        info->max_resid = maxres;
    }
    return st;
}

}  // namespace mlg
