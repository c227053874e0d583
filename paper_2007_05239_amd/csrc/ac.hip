// Multiclass Allen--Cahn scores in the truncated eigenbasis (Algorithm 2,
// steps 2-4; the scheme of Sec. 5 with the eigenbasis iteration of
// Appendix B), FP64.  Compiled with -ffp-contract=off: every product is
// rounded before it is added, and each sum runs in the order below, so the
// result does not depend on the launch shape:
//   den_r   = (1 + c*dt) + (eps*dt)*lambda_r;   Z_ri = phi_ir / den_r
//   a_q     = sum_c |u_ic - delta_qc|            (c ascending)
//   s_p     = 0.25*(a_p*a_p)
//   term_q  = (0.5*a_q) * prod_{p != q} s_p      (p ascending)
//   T_ij    = sum_q (q == j ? -term_q : +term_q) (q ascending)
//   R       = ((1+c dt) U - (dt/(2 eps)) T) - (dt omega_i)(U - F)
//   V = Z R   rows in chunks of 256 summed in row order, then a pairwise
//             tree over chunks (neighbours (2j, 2j+1), odd last carried)
//   U~ = Phi V  sum over r ascending;  Chen & Ye projection onto the simplex
//   change  = max_i ||u_i^new - u_i||^2 / max_i ||u_i^new||^2
//   pred    = row argmax, lowest class id on ties (Sec. 6)
#include <algorithm>

#include "internal.h"

namespace mlg {

constexpr int kAcChunk = 256;
constexpr int kAcMaxM = 64;

__global__ void k_ac_Z(int64_t n, int k, const double *__restrict__ evals,
                       const double *__restrict__ evecs, int64_t ldv, double c, double dt,
                       double eps, double *__restrict__ Z) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * k) return;
    const int64_t r = e / n, i = e - r * n;
    double onepcdt = c * dt;
    onepcdt = 1.0 + onepcdt;
    const double epsdt = eps * dt;
    const double ee = epsdt * evals[r];
    const double den = onepcdt + ee;
    Z[e] = evecs[i + r * ldv] / den;
}

__global__ void k_ac_init(int64_t n, int m, const int32_t *__restrict__ labels,
                          double *__restrict__ U, int *__restrict__ bad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int l = labels[i];
    if (l >= m || l < -1) bad[0] = 1;
    const double inv_m = 1.0 / (double)m;
    for (int j = 0; j < m; ++j) U[i * m + j] = (l >= 0) ? (j == l ? 1.0 : 0.0) : inv_m;
}

__device__ inline void ac_potential_grad(int m, const double *u, double *T) {
    double a[kAcMaxM], s[kAcMaxM], term[kAcMaxM];
    for (int q = 0; q < m; ++q) {
        double acc = 0.0;
        for (int c = 0; c < m; ++c) acc = acc + fabs(u[c] - (c == q ? 1.0 : 0.0));
        a[q] = acc;
        s[q] = 0.25 * (a[q] * a[q]);
    }
    for (int q = 0; q < m; ++q) {
        double prod = 1.0;
        for (int p = 0; p < m; ++p)
            if (p != q) prod = prod * s[p];
        term[q] = (0.5 * a[q]) * prod;
    }
    for (int j = 0; j < m; ++j) {
        double t = 0.0;
        for (int q = 0; q < m; ++q) t = (q == j) ? t - term[q] : t + term[q];
        T[j] = t;
    }
}

__global__ void k_ac_rhs(int64_t n, int m, const double *__restrict__ U,
                         const int32_t *__restrict__ labels, double onepcdt, double coefT,
                         double dt, double omega0, double *__restrict__ R) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double u[kAcMaxM], T[kAcMaxM];
    for (int j = 0; j < m; ++j) u[j] = U[i * m + j];
    ac_potential_grad(m, u, T);
    const int l = labels[i];
    const double om = l >= 0 ? omega0 : 0.0;
    const double w = dt * om;
    for (int j = 0; j < m; ++j) {
        const double f = (l >= 0 && j == l) ? 1.0 : 0.0;
        const double r1 = onepcdt * u[j];
        const double r2 = coefT * T[j];
        const double r3 = r1 - r2;
        const double r4 = u[j] - f;
        const double r5 = w * r4;
        R[i * m + j] = r3 - r5;
    }
}

// part[ch][r][c] = sum over rows of chunk ch (ascending) of Z[r][i]*R[i][c].
__global__ __launch_bounds__(256) void k_ac_zr(int64_t n, int k, int m, const double *__restrict__ Z,
                                               const double *__restrict__ R,
                                               double *__restrict__ part) {
    __shared__ double Rs[kAcChunk * 16];
    const int64_t ch = blockIdx.x;
    const int64_t i0 = ch * kAcChunk;
    const int cnt = (int)((n - i0) < kAcChunk ? (n - i0) : kAcChunk);
    double *out = part + ch * (int64_t)k * m;
    // columns in groups of 16 so the chunk of R fits in LDS
    for (int c0 = 0; c0 < m; c0 += 16) {
        const int cg = (m - c0) < 16 ? (m - c0) : 16;
        __syncthreads();
        for (int e = threadIdx.x; e < cnt * cg; e += blockDim.x) {
            int ii = e / cg, cc = e - ii * cg;
            Rs[ii * 16 + cc] = R[(i0 + ii) * m + c0 + cc];
        }
        __syncthreads();
        for (int e = threadIdx.x; e < k * cg; e += blockDim.x) {
            const int r = e / cg, cc = e - r * cg;
            const double *zr = Z + (int64_t)r * n + i0;
            double acc = 0.0;
            for (int ii = 0; ii < cnt; ++ii) {
                const double pr = zr[ii] * Rs[ii * 16 + cc];
                acc = acc + pr;
            }
            out[r * m + c0 + cc] = acc;
        }
    }
}

// One level of the pairwise tree: dst[j] = src[2j] + src[2j+1]; an odd last
// element is copied.
__global__ void k_ac_tree(int64_t cnt, int len, const double *__restrict__ src,
                          double *__restrict__ dst) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t half = cnt / 2, outc = half + (cnt & 1);
    if (e >= outc * len) return;
    const int64_t j = e / len;
    const int x = (int)(e - j * len);
    if (j < half)
        dst[e] = src[(2 * j) * len + x] + src[(2 * j + 1) * len + x];
    else
        dst[e] = src[(cnt - 1) * len + x];
}

__device__ inline void ac_project(int m, const double *y, double *x) {
    double srt[kAcMaxM];
    for (int i = 0; i < m; ++i) {
        double v = y[i];
        int j = i - 1;
        while (j >= 0 && srt[j] > v) {
            srt[j + 1] = srt[j];
            --j;
        }
        srt[j + 1] = v;
    }
    double s = 0.0, that = 0.0;
    bool found = false;
    for (int i = m - 1; i >= 1; --i) {
        s = s + srt[i];
        const double t = (s - 1.0) / (double)(m - i);
        if (t >= srt[i - 1]) {
            that = t;
            found = true;
            break;
        }
    }
    if (!found) {
        s = s + srt[0];
        that = (s - 1.0) / (double)m;
    }
    for (int i = 0; i < m; ++i) {
        const double dlt = y[i] - that;
        x[i] = dlt > 0.0 ? dlt : 0.0;
    }
}

// U~ = Phi V, projection, per-row squared norms of the change and the new row.
__global__ void k_ac_update(int64_t n, int k, int m, const double *__restrict__ evecs, int64_t ldv,
                            const double *__restrict__ V, double *__restrict__ U,
                            double *__restrict__ rowd, double *__restrict__ rown) {
    __shared__ double Vs[128 * 16];
    const bool vs_ok = k * m <= 128 * 16;
    if (vs_ok)
        for (int e = threadIdx.x; e < k * m; e += blockDim.x) Vs[e] = V[e];
    __syncthreads();
    const double *Vp = vs_ok ? Vs : V;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double ut[kAcMaxM], un[kAcMaxM];
    for (int j = 0; j < m; ++j) {
        double acc = 0.0;
        for (int r = 0; r < k; ++r) {
            const double pr = evecs[i + (int64_t)r * ldv] * Vp[r * m + j];
            acc = acc + pr;
        }
        ut[j] = acc;
    }
    ac_project(m, ut, un);
    double dn = 0.0, nn = 0.0;
    for (int j = 0; j < m; ++j) {
        const double dl = un[j] - U[i * m + j];
        const double p1 = dl * dl;
        dn = dn + p1;
        const double p2 = un[j] * un[j];
        nn = nn + p2;
        U[i * m + j] = un[j];
    }
    rowd[i] = dn;
    rown[i] = nn;
}

// Block maxima (max is exact, so the grouping does not matter).
__global__ void k_max2(int64_t n, const double *__restrict__ a, const double *__restrict__ b,
                       double *__restrict__ out) {
    __shared__ double sa[256], sb[256];
    double ma = 0.0, mb = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        ma = fmax(ma, a[i]);
        mb = fmax(mb, b[i]);
    }
    sa[threadIdx.x] = ma;
    sb[threadIdx.x] = mb;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            sa[threadIdx.x] = fmax(sa[threadIdx.x], sa[threadIdx.x + off]);
            sb[threadIdx.x] = fmax(sb[threadIdx.x], sb[threadIdx.x + off]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[2 * blockIdx.x] = sa[0];
        out[2 * blockIdx.x + 1] = sb[0];
    }
}

__global__ void k_ac_finish_max(int nb, const double *__restrict__ part, double *__restrict__ rc) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double num = 0.0, den = 0.0;
    for (int b = 0; b < nb; ++b) {
        num = fmax(num, part[2 * b]);
        den = fmax(den, part[2 * b + 1]);
    }
    rc[0] = num / den;
}

__global__ void k_ac_argmax(int64_t n, int m, const double *__restrict__ U,
                            int32_t *__restrict__ pred) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int best = 0;
    for (int j = 1; j < m; ++j)
        if (U[i * m + j] > U[i * m + best]) best = j;
    pred[i] = best;
}

void ac_run(int64_t n, int k, int m, const double *evals, const double *evecs, int64_t ldv,
            const int32_t *labels, const mlg_ac_params &prm, double *U, int32_t *pred, int *iters,
            hipStream_t s) {
    MLG_REQUIRE(m <= kAcMaxM, MLG_ERR_ARG, "m must be <= 64");
    DevBuf<double> Z((size_t)n * k), R((size_t)n * m), rowd(n), rown(n);
    const int64_t nch = (n + kAcChunk - 1) / kAcChunk;
    DevBuf<double> pa((size_t)nch * k * m), pb((size_t)((nch + 1) / 2) * k * m + 1), mx(2048),
        rcd(1);
    DevBuf<int> bad(1);
    MLG_HIP(hipMemsetAsync(bad.p, 0, 4, s));
    hipLaunchKernelGGL(k_ac_Z, dim3(ceil_div(n * k, 256)), dim3(256), 0, s, n, k, evals, evecs, ldv,
                       prm.c, prm.dt, prm.eps, Z.p);
    MLG_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_ac_init, dim3(ceil_div(n, 256)), dim3(256), 0, s, n, m, labels, U, bad.p);
    MLG_LAUNCH_CHECK();
    int hb = 0;
    MLG_HIP(hipMemcpyAsync(&hb, bad.p, 4, hipMemcpyDeviceToHost, s));
    MLG_HIP(hipStreamSynchronize(s));
    MLG_REQUIRE(hb == 0, MLG_ERR_ARG, "labels must be -1 or in 0..m-1");
    double onepcdt = prm.c * prm.dt;
    onepcdt = 1.0 + onepcdt;
    const double coefT = prm.dt / (2.0 * prm.eps);
    const int nmx = std::min<int64_t>(1024, ceil_div(n, 256));
    int l = 0;
    double rc = 0.0;
    do {
        hipLaunchKernelGGL(k_ac_rhs, dim3(ceil_div(n, 256)), dim3(256), 0, s, n, m, U, labels, onepcdt,
                           coefT, prm.dt, prm.omega0, R.p);
        MLG_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_ac_zr, dim3((unsigned)nch), dim3(256), 0, s, n, k, m, Z.p, R.p, pa.p);
        MLG_LAUNCH_CHECK();
        double *src = pa.p, *dst = pb.p;
        int64_t cnt = nch;
        while (cnt > 1) {
            const int64_t outc = cnt / 2 + (cnt & 1);
            hipLaunchKernelGGL(k_ac_tree, dim3(ceil_div(outc * k * m, 256)), dim3(256), 0, s, cnt, k * m,
                               src, dst);
            MLG_LAUNCH_CHECK();
            std::swap(src, dst);
            cnt = outc;
        }
        hipLaunchKernelGGL(k_ac_update, dim3(ceil_div(n, 256)), dim3(256), 0, s, n, k, m, evecs, ldv, src,
                           U, rowd.p, rown.p);
        MLG_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_max2, dim3(nmx), dim3(256), 0, s, n, rowd.p, rown.p, mx.p);
        MLG_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_ac_finish_max, dim3(1), dim3(64), 0, s, nmx, mx.p, rcd.p);
        MLG_LAUNCH_CHECK();
        MLG_HIP(hipMemcpyAsync(&rc, rcd.p, 8, hipMemcpyDeviceToHost, s));
        MLG_HIP(hipStreamSynchronize(s));
        l = l + 1;
    } while (rc > prm.tol && l < prm.max_iter);
    hipLaunchKernelGGL(k_ac_argmax, dim3(ceil_div(n, 256)), dim3(256), 0, s, n, m, U, pred);
    MLG_LAUNCH_CHECK();
    MLG_HIP(hipStreamSynchronize(s));
    *iters = l;
}

}  // namespace mlg
