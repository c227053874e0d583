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
constexpr int kAcFastM = 16;    // class counts with register-resident rows

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

// Arrays of compile-time length M hold the m <= M classes, so that the
// per-row state stays in registers when M = m; the loops run over the first
// m entries in the documented order.
template <int M>
__device__ inline void ac_potential_grad(int m, const double *u, double *T) {
    double a[M], s[M], term[M];
#pragma unroll
    for (int q = 0; q < M; ++q) {
        if (q < m) {
            double acc = 0.0;
#pragma unroll
            for (int c = 0; c < M; ++c)
                if (c < m) acc = acc + fabs(u[c] - (c == q ? 1.0 : 0.0));
            a[q] = acc;
            s[q] = 0.25 * (a[q] * a[q]);
        }
    }
#pragma unroll
    for (int q = 0; q < M; ++q) {
        if (q < m) {
            double prod = 1.0;
#pragma unroll
            for (int p = 0; p < M; ++p)
                if (p < m && p != q) prod = prod * s[p];
            term[q] = (0.5 * a[q]) * prod;
        }
    }
#pragma unroll
    for (int j = 0; j < M; ++j) {
        if (j < m) {
            double t = 0.0;
#pragma unroll
            for (int q = 0; q < M; ++q)
                if (q < m) t = (q == j) ? t - term[q] : t + term[q];
            T[j] = t;
        }
    }
}

// Row i of R = ((1+c dt) U - (dt/(2 eps)) T) - (dt omega_i)(U - F).
template <int M>
__device__ inline void ac_rhs_row(int64_t i, int m, const double *u, int l, double onepcdt,
                                  double coefT, double dt, double omega0,
                                  double *__restrict__ R) {
    double T[M];
    ac_potential_grad<M>(m, u, T);
    const double om = l >= 0 ? omega0 : 0.0;
    const double w = dt * om;
#pragma unroll
    for (int j = 0; j < M; ++j) {
        if (j < m) {
            const double f = (l >= 0 && j == l) ? 1.0 : 0.0;
            const double r1 = onepcdt * u[j];
            const double r2 = coefT * T[j];
            const double r3 = r1 - r2;
            const double r4 = u[j] - f;
            const double r5 = w * r4;
            R[i * m + j] = r3 - r5;
        }
    }
}

template <int M>
__global__ __launch_bounds__(256) void k_ac_rhs(int64_t n, int m_rt, const double *__restrict__ U,
                                                const int32_t *__restrict__ labels, double onepcdt,
                                                double coefT, double dt, double omega0,
                                                double *__restrict__ R) {
    // the dispatch passes M = m for m <= kAcFastM: fold the class count
    const int m = (M <= kAcFastM) ? M : m_rt;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double u[M];
#pragma unroll
    for (int j = 0; j < M; ++j) u[j] = j < m ? U[i * m + j] : 0.0;
    ac_rhs_row<M>(i, m, u, labels[i], onepcdt, coefT, dt, omega0, R);
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

// The pairwise tree over chunk partials: each level forms node j from nodes
// 2j and 2j+1 of the level below (src[2j] + src[2j+1]); an odd last node is
// copied up.  One pass does four levels: dst[j] is node j four levels above
// src (cnt nodes), formed from its up to 16 leaves with exactly those pairs
// and copies.
__global__ void k_ac_tree4(int64_t cnt, int len, const double *__restrict__ src,
                           double *__restrict__ dst) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t c[5];
    c[0] = cnt;
#pragma unroll
    for (int l = 0; l < 4; ++l) c[l + 1] = c[l] / 2 + (c[l] & 1);
    if (e >= c[4] * len) return;
    const int64_t j = e / len;
    const int x = (int)(e - j * len);
    double v[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int64_t g = j * 16 + q;
        v[q] = g < cnt ? src[g * len + x] : 0.0;
    }
#pragma unroll
    for (int l = 0; l < 4; ++l) {
        const int w = 8 >> l;  // nodes of level l + 1 under node j
#pragma unroll
        for (int i = 0; i < w; ++i) {
            // node j * w + i of level l + 1 has children 2 (j w + i) and that + 1;
            // one past the level's end is a copy, further ones are never read
            const int64_t g = j * w + i;
            v[i] = 2 * g + 1 < c[l] ? v[2 * i] + v[2 * i + 1] : v[2 * i];
        }
    }
    dst[e] = v[0];
}

// Reduce cnt rows of len doubles at src to one by the pairwise tree, using dst
// as the other buffer; returns the buffer that holds the result.  Four levels
// per launch at every count (below 16 rows the pass ends in one row).
static double *ac_tree_reduce(int64_t cnt, int len, double *src, double *dst, hipStream_t s) {
    while (cnt > 1) {
        int64_t outc = cnt;
        for (int l = 0; l < 4; ++l) outc = outc / 2 + (outc & 1);
        hipLaunchKernelGGL(k_ac_tree4, dim3(ceil_div(outc * len, 256)), dim3(256), 0, s, cnt, len,
                           src, dst);
        MLG_LAUNCH_CHECK();
        std::swap(src, dst);
        cnt = outc;
    }
    return src;
}

// Chen & Ye projection of y onto the simplex.  The sort is an odd-even
// transposition network (the sorted values are the same for any correct
// sort); entries m..M-1 are +inf and sort last.
template <int M>
__device__ inline void ac_project(int m, const double *y, double *x) {
    double srt[M];
#pragma unroll
    for (int i = 0; i < M; ++i) srt[i] = i < m ? y[i] : INFINITY;
#pragma unroll
    for (int pass = 0; pass < M; ++pass) {
#pragma unroll
        for (int i = pass & 1; i + 1 < M; i += 2) {
            const double a = srt[i], b = srt[i + 1];
            const bool sw = a > b;
            srt[i] = sw ? b : a;
            srt[i + 1] = sw ? a : b;
        }
    }
    double s = 0.0, that = 0.0;
    bool found = false;
#pragma unroll
    for (int i = M - 1; i >= 1; --i) {
        if (i <= m - 1 && !found) {
            s = s + srt[i];
            const double t = (s - 1.0) / (double)(m - i);
            if (t >= srt[i - 1]) {
                that = t;
                found = true;
            }
        }
    }
    if (!found) {
        s = s + srt[0];
        that = (s - 1.0) / (double)m;
    }
#pragma unroll
    for (int i = 0; i < M; ++i) {
        if (i < m) {
            const double dlt = y[i] - that;
            x[i] = dlt > 0.0 ? dlt : 0.0;
        }
    }
}

// U~ = Phi V, projection, per-row squared norms of the change and the new row,
// and the next right-hand side row.  Each eigenvector entry is read once and
// used for all m classes; V sits in LDS when it fits (VLDS), else it is read
// from global memory.
template <int M, bool VLDS>
__global__ __launch_bounds__(256) void k_ac_update(int64_t n, int k, int m_rt,
                                                   const double *__restrict__ evecs, int64_t ldv,
                                                   const double *__restrict__ V,
                                                   double *__restrict__ U,
                                                   double *__restrict__ rowd,
                                                   double *__restrict__ rown,
                                                   const int32_t *__restrict__ labels,
                                                   double onepcdt, double coefT, double dt,
                                                   double omega0, double *__restrict__ R) {
    // the dispatch passes M = m for m <= kAcFastM: fold the class count
    const int m = (M <= kAcFastM) ? M : m_rt;
    extern __shared__ double Vs[];
    if constexpr (VLDS) {
        for (int e = threadIdx.x; e < k * m; e += blockDim.x) Vs[e] = V[e];
        __syncthreads();
    }
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double ut[M], un[M];
#pragma unroll
    for (int j = 0; j < M; ++j) ut[j] = 0.0;
#pragma unroll 8
    for (int r = 0; r < k; ++r) {
        const double ph = evecs[i + (int64_t)r * ldv];
#pragma unroll
        for (int j = 0; j < M; ++j) {
            if (j < m) {
                const double pr = ph * (VLDS ? Vs[r * m + j] : V[r * m + j]);
                ut[j] = ut[j] + pr;
            }
        }
    }
    ac_project<M>(m, ut, un);
    double dn = 0.0, nn = 0.0;
#pragma unroll
    for (int j = 0; j < M; ++j) {
        if (j < m) {
            const double dl = un[j] - U[i * m + j];
            const double p1 = dl * dl;
            dn = dn + p1;
            const double p2 = un[j] * un[j];
            nn = nn + p2;
            U[i * m + j] = un[j];
        }
    }
    rowd[i] = dn;
    rown[i] = nn;
    // the next iteration's right-hand side from the new row
    ac_rhs_row<M>(i, m, un, labels[i], onepcdt, coefT, dt, omega0, R);
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

// ---- fused iteration (m <= 16): one pass over the eigenvectors per step ----
// den_r = (1 + c dt) + (eps dt) lambda_r, the divisor of row r of Z.
__global__ void k_ac_den(int k, const double *__restrict__ evals, double c, double dt, double eps,
                         double *__restrict__ den) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= k) return;
    double onepcdt = c * dt;
    onepcdt = 1.0 + onepcdt;
    const double epsdt = eps * dt;
    const double ee = epsdt * evals[r];
    den[r] = onepcdt + ee;
}

// Chunk-major copies of the eigenvectors and of Z:
//   Pc[(ch k + r) 256 + ii] = phi_{ch 256 + ii, r},  Zc[...] = that / den_r
// (0 past n), so that a chunk's k x 256 block is contiguous.
__global__ void k_ac_pack(int64_t n, int k, int64_t nch, const double *__restrict__ evecs,
                          int64_t ldv, const double *__restrict__ den, double *__restrict__ Pc,
                          double *__restrict__ Zc) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nch * k * kAcChunk) return;
    const int ii = (int)(e & (kAcChunk - 1));
    const int64_t rest = e >> 8;
    const int r = (int)(rest % k);
    const int64_t i = (rest / k) * kAcChunk + ii;
    const double ph = i < n ? evecs[i + (int64_t)r * ldv] : 0.0;
    Pc[e] = ph;
    Zc[e] = ph / den[r];
}

// sum over rows q < cnt in order of z_q R[q][c] (R rows at stride m in LDS,
// Rc = &R[0][c]); z from the chunk-major Z row in groups of 16 rows, two
// register buffers in turn: a group's loads are issued one group before it
// is used.  FULL: cnt = 256.
template <bool FULL>
__device__ inline void ac_chain_group(const double2 (&g)[8], const double *Rc, int m, int base,
                                      int cnt, double &acc) {
#pragma unroll
    for (int h = 0; h < 16; ++h) {
        if (FULL || base + h < cnt) {
            const double z = (h & 1) ? g[h >> 1].y : g[h >> 1].x;
            const double p = z * Rc[(base + h) * m];
            acc = acc + p;
        }
    }
}

template <bool FULL>
__device__ inline double ac_chain(const double2 *__restrict__ z2, const double *Rc, int m,
                                  int cnt) {
    double acc = 0.0;
    double2 ga[8], gb[8];
#pragma unroll
    for (int h = 0; h < 8; ++h) ga[h] = z2[h];
    for (int q0 = 0; q0 < cnt; q0 += 32) {
        if (q0 + 16 < cnt) {
#pragma unroll
            for (int h = 0; h < 8; ++h) gb[h] = z2[(q0 + 16) / 2 + h];
        }
        ac_chain_group<FULL>(ga, Rc, m, q0, cnt, acc);
        if (q0 + 32 < cnt) {
#pragma unroll
            for (int h = 0; h < 8; ++h) ga[h] = z2[(q0 + 32) / 2 + h];
        }
        if (q0 + 16 < cnt) ac_chain_group<FULL>(gb, Rc, m, q0 + 16, cnt, acc);
    }
    return acc;
}

// One step for chunk ch = blockIdx.x (256 rows, thread ii owns row ch 256 + ii):
//   update (unless FIRST): u~ = sum_r phi_ir V_r (r ascending), projection,
//     change norms (block maxima), U row written;
//   the right-hand side row of the new U, kept in LDS;
//   the chunk's partials of the next V: part[ch][r][c] = sum over the rows in
//     order of Z_ri R_ic, one thread per (r, c) chain, Z from the chunk-major
//     copy (consecutive threads share r and read the same Z entries).
template <int M, bool FIRST>
__global__ __launch_bounds__(256) void k_ac_iter(int64_t n, int k, int m_rt,
                                                 const double *__restrict__ Pc,
                                                 const double *__restrict__ Zc,
                                                 const double *__restrict__ V,
                                                 double *__restrict__ U,
                                                 const int32_t *__restrict__ labels,
                                                 double onepcdt, double coefT, double dt,
                                                 double omega0, double *__restrict__ part,
                                                 double *__restrict__ mxd,
                                                 double *__restrict__ mxn) {
    // the dispatch passes M = m for m <= kAcFastM: fold the class count
    const int m = (M <= kAcFastM) ? M : m_rt;
    extern __shared__ double lds[];
    double *Rs = lds;                        // 256 x m
    __shared__ double red[2][4];
    const int64_t ch = blockIdx.x;
    const int64_t i0 = ch * kAcChunk;
    const int cnt = (int)((n - i0) < kAcChunk ? (n - i0) : kAcChunk);
    const int ii = threadIdx.x;
    const int64_t i = i0 + ii;
    const bool live = ii < cnt;
    const double *P = Pc + ch * (int64_t)k * kAcChunk;
    double dn = 0.0, nn = 0.0;
    if (live) {
        double u[M];
        if (FIRST) {
#pragma unroll
            for (int j = 0; j < M; ++j) u[j] = j < m ? U[i * m + j] : 0.0;
        } else {
            double ut[M];
#pragma unroll
            for (int j = 0; j < M; ++j) ut[j] = 0.0;
#pragma unroll 8
            // V is the same for every thread: its entries come through the
            // scalar cache (uniform addresses), not LDS
            for (int r = 0; r < k; ++r) {
                const double ph = P[(int64_t)r * kAcChunk + ii];
#pragma unroll
                for (int j = 0; j < M; ++j) {
                    if (j < m) {
                        const double pr = ph * V[r * m + j];
                        ut[j] = ut[j] + pr;
                    }
                }
            }
            ac_project<M>(m, ut, u);
#pragma unroll
            for (int j = 0; j < M; ++j) {
                if (j < m) {
                    const double dl = u[j] - U[i * m + j];
                    const double p1 = dl * dl;
                    dn = dn + p1;
                    const double p2 = u[j] * u[j];
                    nn = nn + p2;
                    U[i * m + j] = u[j];
                }
            }
        }
        ac_rhs_row<M>(ii, m, u, labels[i], onepcdt, coefT, dt, omega0, Rs);
    }
    if (!FIRST) {
        // block maxima of the change norms (max is exact in any order)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            dn = fmax(dn, __shfl_xor(dn, off, 64));
            nn = fmax(nn, __shfl_xor(nn, off, 64));
        }
        if ((threadIdx.x & 63) == 0) {
            red[0][threadIdx.x >> 6] = dn;
            red[1][threadIdx.x >> 6] = nn;
        }
    }
    __syncthreads();
    if (!FIRST && threadIdx.x == 0) {
        mxd[ch] = fmax(fmax(red[0][0], red[0][1]), fmax(red[0][2], red[0][3]));
        mxn[ch] = fmax(fmax(red[1][0], red[1][1]), fmax(red[1][2], red[1][3]));
    }
    const double *Zb = Zc + ch * (int64_t)k * kAcChunk;
    for (int q = threadIdx.x; q < k * m; q += blockDim.x) {
        const int r = q / m, c = q - r * m;
        const double2 *z2 = reinterpret_cast<const double2 *>(Zb + (int64_t)r * kAcChunk);
        const double acc = cnt == kAcChunk ? ac_chain<true>(z2, Rs + c, m, cnt)
                                           : ac_chain<false>(z2, Rs + c, m, cnt);
        part[ch * (int64_t)k * m + q] = acc;
    }
}

// Runs CALL with MM = m for 2 <= m <= 16 (register-resident rows), else with
// MM = kAcMaxM and the runtime m.
#define AC_M_SWITCH(m, CALL)                 \
    switch (m) {                             \
        case 2: { constexpr int MM = 2; CALL; break; }   \
        case 3: { constexpr int MM = 3; CALL; break; }   \
        case 4: { constexpr int MM = 4; CALL; break; }   \
        case 5: { constexpr int MM = 5; CALL; break; }   \
        case 6: { constexpr int MM = 6; CALL; break; }   \
        case 7: { constexpr int MM = 7; CALL; break; }   \
        case 8: { constexpr int MM = 8; CALL; break; }   \
        case 9: { constexpr int MM = 9; CALL; break; }   \
        case 10: { constexpr int MM = 10; CALL; break; } \
        case 11: { constexpr int MM = 11; CALL; break; } \
        case 12: { constexpr int MM = 12; CALL; break; } \
        case 13: { constexpr int MM = 13; CALL; break; } \
        case 14: { constexpr int MM = 14; CALL; break; } \
        case 15: { constexpr int MM = 15; CALL; break; } \
        case 16: { constexpr int MM = 16; CALL; break; } \
        default: { constexpr int MM = kAcMaxM; CALL; break; } \
    }

static size_t ac_fused_lds(int k, int m) {
    (void)k;
    return (size_t)((int64_t)kAcChunk * m) * sizeof(double);
}

// Fused steps on chunk-major copies of the eigenvectors and of Z: each step
// reads both once; U is read and written once, the right-hand side never
// leaves the workgroup.
static void ac_run_fused(int64_t n, int k, int m, const double *evals, const double *evecs,
                         int64_t ldv, const int32_t *labels, const mlg_ac_params &prm, double *U,
                         int32_t *pred, int *iters, hipStream_t s) {
    const int64_t nch = (n + kAcChunk - 1) / kAcChunk;
    DevBuf<double> Pc((size_t)nch * k * kAcChunk), Zc((size_t)nch * k * kAcChunk), den(k), mxd(nch),
        mxn(nch);
    DevBuf<double> pa((size_t)nch * k * m), pb((size_t)((nch + 1) / 2) * k * m + 1), mx(2048),
        rcd(1);
    DevBuf<int> bad(1);
    MLG_HIP(hipMemsetAsync(bad.p, 0, 4, s));
    hipLaunchKernelGGL(k_ac_den, dim3(ceil_div(k, 256)), dim3(256), 0, s, k, evals, prm.c, prm.dt,
                       prm.eps, den.p);
    MLG_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_ac_pack, dim3(ceil_div(nch * k * kAcChunk, 256)), dim3(256), 0, s, n, k,
                       nch, evecs, ldv, den.p, Pc.p, Zc.p);
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
    const size_t lds = ac_fused_lds(k, m);
    const int nmx = std::min<int64_t>(1024, ceil_div(nch, 256));
    AC_M_SWITCH(m, hipLaunchKernelGGL((k_ac_iter<MM, true>), dim3((unsigned)nch), dim3(kAcChunk), lds,
                                      s, n, k, m, Pc.p, Zc.p, nullptr, U, labels, onepcdt, coefT,
                                      prm.dt, prm.omega0, pa.p, mxd.p, mxn.p));
    MLG_LAUNCH_CHECK();
    // one step: tree over the chunk partials, the fused step, the change
    // maximum.  The same launches with the same buffers every step, so they
    // are captured once and replayed (no memset nodes: the step writes every
    // value it later reads).
    auto step = [&]() {
        double *src = ac_tree_reduce(nch, k * m, pa.p, pb.p, s);
        // src holds V; the step overwrites pa with the next partials
        double *Vd = src;
        if (src == pa.p) {
            MLG_HIP(hipMemcpyAsync(pb.p, pa.p, sizeof(double) * k * m, hipMemcpyDeviceToDevice, s));
            Vd = pb.p;
        }
        AC_M_SWITCH(m, hipLaunchKernelGGL((k_ac_iter<MM, false>), dim3((unsigned)nch), dim3(kAcChunk),
                                          lds, s, n, k, m, Pc.p, Zc.p, Vd, U, labels, onepcdt, coefT,
                                          prm.dt, prm.omega0, pa.p, mxd.p, mxn.p));
        MLG_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_max2, dim3(nmx), dim3(256), 0, s, nch, mxd.p, mxn.p, mx.p);
        MLG_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_ac_finish_max, dim3(1), dim3(64), 0, s, nmx, mx.p, rcd.p);
        MLG_LAUNCH_CHECK();
    };
    struct GraphExec {
        hipGraphExec_t e = nullptr;
        ~GraphExec() {
            if (e) (void)hipGraphExecDestroy(e);
        }
    } gx;
    {
        hipGraph_t graph;
        MLG_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        try {
            step();
        } catch (...) {
            hipGraph_t junk = nullptr;
            (void)hipStreamEndCapture(s, &junk);
            if (junk) (void)hipGraphDestroy(junk);
            throw;
        }
        MLG_HIP(hipStreamEndCapture(s, &graph));
        const hipError_t e = hipGraphInstantiate(&gx.e, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        MLG_HIP(e);
    }
    int l = 0;
    double rc = 0.0;
    do {
        MLG_HIP(hipGraphLaunch(gx.e, s));
        MLG_HIP(hipMemcpyAsync(&rc, rcd.p, 8, hipMemcpyDeviceToHost, s));
        MLG_HIP(hipStreamSynchronize(s));
        l = l + 1;
    } while (rc > prm.tol && l < prm.max_iter);
    hipLaunchKernelGGL(k_ac_argmax, dim3(ceil_div(n, 256)), dim3(256), 0, s, n, m, U, pred);
    MLG_LAUNCH_CHECK();
    MLG_HIP(hipStreamSynchronize(s));
    *iters = l;
}

void ac_run(int64_t n, int k, int m, const double *evals, const double *evecs, int64_t ldv,
            const int32_t *labels, const mlg_ac_params &prm, double *U, int32_t *pred, int *iters,
            hipStream_t s) {
    MLG_REQUIRE(m <= kAcMaxM, MLG_ERR_ARG, "m must be <= 64");
    if (m <= kAcFastM && ac_fused_lds(k, m) <= 65536) {
        ac_run_fused(n, k, m, evals, evecs, ldv, labels, prm, U, pred, iters, s);
        return;
    }
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
    const size_t v_lds = (size_t)k * m * sizeof(double);
    const bool v_in_lds = v_lds <= 65536;
    int l = 0;
    double rc = 0.0;
    AC_M_SWITCH(m, hipLaunchKernelGGL(k_ac_rhs<MM>, dim3(ceil_div(n, 256)), dim3(256), 0, s, n, m, U,
                                      labels, onepcdt, coefT, prm.dt, prm.omega0, R.p));
    MLG_LAUNCH_CHECK();
    do {
        hipLaunchKernelGGL(k_ac_zr, dim3((unsigned)nch), dim3(256), 0, s, n, k, m, Z.p, R.p, pa.p);
        MLG_LAUNCH_CHECK();
        double *src = ac_tree_reduce(nch, k * m, pa.p, pb.p, s);
        if (v_in_lds) {
            AC_M_SWITCH(m, hipLaunchKernelGGL((k_ac_update<MM, true>), dim3(ceil_div(n, 256)),
                                              dim3(256), v_lds, s, n, k, m, evecs, ldv, src, U,
                                              rowd.p, rown.p, labels, onepcdt, coefT, prm.dt,
                                              prm.omega0, R.p));
        } else {
            AC_M_SWITCH(m, hipLaunchKernelGGL((k_ac_update<MM, false>), dim3(ceil_div(n, 256)),
                                              dim3(256), 0, s, n, k, m, evecs, ldv, src, U, rowd.p,
                                              rown.p, labels, onepcdt, coefT, prm.dt, prm.omega0,
                                              R.p));
        }
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
