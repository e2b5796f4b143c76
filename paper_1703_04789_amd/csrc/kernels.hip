// Device kernels of the SP-MPS hot path for gfx950 (FP64).
//
// Every contraction of the one-site sweep -- environment updates (Fig.
// [spmpsOpt]) and the local products H_eff x, N_eff x (Eq. [geproblem]) --
// is a list of small dense products between particle-number blocks of the
// environments and (N, M) blocks of the site tensor.  The host runtime
// precomputes these lists once per site (the block structure is fixed); the
// kernels below execute them.  All reductions run in a fixed order (no
// floating-point atomics), so repeated calls give bitwise-identical results.
#include "kernels.h"

namespace spk {

namespace {

constexpr int kThreads = 256;

__device__ inline double block_sum(double v, double* red) {
    // fixed-order tree reduction over the work-group (blockDim.x power of 2)
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    double r = red[0];
    __syncthreads();
    return r;
}

__device__ inline double term_dot(const BufSet& bufs, const BTerm& tm, int r, int c) {
    const double* A = bufs.p[tm.a_buf] + tm.a_off + (long long)r * tm.a_rs;
    const double* B = bufs.p[tm.b_buf] + tm.b_off + (long long)c * tm.b_cs;
    double s = 0.0;
    for (int k = 0; k < tm.K; ++k) s = fma(A[(long long)k * tm.a_cs], B[(long long)k * tm.b_rs], s);
    return s;
}

__global__ __launch_bounds__(kThreads) void k_bgemm(const BTask* __restrict__ tasks,
                                                      const BTerm* __restrict__ terms, BufSet bufs,
                                                      const double* __restrict__ coef) {
    __shared__ double red[kThreads];
    const BTask tk = tasks[blockIdx.x];
    const int MN = tk.M * tk.N;
    if (MN <= 0) return;
    double* C = bufs.p[tk.c_buf] + tk.c_off;
    const int nt = tk.t1 - tk.t0;
    int S = 1;
    if (MN < kThreads && nt > 1) {
        S = kThreads / MN;
        if (S > nt) S = nt;
    }
    if (S == 1) {
        for (int o = threadIdx.x; o < MN; o += kThreads) {
            const int r = o / tk.N, c = o - r * tk.N;
            double acc = 0.0;
            for (int t = tk.t0; t < tk.t1; ++t) {
                const BTerm tm = terms[t];
                acc = fma(coef[tm.cidx], term_dot(bufs, tm, r, c), acc);
            }
            double* cp = C + (long long)r * tk.ldc + c;
            *cp = tk.accumulate ? *cp + acc : acc;
        }
    } else {
        // split the term list over S groups of MN threads, then add the S
        // partial sums in a fixed order
        const int o = threadIdx.x % MN;
        const int sp = threadIdx.x / MN;
        const int r = o / tk.N, c = o - r * tk.N;
        double acc = 0.0;
        if (sp < S) {
            for (int t = tk.t0 + sp; t < tk.t1; t += S) {
                const BTerm tm = terms[t];
                acc = fma(coef[tm.cidx], term_dot(bufs, tm, r, c), acc);
            }
        }
        red[threadIdx.x] = acc;
        __syncthreads();
        if ((int)threadIdx.x < MN) {
            double tot = 0.0;
            for (int q = 0; q < S; ++q) tot += red[q * MN + threadIdx.x];
            double* cp = C + (long long)r * tk.ldc + c;
            *cp = tk.accumulate ? *cp + tot : tot;
        }
    }
}

__global__ __launch_bounds__(kThreads) void k_combine(const CTask* __restrict__ tasks,
                                                        const CTerm* __restrict__ terms,
                                                        BufSet bufs, const double* __restrict__ coef) {
    const CTask tk = tasks[blockIdx.x];
    double* C = bufs.p[tk.c_buf] + tk.c_off;
    for (int e = threadIdx.x; e < tk.n; e += kThreads) {
        double acc = 0.0;
        for (int t = tk.t0; t < tk.t1; ++t) {
            const CTerm tm = terms[t];
            acc = fma(coef[tm.cidx], bufs.p[tm.a_buf][tm.a_off + e], acc);
        }
        C[e] = acc;
    }
}

__global__ __launch_bounds__(kThreads) void k_diag(const DiagBlk* __restrict__ blks,
                                                     const DiagTerm* __restrict__ terms,
                                                     const double* __restrict__ lenv, long long lsize,
                                                     const double* __restrict__ renv, long long rsize,
                                                     const double* __restrict__ coef, int ncoef, int G,
                                                     double* __restrict__ out) {
    const DiagBlk b = blks[blockIdx.x];
    const int n = b.rows * b.cols;
    for (int e = threadIdx.x; e < n; e += kThreads) {
        const int r = e / b.cols, c = e - r * b.cols;
        double acc = 0.0;
        for (int g = 0; g < G; ++g) {
            for (int t = b.t0; t < b.t1; ++t) {
                const DiagTerm tm = terms[t];
                const double lv = lenv[g * lsize + tm.l_off + (long long)r * (tm.l_ld + 1)];
                const double rv = renv[g * rsize + tm.r_off + (long long)c * (tm.r_ld + 1)];
                acc = fma(coef[g * ncoef + tm.cidx], lv * rv, acc);
            }
        }
        out[b.x_off + e] = acc;
    }
}

// Householder QR of one gathered sector matrix (rows >= cols), column-major
// in scratch; Q overwrites the pieces, R (cols x cols, row-major) goes to
// rout.  Signs are fixed so that diag(R) >= 0 (the unique QR of a full-rank
// matrix).
__global__ __launch_bounds__(kThreads) void k_qr(const QrTask* __restrict__ tasks,
                                                   const QrPiece* __restrict__ pieces,
                                                   double* __restrict__ site,
                                                   double* __restrict__ scratch,
                                                   double* __restrict__ rout) {
    __shared__ double red[kThreads];
    __shared__ double tau_s[256];
    __shared__ double diag_s[256];
    __shared__ double dots[256];
    const QrTask tk = tasks[blockIdx.x];
    const int rows = tk.rows, cols = tk.cols;
    double* S = scratch + tk.scratch_off;           // rows x cols, column-major
    double* Q = S + (long long)rows * cols;          // rows x cols, column-major
    // gather
    for (int p = tk.p0; p < tk.p1; ++p) {
        const QrPiece pc = pieces[p];
        const int nr = pc.transposed ? pc.pcol : pc.prow;
        const int nel = nr * cols;
        for (int e = threadIdx.x; e < nel; e += kThreads) {
            const int rr = e / cols, cc = e - rr * cols;
            const double v = pc.transposed ? site[pc.off + (long long)cc * pc.pcol + rr]
                                           : site[pc.off + (long long)rr * pc.pcol + cc];
            S[(long long)cc * rows + pc.row0 + rr] = v;
        }
    }
    __syncthreads();
    for (int j = 0; j < cols; ++j) {
        double ss = 0.0;
        for (int r = j + threadIdx.x; r < rows; r += kThreads) {
            const double v = S[(long long)j * rows + r];
            ss = fma(v, v, ss);
        }
        ss = block_sum(ss, red);
        if (threadIdx.x == 0) {
            const double x0 = S[(long long)j * rows + j];
            const double nrm = sqrt(ss);
            const double alpha = (x0 >= 0.0) ? -nrm : nrm;
            const double v0 = x0 - alpha;
            const double vv = ss - x0 * x0 + v0 * v0;
            tau_s[j] = (vv > 0.0) ? 2.0 / vv : 0.0;
            diag_s[j] = alpha;
            S[(long long)j * rows + j] = v0;
        }
        __syncthreads();
        const double tau = tau_s[j];
        for (int c = j + 1 + threadIdx.x; c < cols; c += kThreads) {
            double d = 0.0;
            for (int r = j; r < rows; ++r) d = fma(S[(long long)j * rows + r], S[(long long)c * rows + r], d);
            const double f = tau * d;
            for (int r = j; r < rows; ++r) S[(long long)c * rows + r] -= f * S[(long long)j * rows + r];
        }
        __syncthreads();
    }
    // R (row-major) with the sign fix
    double* R = rout + tk.r_off;
    for (int e = threadIdx.x; e < cols * cols; e += kThreads) {
        const int i = e / cols, c = e - i * cols;
        double v = 0.0;
        if (c == i) v = diag_s[i];
        else if (c > i) v = S[(long long)c * rows + i];
        if (diag_s[i] < 0.0) v = -v;
        R[e] = v;
    }
    // Q = H_0 ... H_{cols-1} [I; 0]
    for (int e = threadIdx.x; e < rows * cols; e += kThreads) {
        const int c = e / rows, r = e - c * rows;
        Q[e] = (r == c) ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int j = cols - 1; j >= 0; --j) {
        const double tau = tau_s[j];
        for (int c = threadIdx.x; c < cols; c += kThreads) {
            double d = 0.0;
            for (int r = j; r < rows; ++r) d = fma(S[(long long)j * rows + r], Q[(long long)c * rows + r], d);
            dots[c] = tau * d;
        }
        __syncthreads();
        const int span = rows - j;
        for (int e = threadIdx.x; e < span * cols; e += kThreads) {
            const int c = e / span, r = j + (e - c * span);
            Q[(long long)c * rows + r] -= dots[c] * S[(long long)j * rows + r];
        }
        __syncthreads();
    }
    // scatter Q with the sign fix
    for (int p = tk.p0; p < tk.p1; ++p) {
        const QrPiece pc = pieces[p];
        const int nr = pc.transposed ? pc.pcol : pc.prow;
        const int nel = nr * cols;
        for (int e = threadIdx.x; e < nel; e += kThreads) {
            const int rr = e / cols, cc = e - rr * cols;
            double v = Q[(long long)cc * rows + pc.row0 + rr];
            if (diag_s[cc] < 0.0) v = -v;
            if (pc.transposed) site[pc.off + (long long)cc * pc.pcol + rr] = v;
            else site[pc.off + (long long)rr * pc.pcol + cc] = v;
        }
    }
}

// ---- Davidson vector kernels --------------------------------------------

__global__ __launch_bounds__(1024) void k_normalize(const double* __restrict__ in,
                                                     double* __restrict__ out, int n,
                                                     double* __restrict__ norm_out) {
    __shared__ double red[1024];
    double ss = 0.0;
    for (int e = threadIdx.x; e < n; e += 1024) ss = fma(in[e], in[e], ss);
    ss = block_sum(ss, red);
    const double nrm = sqrt(ss);
    const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
    for (int e = threadIdx.x; e < n; e += 1024) out[e] = in[e] * inv;
    if (threadIdx.x == 0 && norm_out) *norm_out = nrm;
}

__global__ __launch_bounds__(kThreads) void k_ritz(const double* __restrict__ V,
                                                     const double* __restrict__ HV,
                                                     const double* __restrict__ NV, long long ld,
                                                     int m, const double* __restrict__ a,
                                                     const double* __restrict__ theta_p,
                                                     const double* __restrict__ dh,
                                                     const double* __restrict__ dn, int n,
                                                     double floor_, double* __restrict__ x,
                                                     double* __restrict__ t,
                                                     double* __restrict__ partials) {
    __shared__ double red[kThreads];
    const int e = blockIdx.x * kThreads + threadIdx.x;
    const double theta = *theta_p;
    double xx = 0.0, uu = 0.0, xn = 0.0;
    if (e < n) {
        double xv = 0.0, hv = 0.0, nv = 0.0;
        for (int j = 0; j < m; ++j) {
            const double aj = a[j];
            xv = fma(aj, V[j * ld + e], xv);
            hv = fma(aj, HV[j * ld + e], hv);
            nv = fma(aj, NV[j * ld + e], nv);
        }
        const double u = hv - theta * nv;
        double den = dh[e] - theta * dn[e];
        if (fabs(den) < floor_) den = (den < 0.0) ? -floor_ : floor_;
        x[e] = xv;
        t[e] = -u / den;
        xx = xv * xv;
        uu = u * u;
        xn = xv * nv;
    }
    xx = block_sum(xx, red);
    uu = block_sum(uu, red);
    xn = block_sum(xn, red);
    if (threadIdx.x == 0) {
        partials[3 * blockIdx.x + 0] = xx;
        partials[3 * blockIdx.x + 1] = uu;
        partials[3 * blockIdx.x + 2] = xn;
    }
}

__global__ __launch_bounds__(kThreads) void k_multidot(const double* __restrict__ A, long long ld,
                                                         const double* __restrict__ u, int n,
                                                         double* __restrict__ out) {
    __shared__ double red[kThreads];
    const double* a = A + blockIdx.x * ld;
    double s = 0.0;
    for (int e = threadIdx.x; e < n; e += kThreads) s = fma(a[e], u[e], s);
    s = block_sum(s, red);
    if (threadIdx.x == 0) out[blockIdx.x] = s;
}

__global__ __launch_bounds__(kThreads) void k_sub_combo(const double* __restrict__ A, long long ld,
                                                          int m, const double* __restrict__ c,
                                                          double* __restrict__ t, int n) {
    const int e = blockIdx.x * kThreads + threadIdx.x;
    if (e >= n) return;
    double s = 0.0;
    for (int j = 0; j < m; ++j) s = fma(c[j], A[j * ld + e], s);
    t[e] -= s;
}

__global__ __launch_bounds__(kThreads) void k_basis_rotate(const double* __restrict__ A,
                                                             long long ld, int m,
                                                             const double* __restrict__ Q, int keep,
                                                             double* __restrict__ out, int n) {
    const int e = blockIdx.x * kThreads + threadIdx.x;
    if (e >= n) return;
    for (int i = 0; i < keep; ++i) {
        double s = 0.0;
        for (int j = 0; j < m; ++j) s = fma(Q[j * keep + i], A[j * ld + e], s);
        out[i * ld + e] = s;
    }
}

__global__ __launch_bounds__(kThreads) void k_gram(const double* __restrict__ V,
                                                     const double* __restrict__ HV,
                                                     const double* __restrict__ NV, long long ld,
                                                     int m, int n, const double* __restrict__ part,
                                                     int npart, double* __restrict__ out) {
    __shared__ double red[kThreads];
    const int b = blockIdx.x;
    const double *pa, *pb;
    if (b <= m) {
        pa = V + b * ld;
        pb = HV + m * ld;
    } else if (b <= 2 * m + 1) {
        pa = V + (b - m - 1) * ld;
        pb = NV + m * ld;
    } else if (b <= 3 * m + 1) {
        pa = V + m * ld;
        pb = HV + (b - 2 * m - 2) * ld;
    } else if (b <= 4 * m + 1) {
        pa = V + m * ld;
        pb = NV + (b - 3 * m - 2) * ld;
    } else {
        // fold the Ritz-kernel partial sums in a fixed order
        if (threadIdx.x < 3) {
            double s = 0.0;
            for (int i = 0; i < npart; ++i) s += part[3 * i + threadIdx.x];
            out[4 * m + 2 + threadIdx.x] = s;
        }
        return;
    }
    double s = 0.0;
    for (int e = threadIdx.x; e < n; e += kThreads) s = fma(pa[e], pb[e], s);
    s = block_sum(s, red);
    if (threadIdx.x == 0) out[b] = s;
}

__global__ __launch_bounds__(kThreads) void k_scale(double* __restrict__ x, int n,
                                                      const double* __restrict__ ss) {
    const int e = blockIdx.x * kThreads + threadIdx.x;
    if (e >= n) return;
    const double s = *ss;
    x[e] = s > 0.0 ? x[e] / sqrt(s) : x[e];
}

// 64x64 output tile per work-group of 256 threads (16 x 16 threads, 4 x 4
// outputs each, rows ty + 16 i and columns tx + 16 j); K staged through LDS
// in chunks of 16 with coalesced global loads for either operand layout.
constexpr int kKC = 16;

__global__ __launch_bounds__(kThreads) void k_tgemm(const TTask* __restrict__ tasks,
                                                      const TSeg* __restrict__ segs, BufSet bufs,
                                                      const double* __restrict__ coef,
                                                      const int* __restrict__ map) {
    __shared__ double As[kKC][kTile + 1];
    __shared__ double Bs[kKC][kTile + 1];
    const TTask tk = tasks[blockIdx.x];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    double acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
    for (int s = tk.s0; s < tk.s1; ++s) {
        const TSeg sg = segs[s];
        const double cf = coef[sg.cidx];
        const double* __restrict__ A = bufs.p[sg.a_buf] + sg.a_off;
        const double* __restrict__ B = bufs.p[sg.b_buf] + sg.b_off;
        for (int kb = sg.k0; kb < sg.k1; kb += kKC) {
            for (int idx = threadIdx.x; idx < kTile * kKC; idx += kThreads) {
                int r, k;
                if (sg.ta == 0) {
                    r = idx / kKC;
                    k = idx % kKC;
                } else {
                    k = idx / kTile;
                    r = idx % kTile;
                }
                const int gr = tk.r0 + r, gk = kb + k;
                double v = 0.0;
                if (gr < tk.M && gk < sg.k1)
                    v = (sg.ta == 0) ? A[(long long)gr * sg.lda + gk] : A[(long long)gk * sg.lda + gr];
                As[k][r] = cf * v;
            }
            for (int idx = threadIdx.x; idx < kTile * kKC; idx += kThreads) {
                int c, k;
                if (sg.tb == 0) {
                    k = idx / kTile;
                    c = idx % kTile;
                } else {
                    c = idx / kKC;
                    k = idx % kKC;
                }
                const int gc = tk.c0 + c, gk = kb + k;
                double v = 0.0;
                if (gc < tk.N && gk < sg.k1)
                    v = (sg.tb == 0) ? B[(long long)gk * sg.ldb + gc] : B[(long long)gc * sg.ldb + gk];
                Bs[k][c] = v;
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < kKC; ++k) {
                double a[4], b[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) a[i] = As[k][ty + 16 * i];
#pragma unroll
                for (int j = 0; j < 4; ++j) b[j] = Bs[k][tx + 16 * j];
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
            }
            __syncthreads();
        }
    }
    double* C = bufs.p[tk.c_buf] + tk.c_off;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int r = tk.r0 + ty + 16 * i;
        if (r >= tk.M) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int c = tk.c0 + tx + 16 * j;
            if (c >= tk.N) continue;
            if (tk.mode == 0) {
                C[(long long)r * tk.ldc + c] = acc[i][j];
            } else {
                const int p = map[tk.pack_off + (long long)r * tk.N + c];
                if (p >= 0) C[p] = acc[i][j];
            }
        }
    }
}

__global__ __launch_bounds__(kThreads) void k_gather(const int* __restrict__ map, const double* __restrict__ src,
                                                       double* __restrict__ dst, long long n) {
    const long long e = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (e >= n) return;
    const int p = map[e];
    dst[e] = p >= 0 ? src[p] : 0.0;
}

__global__ __launch_bounds__(kThreads) void k_gsum2(const double* __restrict__ pa, const double* __restrict__ pb,
                                                      long long stride, int G, int n, double* __restrict__ outa,
                                                      double* __restrict__ outb) {
    const int e = blockIdx.x * kThreads + threadIdx.x;
    if (e >= n) return;
    double sa = 0.0, sb = 0.0;
    for (int g = 0; g < G; ++g) {
        sa += pa[g * stride + e];
        sb += pb[g * stride + e];
    }
    outa[e] = sa;
    outb[e] = sb;
}

inline int nblk(int n) { return (n + kThreads - 1) / kThreads; }

}  // namespace

void tgemm(hipStream_t s, const TTask* tasks, int ntasks, const TSeg* segs, BufSet bufs, const double* coef,
           const int* map) {
    if (ntasks > 0) hipLaunchKernelGGL(k_tgemm, dim3(ntasks), dim3(kThreads), 0, s, tasks, segs, bufs, coef, map);
}
void gather(hipStream_t s, const int* map, const double* src, double* dst, long long n) {
    if (n > 0) hipLaunchKernelGGL(k_gather, dim3((unsigned)((n + kThreads - 1) / kThreads)), dim3(kThreads), 0, s, map, src, dst, n);
}
void gsum2(hipStream_t s, const double* pa, const double* pb, long long stride, int G, int n, double* outa,
           double* outb) {
    hipLaunchKernelGGL(k_gsum2, dim3(nblk(n)), dim3(kThreads), 0, s, pa, pb, stride, G, n, outa, outb);
}
void bgemm(hipStream_t s, const BTask* tasks, int ntasks, const BTerm* terms, BufSet bufs,
           const double* coef) {
    if (ntasks > 0) hipLaunchKernelGGL(k_bgemm, dim3(ntasks), dim3(kThreads), 0, s, tasks, terms, bufs, coef);
}
void combine(hipStream_t s, const CTask* tasks, int ntasks, const CTerm* terms, BufSet bufs,
             const double* coef) {
    if (ntasks > 0) hipLaunchKernelGGL(k_combine, dim3(ntasks), dim3(kThreads), 0, s, tasks, terms, bufs, coef);
}
void heff_diag(hipStream_t s, const DiagBlk* blks, int nb, const DiagTerm* terms, const double* lenv,
               long long lsize, const double* renv, long long rsize, const double* coef, int ncoef,
               int G, double* out) {
    if (nb > 0)
        hipLaunchKernelGGL(k_diag, dim3(nb), dim3(kThreads), 0, s, blks, terms, lenv, lsize, renv, rsize,
                           coef, ncoef, G, out);
}
void qr_sectors(hipStream_t s, const QrTask* tasks, int ntasks, const QrPiece* pieces, double* site,
                double* scratch, double* rout) {
    if (ntasks > 0) hipLaunchKernelGGL(k_qr, dim3(ntasks), dim3(kThreads), 0, s, tasks, pieces, site, scratch, rout);
}
void normalize(hipStream_t s, const double* in, double* out, int n, double* norm_out) {
    hipLaunchKernelGGL(k_normalize, dim3(1), dim3(1024), 0, s, in, out, n, norm_out);
}
void ritz(hipStream_t s, const double* V, const double* HV, const double* NV, long long ld, int m,
          const double* a, const double* theta, const double* dh, const double* dn, int n, double floor_,
          double* x, double* t, double* partials, int* nblocks_out) {
    const int nb = nblk(n);
    hipLaunchKernelGGL(k_ritz, dim3(nb), dim3(kThreads), 0, s, V, HV, NV, ld, m, a, theta, dh, dn, n, floor_,
                       x, t, partials);
    if (nblocks_out) *nblocks_out = nb;
}
void multidot(hipStream_t s, const double* A, long long ld, int m, const double* u, int n, double* out) {
    if (m > 0) hipLaunchKernelGGL(k_multidot, dim3(m), dim3(kThreads), 0, s, A, ld, u, n, out);
}
void sub_combo(hipStream_t s, const double* A, long long ld, int m, const double* c, double* t, int n) {
    if (m > 0) hipLaunchKernelGGL(k_sub_combo, dim3(nblk(n)), dim3(kThreads), 0, s, A, ld, m, c, t, n);
}
void basis_rotate(hipStream_t s, const double* A, long long ld, int m, const double* Q, int keep,
                  double* out, int n) {
    hipLaunchKernelGGL(k_basis_rotate, dim3(nblk(n)), dim3(kThreads), 0, s, A, ld, m, Q, keep, out, n);
}
void gram(hipStream_t s, const double* V, const double* HV, const double* NV, long long ld, int m, int n,
          const double* partials, int npart, double* out) {
    hipLaunchKernelGGL(k_gram, dim3(4 * m + 3), dim3(kThreads), 0, s, V, HV, NV, ld, m, n, partials, npart, out);
}
void scale(hipStream_t s, double* x, int n, const double* ss) {
    hipLaunchKernelGGL(k_scale, dim3(nblk(n)), dim3(kThreads), 0, s, x, n, ss);
}

}  // namespace spk
