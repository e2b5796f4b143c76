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

__device__ inline double wave_sum64(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

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
    // the task's terms (source pointer, coefficient) are staged in LDS by one
    // thread each, 64 at a time, so that the element loop issues independent
    // loads; every element still sums its terms in list order
    constexpr int kTermsAtOnce = 64, kPer = 4;
    __shared__ const double* sp[kTermsAtOnce];
    __shared__ double sc[kTermsAtOnce];
    const CTask tk = tasks[blockIdx.x];
    double* C = bufs.p[tk.c_buf] + tk.c_off;
    for (int eb = 0; eb < tk.n; eb += kPer * kThreads) {
        double acc[kPer];
#pragma unroll
        for (int u = 0; u < kPer; ++u) acc[u] = 0.0;
        for (int tb = tk.t0; tb < tk.t1; tb += kTermsAtOnce) {
            const int nt = min(kTermsAtOnce, tk.t1 - tb);
            __syncthreads();
            if ((int)threadIdx.x < nt) {
                const CTerm tm = terms[tb + threadIdx.x];
                sp[threadIdx.x] = bufs.p[tm.a_buf] + tm.a_off;
                sc[threadIdx.x] = coef[tm.cidx];
            }
            __syncthreads();
            for (int t = 0; t < nt; ++t) {
                const double* __restrict__ a = sp[t];
                const double c = sc[t];
#pragma unroll
                for (int u = 0; u < kPer; ++u) {
                    const int e = eb + threadIdx.x + u * kThreads;
                    if (e < tk.n) acc[u] = fma(c, a[e], acc[u]);
                }
            }
        }
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int e = eb + threadIdx.x + u * kThreads;
            if (e < tk.n) C[e] = acc[u];
        }
    }
}

// Diagonal of H_eff (or N_eff) for one packed (N, M) block: for element
// (r, c), sum over g and the block's terms t of coef * L_g,t(r, r) * R_g,t(c, c).
// The (g, t) range, g outer, is cut into gridDim.y equal parts: part j sums
// its range in order and writes part[j * ntot + index] (one part: straight
// to out), and k_diag_sum adds the parts in ascending j.  Wide MPOs have
// thousands of terms per block, so one work-group per block would run them
// all in sequence.
__global__ __launch_bounds__(kThreads) void k_diag(const DiagBlk* __restrict__ blks,
                                                     const DiagTerm* __restrict__ terms,
                                                     const double* __restrict__ lenv, long long lsize,
                                                     const double* __restrict__ renv, long long rsize,
                                                     const double* __restrict__ coef, int ncoef, int G,
                                                     double* __restrict__ out, double* __restrict__ part,
                                                     long long ntot) {
    const DiagBlk b = blks[blockIdx.x];
    const int n = b.rows * b.cols;
    const int T = b.t1 - b.t0, nsplit = gridDim.y, j = blockIdx.y;
    const long long U = (long long)G * T;
    const long long u0 = U * j / nsplit, u1 = U * (j + 1) / nsplit;
    for (int e = threadIdx.x; e < n; e += kThreads) {
        const int r = e / b.cols, c = e - r * b.cols;
        double acc = 0.0;
        if (T > 0) {
            int g = int(u0 / T), t = b.t0 + int(u0 % T);
            for (long long u = u0; u < u1; ++u) {
                const DiagTerm tm = terms[t];
                const double lv = lenv[g * lsize + tm.l_off + (long long)r * (tm.l_ld + 1)];
                const double rv = renv[g * rsize + tm.r_off + (long long)c * (tm.r_ld + 1)];
                acc = fma(coef[g * ncoef + tm.cidx], lv * rv, acc);
                if (++t == b.t1) {
                    t = b.t0;
                    ++g;
                }
            }
        }
        if (nsplit == 1) out[b.x_off + e] = acc;
        else part[(long long)j * ntot + b.x_off + e] = acc;
    }
}

__global__ __launch_bounds__(kThreads) void k_diag_sum(const double* __restrict__ part, int nsplit, long long ntot,
                                                         double* __restrict__ out) {
    const long long e = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (e >= ntot) return;
    double acc = 0.0;
    for (int j = 0; j < nsplit; ++j) acc += part[(long long)j * ntot + e];
    out[e] = acc;
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

// The same factorisation with both matrices in LDS: the norm of the pivot
// column is a wave reduction, and each trailing (or Q) column is updated by
// one wave (lanes over rows, dot product by cross-lane shuffles).
__global__ __launch_bounds__(kThreads) void k_qr_lds(const QrTask* __restrict__ tasks,
                                                       const QrPiece* __restrict__ pieces,
                                                       double* __restrict__ site, double* __restrict__ rout) {
    extern __shared__ double sh[];
    __shared__ double tau_s[256];
    __shared__ double diag_s[256];
    const QrTask tk = tasks[blockIdx.x];
    const int rows = tk.rows, cols = tk.cols;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double* S = sh;                       // rows x cols, column-major
    double* Q = sh + (long long)rows * cols;
    for (int p = tk.p0; p < tk.p1; ++p) {
        const QrPiece pc = pieces[p];
        const int nr = pc.transposed ? pc.pcol : pc.prow;
        const int nel = nr * cols;
        for (int e = threadIdx.x; e < nel; e += kThreads) {
            const int rr = e / cols, cc = e - rr * cols;
            const double v = pc.transposed ? site[pc.off + (long long)cc * pc.pcol + rr]
                                           : site[pc.off + (long long)rr * pc.pcol + cc];
            S[cc * rows + pc.row0 + rr] = v;
        }
    }
    __syncthreads();
    for (int j = 0; j < cols; ++j) {
        const double* sj = S + j * rows;
        if (wave == 0) {
            double ss = 0.0;
            for (int r = j + lane; r < rows; r += 64) ss = fma(sj[r], sj[r], ss);
            ss = wave_sum64(ss);
            if (lane == 0) {
                const double x0 = sj[j];
                const double nrm = sqrt(ss);
                const double alpha = (x0 >= 0.0) ? -nrm : nrm;
                const double v0 = x0 - alpha;
                const double vv = ss - x0 * x0 + v0 * v0;
                tau_s[j] = (vv > 0.0) ? 2.0 / vv : 0.0;
                diag_s[j] = alpha;
                S[j * rows + j] = v0;
            }
        }
        __syncthreads();
        const double tau = tau_s[j];
        for (int c = j + 1 + wave; c < cols; c += kThreads / 64) {
            double* sc = S + c * rows;
            double d = 0.0;
            for (int r = j + lane; r < rows; r += 64) d = fma(sj[r], sc[r], d);
            const double f = tau * wave_sum64(d);
            for (int r = j + lane; r < rows; r += 64) sc[r] -= f * sj[r];
        }
        __syncthreads();
    }
    double* R = rout + tk.r_off;
    for (int e = threadIdx.x; e < cols * cols; e += kThreads) {
        const int i = e / cols, c = e - i * cols;
        double v = 0.0;
        if (c == i) v = diag_s[i];
        else if (c > i) v = S[c * rows + i];
        if (diag_s[i] < 0.0) v = -v;
        R[e] = v;
    }
    for (int e = threadIdx.x; e < rows * cols; e += kThreads) {
        const int c = e / rows, r = e - c * rows;
        Q[e] = (r == c) ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int j = cols - 1; j >= 0; --j) {
        const double tau = tau_s[j];
        const double* sj = S + j * rows;
        for (int c = wave; c < cols; c += kThreads / 64) {
            double* qc = Q + c * rows;
            double d = 0.0;
            for (int r = j + lane; r < rows; r += 64) d = fma(sj[r], qc[r], d);
            const double f = tau * wave_sum64(d);
            for (int r = j + lane; r < rows; r += 64) qc[r] -= f * sj[r];
        }
        __syncthreads();
    }
    for (int p = tk.p0; p < tk.p1; ++p) {
        const QrPiece pc = pieces[p];
        const int nr = pc.transposed ? pc.pcol : pc.prow;
        const int nel = nr * cols;
        for (int e = threadIdx.x; e < nel; e += kThreads) {
            const int rr = e / cols, cc = e - rr * cols;
            double v = Q[cc * rows + pc.row0 + rr];
            if (diag_s[cc] < 0.0) v = -v;
            if (pc.transposed) site[pc.off + (long long)cc * pc.pcol + rr] = v;
            else site[pc.off + (long long)rr * pc.pcol + cc] = v;
        }
    }
}

// ---- Davidson vector kernels --------------------------------------------

__global__ __launch_bounds__(kThreads) void k_fill(double* __restrict__ p, long long n, double value) {
    for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < n; i += (long long)gridDim.x * kThreads)
        p[i] = value;
}

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

// out_i = sum_j Q[j][i] A_j for i < keep: eight outputs per pass, the A
// loads of a pass batched eight vectors at a time
__global__ __launch_bounds__(kThreads) void k_basis_rotate(const double* __restrict__ A,
                                                             long long ld, int m,
                                                             const double* __restrict__ Q, int keep,
                                                             double* __restrict__ out, int n) {
    const int e = blockIdx.x * kThreads + threadIdx.x;
    if (e >= n) return;
    for (int i0 = 0; i0 < keep; i0 += 8) {
        double acc[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc[u] = 0.0;
        for (int j0 = 0; j0 < m; j0 += 8) {
            double av[8];
#pragma unroll
            for (int v = 0; v < 8; ++v) av[v] = (j0 + v < m) ? A[(long long)(j0 + v) * ld + e] : 0.0;
#pragma unroll
            for (int v = 0; v < 8; ++v) {
                if (j0 + v >= m) break;
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (i0 + u < keep) acc[u] = fma(Q[(j0 + v) * keep + i0 + u], av[v], acc[u]);
            }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (i0 + u < keep) out[(long long)(i0 + u) * ld + e] = acc[u];
    }
}

// TILE x TILE output tile per work-group of (TILE/4)^2 threads, i.e.
// (TILE/32)^2 wavefronts; each wavefront owns a 32 x 32 quarter (TILE = 64)
// or the whole tile (TILE = 32) as 2 x 2 FP64 matrix-core blocks of 16 x 16
// (v_mfma_f64_16x16x4: lane l supplies A(l % 16, l / 16) and B(l / 16, l % 16)
// of a 16 x 4 by 4 x 16 step and holds D(4 v + l / 16, l % 16), v < 4).  K is
// staged through LDS in chunks of kKC with coalesced global loads for either
// operand layout, zero-padded past the segment and the tile edge.  The chunk
// is short (8) so that a 64-thread work-group needs 4 KB of LDS and a CU can
// hold as many of these latency-bound work-groups as it has wave slots (a
// chunk of 16 halves that and is 1.3x slower at the ab-initio centre, 32 is
// 1.8x slower); the chunk size does not change the sequence of 4-deep steps,
// so results are the same bits for any chunk.  The chunks of all segments
// run as one sequence in which each chunk's global loads are issued before
// the products of the previous one: 1.14x faster than a plain load-then-
// multiply loop at the K = 12 ab-initio centre in the 64-thread tile, and
// 1.16-1.23x at K = 16-24 in the 256-thread tile (36 VGPRs, 7 waves per
// SIMD; an earlier form of that tile had needed enough registers to halve
// its occupancy and was slower).  TILE = 64
// (256 threads) for wide particle-number blocks, 32 (64 threads) for narrow
// ones; every output accumulates the same sequence of 4-deep matrix-core
// steps for either tile, so both tiles give the same bits.
constexpr int kKC = 8;
typedef double d4_t __attribute__((ext_vector_type(4)));

template <int TILE>
__global__ __launch_bounds__((TILE / 4) * (TILE / 4)) void k_tgemm(const TTask* __restrict__ tasks,
                                                                  const TSeg* __restrict__ segs, BufSet bufs,
                                                                  const double* __restrict__ coef,
                                                                  const int* __restrict__ map) {
    constexpr int NT = (TILE / 4) * (TILE / 4), WPR = TILE / 32;
    static_assert(NT == 64 * WPR * WPR, "one wavefront per 32 x 32 quarter");
    __shared__ double As[kKC][TILE + 1];
    __shared__ double Bs[kKC][TILE + 1];
    const TTask tk = tasks[blockIdx.x];
    const int lane = threadIdx.x % 64, wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
    const int wr = (wave / WPR) * 32, wc = (wave % WPR) * 32;
    // the 16 x 16 blocks of the wavefront's quarter that hold outputs of the
    // task: a tile at the edge of a narrow block skips the rest's products
    bool live[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) live[i][j] = tk.r0 + wr + 16 * i < tk.M && tk.c0 + wc + 16 * j < tk.N;
    const int li = lane % 16, lk = lane / 16;
    d4_t acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = d4_t{0.0, 0.0, 0.0, 0.0};
    // the chunks of all segments in order; the global loads of the next
    // chunk are issued before the products of the current one
    constexpr int PER = TILE * kKC / NT;
    static_assert(PER * NT == TILE * kKC, "a chunk is PER values per thread and operand");
    int s = tk.s0, kb = 0;
    TSeg sg{};
    while (s < tk.s1) {
        sg = segs[s];
        if (sg.k0 < sg.k1) {
            kb = sg.k0;
            break;
        }
        ++s;
    }
    double ra[PER], rb[PER];
    int cta = 0, ctb = 0;
    auto fetch = [&]() {
        const double cf = coef[sg.cidx];
        const double* __restrict__ A = bufs.p[sg.a_buf] + sg.a_off;
        const double* __restrict__ B = bufs.p[sg.b_buf] + sg.b_off;
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            const int idx = threadIdx.x + p * NT;
            int r, k;
            if (sg.ta == 0) {
                r = idx / kKC;
                k = idx % kKC;
            } else {
                k = idx / TILE;
                r = idx % TILE;
            }
            const int gr = tk.r0 + r, gk = kb + k;
            double v = 0.0;
            if (gr < tk.M && gk < sg.k1)
                v = (sg.ta == 0) ? A[(long long)gr * sg.lda + gk] : A[(long long)gk * sg.lda + gr];
            ra[p] = cf * v;
        }
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            const int idx = threadIdx.x + p * NT;
            int c, k;
            if (sg.tb == 0) {
                k = idx / TILE;
                c = idx % TILE;
            } else {
                c = idx / kKC;
                k = idx % kKC;
            }
            const int gc = tk.c0 + c, gk = kb + k;
            double v = 0.0;
            if (gc < tk.N && gk < sg.k1)
                v = (sg.tb == 0) ? B[(long long)gk * sg.ldb + gc] : B[(long long)gc * sg.ldb + gk];
            rb[p] = v;
        }
        cta = sg.ta;
        ctb = sg.tb;
    };
    if (s < tk.s1) fetch();
    while (s < tk.s1) {
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            const int idx = threadIdx.x + p * NT;
            if (cta == 0) As[idx % kKC][idx / kKC] = ra[p];
            else As[idx / TILE][idx % TILE] = ra[p];
            if (ctb == 0) Bs[idx / TILE][idx % TILE] = rb[p];
            else Bs[idx % kKC][idx / kKC] = rb[p];
        }
        __syncthreads();
        kb += kKC;
        if (kb >= sg.k1) {
            ++s;
            while (s < tk.s1) {
                sg = segs[s];
                if (sg.k0 < sg.k1) {
                    kb = sg.k0;
                    break;
                }
                ++s;
            }
        }
        if (s < tk.s1) fetch();
#pragma unroll
        for (int ks = 0; ks < kKC; ks += 4) {
            const double a0 = As[ks + lk][wr + li], a1 = As[ks + lk][wr + 16 + li];
            const double b0 = Bs[ks + lk][wc + li], b1 = Bs[ks + lk][wc + 16 + li];
            if (live[0][0]) acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
            if (live[0][1]) acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
            if (live[1][0]) acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
            if (live[1][1]) acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
        }
        __syncthreads();
    }
    double* C = bufs.p[tk.c_buf] + tk.c_off;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = tk.r0 + wr + 16 * i + 4 * v + lk;
            if (r >= tk.M) continue;
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int c = tk.c0 + wc + 16 * j + li;
                if (c >= tk.N) continue;
                if (tk.mode == 0) {
                    C[(long long)r * tk.ldc + c] = acc[i][j][v];
                } else {
                    const int p = map[tk.pack_off + (long long)r * tk.N + c];
                    if (p >= 0) C[p] = acc[i][j][v];
                }
            }
        }
    }
}

// The same block products in split BF16 (three matrix-core products per
// step, FP32 accumulation).  Every operand value v (FP64, the A operand
// already times its segment coefficient) is split as v ~ hi + lo with
// hi = bf16(v) and lo = bf16(v - hi), round to nearest even, and
// A B ~ hi_A hi_B + hi_A lo_B + lo_A hi_B (the lo lo term is dropped): about
// 16 significant bits per operand, so products carry a relative error of
// order 1e-5.  K is staged in chunks of 16 as bf16 pairs, k contiguous per
// row of A and per column of B, so that a lane fetches its four k values of
// a v_mfma_f32_16x16x16_bf16 step with one 8-byte LDS read (lane l supplies
// A(l % 16, 4 (l / 16) + t) and B(4 (l / 16) + t, l % 16), t < 4, and holds
// D(4 (l / 16) + v, l % 16), v < 4).  The 16-deep steps keep a 64-thread
// work-group at 5 KB of LDS and 48 VGPRs, so a CU holds as many as it has
// wave slots (the 32-deep v_mfma_f32_16x16x32_bf16 with chunks of 32 needed
// 10 KB and 97 VGPRs and was 1.5x slower at the K = 12 ab-initio centre).
// The chunk loads are pipelined as in k_tgemm (1.4x faster in the 64-thread
// tile, 1.2-1.25x in the 256-thread tile at K = 16-24).  Tiles, wavefront
// layout and output addressing as in k_tgemm;
// values must lie in the FP32 range.
constexpr int kKC3 = 16;
constexpr int kKC3Pad = kKC3 + 4;  // bf16 per LDS row (8-byte aligned rows)
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef short s4_t __attribute__((ext_vector_type(4)));

__device__ inline unsigned short bf16_rne(float f) {
    unsigned int u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ inline void split_bf16(double v, unsigned short& hi, unsigned short& lo) {
    hi = bf16_rne(float(v));
    const double h = double(__uint_as_float((unsigned int)hi << 16));
    lo = bf16_rne(float(v - h));
}

template <int TILE>
__global__ __launch_bounds__((TILE / 4) * (TILE / 4)) void k_tgemm_bf3(const TTask* __restrict__ tasks,
                                                                      const TSeg* __restrict__ segs, BufSet bufs,
                                                                      const double* __restrict__ coef,
                                                                      const int* __restrict__ map) {
    constexpr int NT = (TILE / 4) * (TILE / 4), WPR = TILE / 32;
    static_assert(NT == 64 * WPR * WPR, "one wavefront per 32 x 32 quarter");
    __shared__ __align__(16) unsigned short Ah[TILE][kKC3Pad], Al[TILE][kKC3Pad];
    __shared__ __align__(16) unsigned short Bh[TILE][kKC3Pad], Bl[TILE][kKC3Pad];
    const TTask tk = tasks[blockIdx.x];
    const int lane = threadIdx.x % 64, wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
    const int wr = (wave / WPR) * 32, wc = (wave % WPR) * 32;
    // the 16 x 16 blocks of the wavefront's quarter that hold outputs of the
    // task: a tile at the edge of a narrow block skips the rest's products
    bool live[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) live[i][j] = tk.r0 + wr + 16 * i < tk.M && tk.c0 + wc + 16 * j < tk.N;
    const int li = lane % 16, lk = lane / 16;
    f4_t acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f4_t{0.f, 0.f, 0.f, 0.f};
    // as in k_tgemm: the chunks of all segments in order, each chunk's
    // global loads issued before the products of the previous one
    constexpr int PER = TILE * kKC3 / NT;
    static_assert(PER * NT == TILE * kKC3, "a chunk is PER values per thread and operand");
    int s = tk.s0, kb = 0;
    TSeg sg{};
    while (s < tk.s1) {
        sg = segs[s];
        if (sg.k0 < sg.k1) {
            kb = sg.k0;
            break;
        }
        ++s;
    }
    double ra[PER], rb[PER];
    int cta = 0, ctb = 0;
    auto fetch = [&]() {
        const double cf = coef[sg.cidx];
        const double* __restrict__ A = bufs.p[sg.a_buf] + sg.a_off;
        const double* __restrict__ B = bufs.p[sg.b_buf] + sg.b_off;
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            const int idx = threadIdx.x + p * NT;
            int r, k;
            if (sg.ta == 0) {
                r = idx / kKC3;
                k = idx % kKC3;
            } else {
                k = idx / TILE;
                r = idx % TILE;
            }
            const int gr = tk.r0 + r, gk = kb + k;
            double v = 0.0;
            if (gr < tk.M && gk < sg.k1)
                v = (sg.ta == 0) ? A[(long long)gr * sg.lda + gk] : A[(long long)gk * sg.lda + gr];
            ra[p] = cf * v;
        }
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            const int idx = threadIdx.x + p * NT;
            int c, k;
            if (sg.tb == 0) {
                k = idx / TILE;
                c = idx % TILE;
            } else {
                c = idx / kKC3;
                k = idx % kKC3;
            }
            const int gc = tk.c0 + c, gk = kb + k;
            double v = 0.0;
            if (gc < tk.N && gk < sg.k1)
                v = (sg.tb == 0) ? B[(long long)gk * sg.ldb + gc] : B[(long long)gc * sg.ldb + gk];
            rb[p] = v;
        }
        cta = sg.ta;
        ctb = sg.tb;
    };
    if (s < tk.s1) fetch();
    while (s < tk.s1) {
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            const int idx = threadIdx.x + p * NT;
            const int ar = cta == 0 ? idx / kKC3 : idx % TILE, ak = cta == 0 ? idx % kKC3 : idx / TILE;
            const int bc = ctb == 0 ? idx % TILE : idx / kKC3, bk = ctb == 0 ? idx / TILE : idx % kKC3;
            split_bf16(ra[p], Ah[ar][ak], Al[ar][ak]);
            split_bf16(rb[p], Bh[bc][bk], Bl[bc][bk]);
        }
        __syncthreads();
        kb += kKC3;
        if (kb >= sg.k1) {
            ++s;
            while (s < tk.s1) {
                sg = segs[s];
                if (sg.k0 < sg.k1) {
                    kb = sg.k0;
                    break;
                }
                ++s;
            }
        }
        if (s < tk.s1) fetch();
        s4_t ah[2], al[2], bh[2], bl[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            ah[i] = *reinterpret_cast<const s4_t*>(&Ah[wr + 16 * i + li][4 * lk]);
            al[i] = *reinterpret_cast<const s4_t*>(&Al[wr + 16 * i + li][4 * lk]);
            bh[i] = *reinterpret_cast<const s4_t*>(&Bh[wc + 16 * i + li][4 * lk]);
            bl[i] = *reinterpret_cast<const s4_t*>(&Bl[wc + 16 * i + li][4 * lk]);
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                if (!live[i][j]) continue;
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al[i], bh[j], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah[i], bl[j], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah[i], bh[j], acc[i][j], 0, 0, 0);
            }
        __syncthreads();
    }
    double* C = bufs.p[tk.c_buf] + tk.c_off;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = tk.r0 + wr + 16 * i + 4 * lk + v;
            if (r >= tk.M) continue;
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int c = tk.c0 + wc + 16 * j + li;
                if (c >= tk.N) continue;
                if (tk.mode == 0) {
                    C[(long long)r * tk.ldc + c] = double(acc[i][j][v]);
                } else {
                    const int p = map[tk.pack_off + (long long)r * tk.N + c];
                    if (p >= 0) C[p] = double(acc[i][j][v]);
                }
            }
        }
    }
}

__global__ __launch_bounds__(kThreads) void k_to_f32(const double* __restrict__ in, float* __restrict__ out,
                                                       long long n) {
    const long long e = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (e < n) out[e] = float(in[e]);
}

__global__ __launch_bounds__(kThreads) void k_gather(const int* __restrict__ map, const double* __restrict__ src,
                                                       double* __restrict__ dst, long long n) {
    const long long e = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (e >= n) return;
    const int p = map[e];
    dst[e] = p >= 0 ? src[p] : 0.0;
}

// sa += pa[g stride + e], sb += pb[g stride + e] for g = 0..G-1 in order,
// the loads of U slots issued together (wide sums: the tiled products leave
// G x tr_split slots, over a hundred)
template <int U>
__device__ inline void sum_slots(const double* __restrict__ pa, const double* __restrict__ pb, long long stride,
                                 int G, long long e, double& sa, double& sb) {
    int g = 0;
    for (; g + U <= G; g += U) {
        double a[U], b[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            a[u] = pa[(g + u) * stride + e];
            b[u] = pb[(g + u) * stride + e];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            sa += a[u];
            sb += b[u];
        }
    }
    for (; g < G; ++g) {
        sa += pa[g * stride + e];
        sb += pb[g * stride + e];
    }
}

__global__ __launch_bounds__(kThreads) void k_gsum2(const double* __restrict__ pa, const double* __restrict__ pb,
                                                      long long stride, int G, int n, double* __restrict__ outa,
                                                      double* __restrict__ outb) {
    const int e = blockIdx.x * kThreads + threadIdx.x;
    if (e >= n) return;
    double sa = 0.0, sb = 0.0;
    sum_slots<16>(pa, pb, stride, G, e, sa, sb);
    outa[e] = sa;
    outb[e] = sb;
}

// ---- grid-parallel Davidson passes ----------------------------------------
// A work-group owns kDavChunk consecutive elements.  The Ritz and CGS passes
// run 1024 threads per work-group: four groups of 256 threads split the
// subspace index, each thread loading all of its vectors in one batch, and
// their partial sums are added in LDS in a fixed order.

constexpr int kDavWide = 1024;
constexpr int kDavGroups = kDavWide / kDavChunk;  // 4
constexpr int kDavWaves = kDavWide / 64;          // 16
static_assert(kDavChunk == kThreads, "one element per thread of a group");
constexpr int kBatch = 8;

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// out[j] = sum over q < nchunk of part[q * stride + j], for j < m.  Wave w
// of NW adds the chunks q = w mod NW (ascending), then the NW wave sums are
// added in wave order: a fixed order, so the result is deterministic.
template <int NW>
__device__ inline void reduce_partials(const double* __restrict__ part, int nchunk, int stride, int m,
                                       double (*wred)[64], double* out) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int j0 = 0; j0 < m; j0 += 64) {
        const int j = j0 + lane;
        double acc = 0.0;
        if (j < m) {
            int q = wave;
            for (; q + 3 * NW < nchunk; q += 4 * NW) {
                const double p0 = part[(long long)q * stride + j];
                const double p1 = part[(long long)(q + NW) * stride + j];
                const double p2 = part[(long long)(q + 2 * NW) * stride + j];
                const double p3 = part[(long long)(q + 3 * NW) * stride + j];
                acc += p0;
                acc += p1;
                acc += p2;
                acc += p3;
            }
            for (; q < nchunk; q += NW) acc += part[(long long)q * stride + j];
        }
        wred[wave][lane] = acc;
        __syncthreads();
        if (threadIdx.x < 64 && j < m) {
            double r = 0.0;
#pragma unroll
            for (int w = 0; w < NW; ++w) r += wred[w][lane];
            out[j] = r;
        }
        __syncthreads();
    }
}

// out[j] = sum over the chunk of src_j[e] w[e] for j < m, src_j = base + j ld,
// with w staged in LDS (ws, kDavChunk values).  Wave w of NW takes
// j = w mod NW, four vectors per pass (16 loads in flight per lane).
template <int NW>
__device__ inline void chunk_dots(const double* __restrict__ base, long long ld, int m, int e0, int n,
                                  const double* ws, double* __restrict__ out) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nval = min(kDavChunk, n - e0);
    double wv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) wv[q] = ws[lane + 64 * q];
    for (int j = wave; j < m; j += 4 * NW) {
        double acc[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            acc[u] = 0.0;
            const int jj = j + NW * u;
            if (jj < m) {
                const double* __restrict__ src = base + (long long)jj * ld + e0;
                double v[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) v[q] = (lane + 64 * q < nval) ? src[lane + 64 * q] : 0.0;
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[u] = fma(v[q], wv[q], acc[u]);
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const double r = wave_sum(acc[u]);
            if (lane == 0 && j + NW * u < m) out[j + NW * u] = r;
        }
    }
}

// the subspace range [j0, j1) of thread group jg when m vectors are split
// over kDavGroups groups
__device__ inline void group_range(int m, int jg, int& j0, int& j1) {
    const int per = (m + kDavGroups - 1) / kDavGroups;
    j0 = min(m, jg * per);
    j1 = min(m, j0 + per);
}

__device__ inline void dav_ritz_body(const double* __restrict__ V, const double* __restrict__ HV,
                                                         const double* __restrict__ NV, long long ld, int m,
                                                         const double* __restrict__ aq,
                                                         const double* __restrict__ dh,
                                                         const double* __restrict__ dn, int n, double floor_,
                                                         double* __restrict__ x, double* __restrict__ t,
                                                         double* __restrict__ part_x, double* __restrict__ part_c, int chunk) {
    __shared__ double sa[kDavMaxVec + 1];
    __shared__ double red[3][kDavGroups][kDavChunk];
    __shared__ double ts[kDavChunk];
    __shared__ double wsum[4][3];
    for (int j = threadIdx.x; j <= m; j += kDavWide) sa[j] = aq[j];
    __syncthreads();
    const double theta = sa[m];
    const int el = threadIdx.x & (kDavChunk - 1), jg = threadIdx.x / kDavChunk;
    const int e0 = chunk * kDavChunk;
    const int e = e0 + el;
    {
        double xv = 0.0, hv = 0.0, nv = 0.0;
        if (e < n) {
            int j0, j1;
            group_range(m, jg, j0, j1);
            int j = j0;
            for (; j + kBatch <= j1; j += kBatch) {
                double v[kBatch], h[kBatch], q[kBatch];
#pragma unroll
                for (int u = 0; u < kBatch; ++u) {
                    const long long o = (long long)(j + u) * ld + e;
                    v[u] = V[o];
                    h[u] = HV[o];
                    q[u] = NV[o];
                }
#pragma unroll
                for (int u = 0; u < kBatch; ++u) {
                    xv = fma(sa[j + u], v[u], xv);
                    hv = fma(sa[j + u], h[u], hv);
                    nv = fma(sa[j + u], q[u], nv);
                }
            }
            for (; j < j1; ++j) {
                const long long o = (long long)j * ld + e;
                xv = fma(sa[j], V[o], xv);
                hv = fma(sa[j], HV[o], hv);
                nv = fma(sa[j], NV[o], nv);
            }
        }
        red[0][jg][el] = xv;
        red[1][jg][el] = hv;
        red[2][jg][el] = nv;
    }
    __syncthreads();
    if (jg == 0) {
        double tv = 0.0, xx = 0.0, uu = 0.0, xn = 0.0;
        if (e < n) {
            const double xv = (red[0][0][el] + red[0][1][el]) + (red[0][2][el] + red[0][3][el]);
            const double hv = (red[1][0][el] + red[1][1][el]) + (red[1][2][el] + red[1][3][el]);
            const double nv = (red[2][0][el] + red[2][1][el]) + (red[2][2][el] + red[2][3][el]);
            const double u = hv - theta * nv;
            double den = dh[e] - theta * dn[e];
            if (fabs(den) < floor_) den = (den < 0.0) ? -floor_ : floor_;
            tv = -u / den;
            x[e] = xv;
            t[e] = tv;
            xx = xv * xv;
            uu = u * u;
            xn = xv * nv;
        }
        ts[el] = tv;
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        xx = wave_sum(xx);
        uu = wave_sum(uu);
        xn = wave_sum(xn);
        if (lane == 0) {
            wsum[wave][0] = xx;
            wsum[wave][1] = uu;
            wsum[wave][2] = xn;
        }
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        const int c = threadIdx.x;
        part_x[3 * chunk + c] = (wsum[0][c] + wsum[1][c]) + (wsum[2][c] + wsum[3][c]);
    }
    chunk_dots<kDavWaves>(V, ld, m, e0, n, ts, part_c + (long long)chunk * m);
}

__device__ inline void dav_cgs_body(const double* __restrict__ V, long long ld, int m,
                                                        int m_dot, const double* __restrict__ part_in, int nchunk,
                                                        double* __restrict__ t, int n,
                                                        double* __restrict__ part_out, int mode, int chunk) {
    __shared__ double c[kDavMaxVec];
    __shared__ double wred[kDavWaves][64];
    __shared__ double red[kDavGroups][kDavChunk];
    __shared__ double ts[kDavChunk];
    __shared__ double wsum[4];
    reduce_partials<kDavWaves>(part_in, nchunk, m, m, wred, c);
    const int el = threadIdx.x & (kDavChunk - 1), jg = threadIdx.x / kDavChunk;
    const int e0 = chunk * kDavChunk;
    const int e = e0 + el;
    {
        double s = 0.0;
        if (e < n) {
            int j0, j1;
            group_range(m, jg, j0, j1);
            int j = j0;
            for (; j + kBatch <= j1; j += kBatch) {
                double w[kBatch];
#pragma unroll
                for (int u = 0; u < kBatch; ++u) w[u] = V[(long long)(j + u) * ld + e];
#pragma unroll
                for (int u = 0; u < kBatch; ++u) s = fma(c[j + u], w[u], s);
            }
            for (; j < j1; ++j) s = fma(c[j], V[(long long)j * ld + e], s);
        }
        red[jg][el] = s;
    }
    __syncthreads();
    double v = 0.0;
    if (jg == 0) {
        if (e < n) {
            v = t[e] - ((red[0][el] + red[1][el]) + (red[2][el] + red[3][el]));
            t[e] = v;
        }
        ts[el] = v;
    }
    if (mode == 0) {
        __syncthreads();
        chunk_dots<kDavWaves>(V, ld, m_dot, e0, n, ts, part_out + (long long)chunk * m_dot);
    } else {
        // norm partial (the first four waves hold the chunk)
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        double ss = wave_sum(v * v);
        if (jg == 0 && lane == 0) wsum[wave] = ss;
        __syncthreads();
        if (threadIdx.x == 0) part_out[chunk] = (wsum[0] + wsum[1]) + (wsum[2] + wsum[3]);
    }
}

__global__ __launch_bounds__(kThreads) void k_dav_normalize(const double* __restrict__ part, int nchunk,
                                                              const double* __restrict__ t,
                                                              double* __restrict__ vout, int n,
                                                              double* __restrict__ tnorm) {
    __shared__ double wred[4][64];
    __shared__ double tot[1];
    reduce_partials<4>(part, nchunk, 1, 1, wred, tot);
    const double nrm = sqrt(tot[0]);
    const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
    const int e = blockIdx.x * kDavChunk + threadIdx.x;
    if (e < n) vout[e] = t[e] * inv;
    if (blockIdx.x == 0 && threadIdx.x == 0) *tnorm = nrm;
}

// Gram rows of the new vector m.  With t != nullptr the new vector is
// t / |t| (|t|^2 = the sum of the nchunk partials pn, written to *tnorm): the
// work-groups with blockIdx.y == 0 store it as V_m, and H_eff t, N_eff t are
// scaled by 1/|t| the same way (H_eff is linear).  With ypart != nullptr
// H_eff t and N_eff t are the sums over the G quadrature partials (ascending
// g) and stored, scaled, in HV_m, NV_m; else (t must then be nullptr) they
// are read from HV_m, NV_m as they are.
__device__ inline void dav_gram_body(double* __restrict__ V, double* __restrict__ HV,
                                                         double* __restrict__ NV, long long ld, int m, int n,
                                                         const double* __restrict__ t,
                                                         const double* __restrict__ pn, int npn,
                                                         double* __restrict__ tnorm,
                                                         const double* __restrict__ ypart,
                                                         const double* __restrict__ nypart, long long gstride, int G,
                                                         double* __restrict__ part, int chunk, int grp) {
    __shared__ double vs[kDavChunk], hs[kDavChunk], ns[kDavChunk];
    __shared__ double wred[4][64];
    __shared__ double tot[1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nd = 4 * m + 2;
    const int e0 = chunk * kDavChunk;
    const int e = e0 + threadIdx.x;
    const int nval = min(kDavChunk, n - e0);
    double inv = 1.0;
    if (t) {
        reduce_partials<4>(pn, npn, 1, 1, wred, tot);
        const double nrm = sqrt(tot[0]);
        inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
        if (chunk == 0 && grp == 0 && threadIdx.x == 0) *tnorm = nrm;
    }
    double vm = 0.0, hm = 0.0, nm = 0.0;
    if (e < n) {
        const long long o = (long long)m * ld + e;
        vm = t ? t[e] * inv : V[o];
        if (ypart) {
            sum_slots<8>(ypart, nypart, gstride, G, e, hm, nm);
        } else {
            hm = HV[o];
            nm = NV[o];
        }
        hm *= inv;
        nm *= inv;
    }
    vs[threadIdx.x] = vm;
    hs[threadIdx.x] = hm;
    ns[threadIdx.x] = nm;
    __syncthreads();
    // every work-group has read what it needs of HV_m, NV_m (only its own
    // chunk, by its own threads) before the y == 0 groups overwrite them
    if (grp == 0 && e < n && ypart) {
        const long long o = (long long)m * ld + e;
        if (t) V[o] = vm;
        HV[o] = hm;
        NV[o] = nm;
    }
    double* out = part + (long long)chunk * nd;
    const int d0 = grp * kGramGroup;
    const int d1 = min(nd, d0 + kGramGroup);
    // d <= m: V_d.HV_m; then V_j.NV_m (j <= m); HV_j.V_m (j < m); NV_j.V_m (j < m).
    // V_m itself is taken from LDS (it may be being stored right now).
    for (int d = d0 + wave; d < d1; d += 16) {
        double acc[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            acc[u] = 0.0;
            const int dd = d + 4 * u;
            if (dd < d1) {
                int row;
                const double* __restrict__ base;
                const double* w;
                if (dd <= m) {
                    row = dd;
                    base = V;
                    w = hs;
                } else if (dd <= 2 * m + 1) {
                    row = dd - m - 1;
                    base = V;
                    w = ns;
                } else if (dd <= 3 * m + 1) {
                    row = dd - 2 * m - 2;
                    base = HV;
                    w = vs;
                } else {
                    row = dd - 3 * m - 2;
                    base = NV;
                    w = vs;
                }
                if (row == m) {  // V_m . (HV_m or NV_m), both in LDS
#pragma unroll
                    for (int q = 0; q < 4; ++q) acc[u] = fma(vs[lane + 64 * q], w[lane + 64 * q], acc[u]);
                } else {
                    const double* __restrict__ src = base + (long long)row * ld + e0;
                    double v[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) v[q] = (lane + 64 * q < nval) ? src[lane + 64 * q] : 0.0;
#pragma unroll
                    for (int q = 0; q < 4; ++q) acc[u] = fma(v[q], w[lane + 64 * q], acc[u]);
                }
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const double r = wave_sum(acc[u]);
            if (lane == 0 && d + 4 * u < d1) out[d + 4 * u] = r;
        }
    }
}

__global__ __launch_bounds__(kDavWide) void k_dav_ritz(const double* __restrict__ V, const double* __restrict__ HV,
                                                         const double* __restrict__ NV, long long ld, int m,
                                                         const double* __restrict__ aq,
                                                         const double* __restrict__ dh,
                                                         const double* __restrict__ dn, int n, double floor_,
                                                         double* __restrict__ x, double* __restrict__ t,
                                                         double* __restrict__ part_x, double* __restrict__ part_c) {
    dav_ritz_body(V, HV, NV, ld, m, aq, dh, dn, n, floor_, x, t, part_x, part_c, blockIdx.x);
}

__global__ __launch_bounds__(kDavWide) void k_dav_cgs(const double* __restrict__ V, long long ld, int m,
                                                        int m_dot, const double* __restrict__ part_in, int nchunk,
                                                        double* __restrict__ t, int n,
                                                        double* __restrict__ part_out, int mode) {
    dav_cgs_body(V, ld, m, m_dot, part_in, nchunk, t, n, part_out, mode, blockIdx.x);
}

__global__ __launch_bounds__(kThreads) void k_dav_gram(double* __restrict__ V, double* __restrict__ HV,
                                                         double* __restrict__ NV, long long ld, int m, int n,
                                                         const double* __restrict__ t,
                                                         const double* __restrict__ pn, int npn,
                                                         double* __restrict__ tnorm,
                                                         const double* __restrict__ ypart,
                                                         const double* __restrict__ nypart, long long gstride, int G,
                                                         double* __restrict__ part) {
    dav_gram_body(V, HV, NV, ld, m, n, t, pn, npn, tnorm, ypart, nypart, gstride, G, part, blockIdx.x, blockIdx.y);
}

// batched passes: blockIdx.y (blockIdx.z for the Gram pass) is the instance;
// work-groups past an instance's chunk or dot count, or of an inactive
// instance, exit at once
__global__ __launch_bounds__(kDavWide) void k_bdav_ritz(const DavInst* __restrict__ insts) {
    const DavInst I = insts[blockIdx.y];
    if (!I.active || (int)blockIdx.x >= dav_chunks(I.n)) return;
    dav_ritz_body(I.V, I.HV, I.NV, I.ld, I.mr, I.aq, I.dh, I.dn, I.n, I.floor_, I.x, I.t, I.part_x, I.pc1, blockIdx.x);
}

__global__ __launch_bounds__(kDavWide) void k_bdav_cgs(const DavInst* __restrict__ insts, int mode) {
    const DavInst I = insts[blockIdx.y];
    if (!I.active || !I.ext || (int)blockIdx.x >= dav_chunks(I.n)) return;
    const int nch = dav_chunks(I.n);
    if (mode == 0) dav_cgs_body(I.V, I.ld, I.m, I.m, I.pc1, nch, I.t, I.n, I.pc2, 0, blockIdx.x);
    else if (mode == 1) dav_cgs_body(I.V, I.ld, I.m, 0, I.pc2, nch, I.t, I.n, I.pn, 1, blockIdx.x);
    else if (I.restart) dav_cgs_body(I.V, I.ld, 0, I.m, I.pc2, nch, I.t, I.n, I.pc1, 0, blockIdx.x);
}

__global__ __launch_bounds__(kThreads) void k_bdav_gram(const DavInst* __restrict__ insts) {
    const DavInst I = insts[blockIdx.z];
    const int nd = 4 * I.m + 2;
    if (!I.active || !I.ext || (int)blockIdx.x >= dav_chunks(I.n) || (int)blockIdx.y * kGramGroup >= nd) return;
    dav_gram_body(I.V, I.HV, I.NV, I.ld, I.m, I.n, I.from_t ? I.t : nullptr, I.pn, dav_chunks(I.n), I.tnorm,
                  I.ypart, I.nypart, I.gstride, I.G, I.pg, blockIdx.x, blockIdx.y);
}

inline int nblk(int n) { return (n + kThreads - 1) / kThreads; }

}  // namespace

void tgemm_bf3(hipStream_t s, const TTask* tasks, int ntasks, const TSeg* segs, BufSet bufs, const double* coef,
               const int* map, int tile) {
    if (ntasks <= 0) return;
    if (tile == 32)
        hipLaunchKernelGGL(k_tgemm_bf3<32>, dim3(ntasks), dim3(64), 0, s, tasks, segs, bufs, coef, map);
    else
        hipLaunchKernelGGL(k_tgemm_bf3<64>, dim3(ntasks), dim3(256), 0, s, tasks, segs, bufs, coef, map);
}

void tgemm(hipStream_t s, const TTask* tasks, int ntasks, const TSeg* segs, BufSet bufs, const double* coef,
           const int* map, int tile) {
    if (ntasks <= 0) return;
    if (tile == 32)
        hipLaunchKernelGGL(k_tgemm<32>, dim3(ntasks), dim3(64), 0, s, tasks, segs, bufs, coef, map);
    else
        hipLaunchKernelGGL(k_tgemm<64>, dim3(ntasks), dim3(256), 0, s, tasks, segs, bufs, coef, map);
}
void to_f32(hipStream_t s, const double* in, float* out, long long n) {
    if (n > 0)
        hipLaunchKernelGGL(k_to_f32, dim3((unsigned)((n + kThreads - 1) / kThreads)), dim3(kThreads), 0, s, in, out, n);
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
               int G, double* out, int nsplit, double* part, long long ntot) {
    if (nb <= 0) return;
    if (nsplit < 1 || (nsplit > 1 && !part)) nsplit = 1;
    hipLaunchKernelGGL(k_diag, dim3(nb, nsplit), dim3(kThreads), 0, s, blks, terms, lenv, lsize, renv, rsize,
                       coef, ncoef, G, out, part, ntot);
    if (nsplit > 1)
        hipLaunchKernelGGL(k_diag_sum, dim3((unsigned)((ntot + kThreads - 1) / kThreads)), dim3(kThreads), 0, s,
                           part, nsplit, ntot, out);
}
void qr_sectors(hipStream_t s, const QrTask* tasks, int ntasks, const QrPiece* pieces, double* site,
                double* scratch, double* rout, int lds_doubles) {
    if (ntasks <= 0) return;
    if (lds_doubles > 0 && lds_doubles <= kQrLdsMax)
        hipLaunchKernelGGL(k_qr_lds, dim3(ntasks), dim3(kThreads), size_t(lds_doubles) * sizeof(double), s, tasks,
                           pieces, site, rout);
    else
        hipLaunchKernelGGL(k_qr, dim3(ntasks), dim3(kThreads), 0, s, tasks, pieces, site, scratch, rout);
}
void fill(hipStream_t s, double* p, long long n, double value) {
    if (n <= 0) return;
    const long long nb = std::min<long long>((n + kThreads - 1) / kThreads, 4096);
    hipLaunchKernelGGL(k_fill, dim3(unsigned(nb)), dim3(kThreads), 0, s, p, n, value);
}
void normalize(hipStream_t s, const double* in, double* out, int n, double* norm_out) {
    hipLaunchKernelGGL(k_normalize, dim3(1), dim3(1024), 0, s, in, out, n, norm_out);
}
void multidot(hipStream_t s, const double* A, long long ld, int m, const double* u, int n, double* out) {
    if (m > 0) hipLaunchKernelGGL(k_multidot, dim3(m), dim3(kThreads), 0, s, A, ld, u, n, out);
}
void basis_rotate(hipStream_t s, const double* A, long long ld, int m, const double* Q, int keep,
                  double* out, int n) {
    hipLaunchKernelGGL(k_basis_rotate, dim3(nblk(n)), dim3(kThreads), 0, s, A, ld, m, Q, keep, out, n);
}
void dav_ritz(hipStream_t s, const double* V, const double* HV, const double* NV, long long ld, int m,
              const double* aq, const double* dh, const double* dn, int n, double floor_, double* x, double* t,
              double* part_x, double* part_c) {
    hipLaunchKernelGGL(k_dav_ritz, dim3(dav_chunks(n)), dim3(kDavWide), 0, s, V, HV, NV, ld, m, aq, dh, dn, n, floor_,
                       x, t, part_x, part_c);
}
void dav_cgs(hipStream_t s, const double* V, long long ld, int m_sub, int m_dot, const double* part_in,
             int nchunk, double* t, int n, double* part_out, int mode) {
    hipLaunchKernelGGL(k_dav_cgs, dim3(dav_chunks(n)), dim3(kDavWide), 0, s, V, ld, m_sub, m_dot, part_in, nchunk, t,
                       n, part_out, mode);
}
void dav_normalize(hipStream_t s, const double* part, int nchunk, const double* t, double* vout, int n,
                   double* tnorm) {
    hipLaunchKernelGGL(k_dav_normalize, dim3(dav_chunks(n)), dim3(kThreads), 0, s, part, nchunk, t, vout, n, tnorm);
}
void dav_gram(hipStream_t s, double* V, double* HV, double* NV, long long ld, int m, int n, const double* t,
              const double* pn, int npn, double* tnorm, const double* ypart, const double* nypart, long long gstride,
              int G, double* part) {
    const int nd = 4 * m + 2;
    hipLaunchKernelGGL(k_dav_gram, dim3(dav_chunks(n), (nd + kGramGroup - 1) / kGramGroup), dim3(kThreads), 0, s, V, HV,
                       NV, ld, m, n, t, pn, npn, tnorm, ypart, nypart, gstride, G, part);
}

void bdav_ritz(hipStream_t s, const DavInst* insts, int ninst, int max_n) {
    if (ninst > 0) hipLaunchKernelGGL(k_bdav_ritz, dim3(dav_chunks(max_n), ninst), dim3(kDavWide), 0, s, insts);
}
void bdav_cgs(hipStream_t s, const DavInst* insts, int ninst, int max_n, int mode) {
    if (ninst > 0) hipLaunchKernelGGL(k_bdav_cgs, dim3(dav_chunks(max_n), ninst), dim3(kDavWide), 0, s, insts, mode);
}
void bdav_gram(hipStream_t s, const DavInst* insts, int ninst, int max_n, int max_m) {
    const int nd = 4 * max_m + 2;
    if (ninst > 0)
        hipLaunchKernelGGL(k_bdav_gram, dim3(dav_chunks(max_n), (nd + kGramGroup - 1) / kGramGroup, ninst),
                           dim3(kThreads), 0, s, insts);
}

}  // namespace spk
