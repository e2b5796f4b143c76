// Device-resident Davidson iteration for the local problem of Eq.
// [geproblem] (Sec. 2.3): the FP64 subspace solve of the projected pencil
// in one work-group per state and the bookkeeping between the vector
// passes, so that an iteration needs no decision on the host and a whole
// iteration of many states can be replayed from one HIP graph.
//
// The arithmetic is that of the host solver: the projected matrices are
// symmetrised; when N - drop U I (U the Gershgorin bound of N) is positive
// definite no eigenvalue of N falls below drop lambda_max and the pencil is
// reduced with the Cholesky factor of N (lowest pair by Householder
// tridiagonalisation, Sturm bisection and inverse iteration); otherwise, and
// at a restart, N and the reduced matrix are diagonalised (cyclic Jacobi)
// and the eigenvectors of N below drop lambda_max are dropped (canonical
// orthogonalisation).  A restart keeps the lowest Ritz vectors,
// orthonormalised by modified Gram-Schmidt.  Some reductions run in another
// order than on the host, so the two agree to rounding.
#include "kernels.h"

#include <vector>

namespace spk {

namespace {

constexpr int kST = 256;  // threads of a subspace-solve work-group
constexpr int kSpErrNorm = -2;  // the projected metric vanishes (SP_ENORM)
constexpr int kSpErrNan = -6;   // non-finite value (SP_ENAN)

// fixed-order tree reduction over the work-group (kST threads)
__device__ inline double wg_sum(double v, double* red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = kST / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}
__device__ inline double wg_max(double v, double* red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = kST / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// sum over q < nch of part[q * stride + idx], ascending q (the host's
// order); eight loads in flight at a time
__device__ inline double chunk_total(const double* part, int nch, int stride, int idx) {
    double acc = 0.0;
    int q = 0;
    for (; q + 8 <= nch; q += 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = part[(long long)(q + u) * stride + idx];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += v[u];
    }
    for (; q < nch; ++q) acc += part[(long long)q * stride + idx];
    return acc;
}

// sum over the lanes of wave 0 (callers: threads of wave 0 only)
__device__ inline double wave0_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// LDS of one solve, m <= kDevSubMax: seven m x m matrices, eight m-vectors
// and 512 doubles of scalars and scratch (misc: [0, 64) scalars of the
// steps, [64, 256) the rotations of a Jacobi round, [256, 512) the band
// scratch of inverse iteration); the reduction buffer is static
struct Work {
    double *H, *N, *L, *L2, *W, *B, *Z;
    double *v0, *v1, *v2, *v3, *v4, *v5, *v6, *v7;
    double* misc;
};
__device__ inline Work carve(double* base, int m) {
    Work w;
    const int mm = m * m;
    w.H = base;
    w.N = w.H + mm;
    w.L = w.N + mm;
    w.L2 = w.L + mm;
    w.W = w.L2 + mm;
    w.B = w.W + mm;
    w.Z = w.B + mm;
    w.v0 = w.Z + mm;
    w.v1 = w.v0 + m;
    w.v2 = w.v1 + m;
    w.v3 = w.v2 + m;
    w.v4 = w.v3 + m;
    w.v5 = w.v4 + m;
    w.v6 = w.v5 + m;
    w.v7 = w.v6 + m;
    w.misc = w.v7 + m;
    return w;
}

// Cholesky factors of N - shift I (L2) and of N (L), lower, stored
// column-major (entry (i, k) at k m + i, so that the dot products of the rows
// read consecutive LDS words), in one pass over the columns; false if a
// pivot of either is not positive
__device__ bool chol2(int m, const double* N, double shift, double* L, double* L2, double* flag) {
    const int tid = threadIdx.x;
    for (int e = tid; e < m * m; e += kST) L[e] = L2[e] = 0.0;
    if (tid == 0) flag[0] = 1.0;
    __syncthreads();
    for (int j = 0; j < m; ++j) {
        if (tid < 64) {
            const double a = (tid < j) ? L2[tid * m + j] : 0.0;
            const double b = (tid < j) ? L[tid * m + j] : 0.0;
            const double s1 = wave0_sum(a * a), s0 = wave0_sum(b * b);
            if (tid == 0) {
                const double d1 = N[j * m + j] - shift - s1, d0 = N[j * m + j] - s0;
                if (!(d1 > 0.0) || !(d0 > 0.0)) {
                    flag[0] = 0.0;
                } else {
                    L2[j * m + j] = sqrt(d1);
                    L[j * m + j] = sqrt(d0);
                }
            }
        }
        __syncthreads();
        if (flag[0] == 0.0) return false;
        const double ljj = L[j * m + j], l2jj = L2[j * m + j];
        for (int i = j + 1 + tid; i < m; i += kST) {
            double s0 = N[i * m + j], s1 = 0.0, t0 = N[i * m + j], t1 = 0.0;
            int k = 0;
            for (; k + 2 <= j; k += 2) {
                s0 -= L[k * m + i] * L[k * m + j];
                s1 -= L[(k + 1) * m + i] * L[(k + 1) * m + j];
                t0 -= L2[k * m + i] * L2[k * m + j];
                t1 -= L2[(k + 1) * m + i] * L2[(k + 1) * m + j];
            }
            for (; k < j; ++k) {
                s0 -= L[k * m + i] * L[k * m + j];
                t0 -= L2[k * m + i] * L2[k * m + j];
            }
            L[j * m + i] = (s0 + s1) / ljj;
            L2[j * m + i] = (t0 + t1) / l2jj;
        }
        __syncthreads();
    }
    return true;
}

// out = L^-1 in (L column-major as from chol2), column by column, one
// thread per column of `in` (reads of `in` and `out` are consecutive across
// threads, L entries are the same for all)
__device__ void tri_solve(int m, const double* L, const double* in, double* out) {
    const int c = threadIdx.x;
    if (c < m) {
        for (int i = 0; i < m; ++i) {
            double acc = in[i * m + c];
            for (int k = 0; k < i; ++k) acc -= L[k * m + i] * out[k * m + c];
            out[i * m + c] = acc * (1.0 / L[i * m + i]);
        }
    }
    __syncthreads();
}

__device__ void transpose(int m, const double* in, double* out) {
    for (int e = threadIdx.x; e < m * m; e += kST) {
        const int r = e / m, c = e - r * m;
        out[c * m + r] = in[e];
    }
    __syncthreads();
}

__device__ void symmetrise(int m, double* B) {
    for (int e = threadIdx.x; e < m * m; e += kST) {
        const int r = e / m, c = e - r * m;
        if (c < r) B[r * m + c] = B[c * m + r] = 0.5 * (B[r * m + c] + B[c * m + r]);
    }
    __syncthreads();
}

// Householder reduction of the symmetric A (m x m, destroyed) to tridiagonal
// (d, e); the vectors of the steps are kept in hv (row k), their factors in
// beta.  misc[0..3] are scratch scalars.
__device__ void tridiagonalise(int m, double* A, double* hv, double* beta, double* d, double* e, double* p,
                               double* w, double* misc) {
    const int tid = threadIdx.x;
    for (int k = tid; k < m; k += kST) beta[k] = 0.0;
    __syncthreads();
    for (int k = 0; k + 2 < m; ++k) {
        const int len = m - k - 1;
        double* v = hv + k * m;
        const double vt = (tid < len) ? A[k * m + k + 1 + tid] : 0.0;  // row k = column k (symmetric)
        if (tid < len) v[tid] = vt;
        double ss = 0.0;
        if (tid < 64) ss = wave0_sum(vt * vt);
        __syncthreads();
        if (tid == 0) {
            const double nrm = sqrt(ss);
            misc[0] = 0.0;  // skip
            if (nrm == 0.0) {
                misc[0] = 1.0;
            } else {
                const double x0 = v[0];
                const double alpha = (x0 >= 0.0) ? -nrm : nrm;
                v[0] = x0 - alpha;
                const double vv = ss - x0 * x0 + v[0] * v[0];
                if (vv == 0.0) {
                    misc[0] = 1.0;
                } else {
                    beta[k] = 2.0 / vv;
                    misc[1] = alpha;
                }
            }
        }
        __syncthreads();
        if (misc[0] != 0.0) continue;
        const double bk = beta[k];
        double pt = 0.0;
        if (tid < len) {
            // row (k+1+tid) of the trailing block read as its column
            const double* col = A + (k + 1) * m + k + 1 + tid;
            double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
            int j = 0;
            for (; j + 4 <= len; j += 4) {
                s0 += col[j * m] * v[j];
                s1 += col[(j + 1) * m] * v[j + 1];
                s2 += col[(j + 2) * m] * v[j + 2];
                s3 += col[(j + 3) * m] * v[j + 3];
            }
            for (; j < len; ++j) s0 += col[j * m] * v[j];
            pt = bk * ((s0 + s1) + (s2 + s3));
            p[tid] = pt;
        }
        if (tid < 64) {
            const double vp = wave0_sum((tid < len) ? v[tid] * pt : 0.0);
            if (tid == 0) misc[2] = 0.5 * bk * vp;
        }
        __syncthreads();
        const double K = misc[2];
        if (tid < len) w[tid] = p[tid] - K * v[tid];
        __syncthreads();
        for (int q = tid; q < len * len; q += kST) {
            const int i = q / len, j = q - i * len;
            A[(k + 1 + i) * m + k + 1 + j] -= v[i] * w[j] + w[i] * v[j];
        }
        if (tid < len) A[(k + 1 + tid) * m + k] = A[k * m + k + 1 + tid] = (tid == 0) ? misc[1] : 0.0;
        __syncthreads();
    }
    for (int i = tid; i < m; i += kST) {
        d[i] = A[i * m + i];
        e[i] = (i + 1 < m) ? A[(i + 1) * m + i] : 0.0;
    }
    __syncthreads();
}

__device__ int sturm_count(int n, const double* d, const double* e, double x) {
    int cnt = 0;
    double q = d[0] - x;
    if (q < 0.0) ++cnt;
    for (int i = 1; i < n; ++i) {
        const double qq = (q == 0.0) ? 1e-300 : q;
        q = d[i] - x - e[i - 1] * e[i - 1] / qq;
        if (q < 0.0) ++cnt;
    }
    return cnt;
}

// solve (T - shift) z = z in place (elimination with partial pivoting on the
// band) and normalise z; one thread; scratch of 5 n doubles
__device__ void tridiag_inverse_step(int n, const double* d, const double* e, double shift, double* z,
                                     double* sc) {
    double* dd = sc;
    double* du = sc + n;
    double* du2 = sc + 2 * n;
    double* dl = sc + 3 * n;
    double* swp = sc + 4 * n;
    for (int i = 0; i < n; ++i) {
        dd[i] = d[i] - shift;
        du[i] = du2[i] = dl[i] = 0.0;
        swp[i] = 0.0;
    }
    for (int i = 0; i + 1 < n; ++i) du[i] = dl[i] = e[i];
    for (int i = 0; i + 1 < n; ++i) {
        if (fabs(dd[i]) >= fabs(dl[i])) {
            const double f = (dd[i] != 0.0) ? dl[i] / dd[i] : 0.0;
            dl[i] = f;
            dd[i + 1] -= f * du[i];
        } else {
            swp[i] = 1.0;
            const double f = dd[i] / dl[i];
            dd[i] = dl[i];
            dl[i] = f;
            const double t = du[i];
            du[i] = dd[i + 1];
            dd[i + 1] = t - f * dd[i + 1];
            if (i + 2 < n) {
                du2[i] = du[i + 1];
                du[i + 1] = -f * du[i + 1];
            }
        }
    }
    for (int i = 0; i < n; ++i)
        if (dd[i] == 0.0) dd[i] = 1e-300;
    for (int i = 0; i + 1 < n; ++i) {
        if (swp[i] == 0.0) {
            z[i + 1] -= dl[i] * z[i];
        } else {
            const double t = z[i];
            z[i] = z[i + 1];
            z[i + 1] = t - dl[i] * z[i];
        }
    }
    z[n - 1] /= dd[n - 1];
    if (n > 1) z[n - 2] = (z[n - 2] - du[n - 2] * z[n - 1]) / dd[n - 2];
    for (int i = n - 3; i >= 0; --i) z[i] = (z[i] - du[i] * z[i + 1] - du2[i] * z[i + 2]) / dd[i];
    double nr = 0.0;
    for (int i = 0; i < n; ++i) nr += z[i] * z[i];
    nr = sqrt(nr);
    for (int i = 0; i < n; ++i) z[i] /= nr;
}

// lowest eigenpair of the tridiagonal (d, e): multisection with Sturm counts
// (kST points per round) narrows [lo, hi] around the lowest eigenvalue to
// 1e-7 of the Gershgorin spread with count(lo) = 0, inverse iteration
// shifted to lo gives the vector, its Rayleigh quotient the value (written
// to misc[0]).  sc: 5 n doubles of scratch; flags: kST doubles.
__device__ void tridiag_lowest(int n, const double* d, const double* e, double* z, double* sc, double* flags,
                               double* misc) {
    const int tid = threadIdx.x;
    if (n == 1) {
        if (tid == 0) {
            misc[0] = d[0];
            z[0] = 1.0;
        }
        __syncthreads();
        return;
    }
    if (tid == 0) {
        double lo = d[0], hi = d[0];
        for (int i = 0; i < n; ++i) {
            const double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < n ? fabs(e[i]) : 0.0);
            lo = fmin(lo, d[i] - r);
            hi = fmax(hi, d[i] + r);
        }
        const double spread = fmax(hi - lo, 1e-300);
        misc[1] = lo - 1e-3 * spread;
        misc[2] = hi + 1e-3 * spread;
        misc[3] = spread;
    }
    __syncthreads();
    for (int round = 0; round < 12; ++round) {
        const double lo = misc[1], hi = misc[2];
        if (!(hi - lo > 1e-7 * misc[3])) break;
        const double x = lo + (hi - lo) * double(tid + 1) / double(kST + 1);
        flags[tid] = (sturm_count(n, d, e, x) >= 1) ? double(tid) : double(kST);
        __syncthreads();
        for (int s = kST / 2; s > 0; s >>= 1) {
            if (tid < s) flags[tid] = fmin(flags[tid], flags[tid + s]);
            __syncthreads();
        }
        if (tid == 0) {
            const int t = int(flags[0]);
            if (t < kST) {
                misc[2] = lo + (hi - lo) * double(t + 1) / double(kST + 1);
                if (t > 0) misc[1] = lo + (hi - lo) * double(t) / double(kST + 1);
            } else {
                misc[1] = lo + (hi - lo) * double(kST) / double(kST + 1);
            }
        }
        __syncthreads();
    }
    if (tid == 0) {
        const double lo = misc[1];
        for (int i = 0; i < n; ++i) z[i] = 1.0 / sqrt(double(n)) * (1.0 + 0.01 * i);
        for (int it = 0; it < 3; ++it) tridiag_inverse_step(n, d, e, lo, z, sc);
        double rq = 0.0;
        for (int i = 0; i < n; ++i) {
            double tz = d[i] * z[i];
            if (i > 0) tz += e[i - 1] * z[i - 1];
            if (i + 1 < n) tz += e[i] * z[i + 1];
            rq += z[i] * tz;
        }
        misc[0] = rq;
    }
    __syncthreads();
}

// z <- Q z with Q = H_0 ... H_{m-3} of tridiagonalise
__device__ void apply_q(int m, const double* hv, const double* beta, double* z, double* misc) {
    const int tid = threadIdx.x;
    for (int k = m - 3; k >= 0; --k) {
        if (beta[k] == 0.0) continue;
        const int len = m - k - 1;
        const double* v = hv + k * m;
        if (tid < 64) {
            const double t = wave0_sum((tid < len) ? v[tid] * z[k + 1 + tid] : 0.0);
            if (tid == 0) misc[0] = t;
        }
        __syncthreads();
        const double t = misc[0];
        if (tid < len) z[k + 1 + tid] -= beta[k] * v[tid] * t;
        __syncthreads();
    }
}

// cyclic Jacobi on the symmetric A (m x m): on return the diagonal of A
// holds the eigenvalues and the columns of V the eigenvectors (unsorted).
// Rounds of m/2 disjoint rotations (round-robin pairing); rot: 4 kST doubles.
__device__ void jacobi(int m, double* A, double* V, double* rot, double* red) {
    const int tid = threadIdx.x;
    for (int e = tid; e < m * m; e += kST) V[e] = (e / m == e % m) ? 1.0 : 0.0;
    __syncthreads();
    const int mp = m + (m & 1), half = mp / 2;
    for (int sweep = 0; sweep < 40; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int e = tid; e < m * m; e += kST) {
            const double a = A[e];
            tot += a * a;
            if (e / m != e % m) off += a * a;
        }
        off = wg_sum(off, red);
        tot = wg_sum(tot, red);
        if (!(off > 1e-30 * tot)) break;
        for (int r = 0; r + 1 < mp; ++r) {
            if (tid < half) {
                const int a = (r + tid) % (mp - 1);
                const int b = (tid == 0) ? mp - 1 : (r + mp - 1 - tid) % (mp - 1);
                const int p = min(a, b), q = max(a, b);
                double c = 1.0, s = 0.0;
                if (q < m) {
                    const double apq = A[p * m + q];
                    if (apq != 0.0) {
                        const double th = (A[q * m + q] - A[p * m + p]) / (2.0 * apq);
                        const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                        c = 1.0 / sqrt(t * t + 1.0);
                        s = t * c;
                    }
                }
                rot[4 * tid] = p;
                rot[4 * tid + 1] = q;
                rot[4 * tid + 2] = c;
                rot[4 * tid + 3] = s;
            }
            __syncthreads();
            for (int e = tid; e < half * m; e += kST) {  // rows p, q
                const int sl = e / m, j = e - sl * m;
                const int p = int(rot[4 * sl]), q = int(rot[4 * sl + 1]);
                if (q >= m) continue;
                const double c = rot[4 * sl + 2], s = rot[4 * sl + 3];
                const double a0 = A[p * m + j], a1 = A[q * m + j];
                A[p * m + j] = c * a0 - s * a1;
                A[q * m + j] = s * a0 + c * a1;
            }
            __syncthreads();
            for (int e = tid; e < half * m; e += kST) {  // columns p, q of A and V
                const int i = e / half, sl = e - i * half;
                const int p = int(rot[4 * sl]), q = int(rot[4 * sl + 1]);
                if (q >= m) continue;
                const double c = rot[4 * sl + 2], s = rot[4 * sl + 3];
                const double a0 = A[i * m + p], a1 = A[i * m + q];
                A[i * m + p] = c * a0 - s * a1;
                A[i * m + q] = s * a0 + c * a1;
                const double v0 = V[i * m + p], v1 = V[i * m + q];
                V[i * m + p] = c * v0 - s * v1;
                V[i * m + q] = s * v0 + c * v1;
            }
            __syncthreads();
        }
    }
}

// ascending order of the diagonal of A: ord[r] = index of the r-th smallest
__device__ void sort_diag(int m, const double* A, double* ev, double* ord) {
    const int tid = threadIdx.x;
    if (tid < m) {
        const double x = A[tid * m + tid];
        int r = 0;
        for (int j = 0; j < m; ++j) {
            const double y = A[j * m + j];
            if (y < x || (y == x && j < tid)) ++r;
        }
        ev[r] = x;
        ord[r] = double(tid);
    }
    __syncthreads();
}

// The subspace solve of one state, every thread of the work-group: H, N
// (m x m, symmetrised) in LDS; on return misc[0] = theta, misc[1] = rank
// (0: the metric vanishes), a (m) the coefficients with a^T N a = 1; with
// need_all the m x rank Ritz coefficient vectors (ascending Ritz values)
// are in Xc (= w.W).
__device__ void solve_pencil(int m, Work& w, double drop, bool need_all, double* red) {
    const int tid = threadIdx.x;
    double* misc = w.misc;
    // fast path: no metric eigenvalue can be dropped, Cholesky reduction
    if (!need_all) {
        double U = 0.0;
        if (tid < m) {
            for (int j = 0; j < m; ++j) U += fabs(w.N[tid * m + j]);
        }
        U = wg_max(U, red);
        if (U > 1e-12 && chol2(m, w.N, drop * U, w.L, w.L2, misc + 8)) {
            tri_solve(m, w.L, w.H, w.W);   // W = L^-1 H
            transpose(m, w.W, w.L2);       // W^T (the shifted factor is no longer needed)
            tri_solve(m, w.L, w.L2, w.B);  // B = L^-1 W^T
            symmetrise(m, w.B);
            // lowest pair of B: tridiagonal form (vectors in Z), bisection,
            // inverse iteration, back-transformation
            tridiagonalise(m, w.B, w.Z, w.v0, w.v1, w.v2, w.v3, w.v4, misc + 16);
            tridiag_lowest(m, w.v1, w.v2, w.v5, misc + 256, red, misc + 24);
            apply_q(m, w.Z, w.v0, w.v5, misc + 32);
            if (tid == 0) {
                // a = L^-T c0
                for (int i = m - 1; i >= 0; --i) {
                    double v = w.v5[i];
                    for (int k = i + 1; k < m; ++k) v -= w.L[i * m + k] * w.v6[k];  // L(k, i), column-major
                    w.v6[i] = v / w.L[i * m + i];
                }
                misc[0] = misc[24];
                misc[1] = m;
            }
            __syncthreads();
            return;
        }
    }
    // canonical orthogonalisation through the eigenvectors of N
    for (int e = tid; e < m * m; e += kST) w.L[e] = w.N[e];
    __syncthreads();
    jacobi(m, w.L, w.L2, w.misc + 64, red);  // eigenvectors of N in L2
    sort_diag(m, w.L, w.v0, w.v1);
    if (tid == 0) {
        const double lmax = w.v0[m - 1];
        int rk = 0;
        if (lmax > 1e-12)
            for (int i = 0; i < m; ++i)
                if (w.v0[i] > drop * lmax) w.v2[rk++] = w.v1[i];  // kept eigenvector indices, ascending
        misc[1] = rk;
        misc[3] = lmax;
    }
    __syncthreads();
    const int rk = int(misc[1]);
    if (rk == 0) return;
    // X (m x rk) = U_kept / sqrt(ev) into Z; HX = H X into B; Bm = X^T HX into L
    for (int e = tid; e < m * rk; e += kST) {
        const int i = e / rk, c = e - i * rk;
        const int col = int(w.v2[c]);
        w.Z[i * rk + c] = w.L2[i * m + col] / sqrt(w.L[col * m + col]);
    }
    __syncthreads();
    for (int e = tid; e < m * rk; e += kST) {
        const int i = e / rk, c = e - i * rk;
        double acc = 0.0;
        for (int j = 0; j < m; ++j) acc += w.H[i * m + j] * w.Z[j * rk + c];
        w.B[i * rk + c] = acc;
    }
    __syncthreads();
    for (int e = tid; e < rk * rk; e += kST) {
        const int r = e / rk, c = e - r * rk;
        double acc = 0.0;
        for (int i = 0; i < m; ++i) acc += w.Z[i * rk + r] * w.B[i * rk + c];
        w.L[r * rk + c] = acc;
    }
    __syncthreads();
    symmetrise(rk, w.L);
    jacobi(rk, w.L, w.N, w.misc + 64, red);  // Ritz coefficients (in the kept basis) in N
    sort_diag(rk, w.L, w.v3, w.v4);
    // Xc = X C (columns in ascending Ritz order) into W; a = Xc[:, 0]
    for (int e = tid; e < m * rk; e += kST) {
        const int i = e / rk, c = e - i * rk;
        const int col = int(w.v4[c]);
        double acc = 0.0;
        for (int j = 0; j < rk; ++j) acc += w.Z[i * rk + j] * w.N[j * rk + col];
        w.W[i * rk + c] = acc;
    }
    __syncthreads();
    if (tid < m) w.v6[tid] = w.W[tid * rk];
    if (tid == 0) misc[0] = w.v3[0];
    __syncthreads();
}

// restart basis: Qk (m x nk) = modified Gram-Schmidt of the first nk
// columns of Xc (m x rk)
__device__ void restart_basis(int m, int rk, int nk, const double* Xc, double* Qk, double* red) {
    const int tid = threadIdx.x;
    for (int c = 0; c < nk; ++c) {
        double vi = (tid < m) ? Xc[tid * rk + c] : 0.0;
        for (int p = 0; p < c; ++p) {
            const double qp = (tid < m) ? Qk[tid * nk + p] : 0.0;
            const double d = wg_sum(qp * vi, red);
            vi -= d * qp;
        }
        const double nr = sqrt(wg_sum(vi * vi, red));
        if (tid < m) Qk[tid * nk + c] = vi / nr;
        __syncthreads();
    }
}

// M (stride S, leading m x m) <- Qk^T M Qk (nk x nk); tmp: m x nk
__device__ void rotate_projected(int m, int nk, int S, double* M, const double* Qk, double* tmp, double* res) {
    const int tid = threadIdx.x;
    for (int e = tid; e < m * nk; e += kST) {
        const int r = e / nk, c = e - r * nk;
        double v = 0.0;
        for (int j = 0; j < m; ++j) v += M[(long long)r * S + j] * Qk[j * nk + c];
        tmp[r * nk + c] = v;
    }
    __syncthreads();
    for (int e = tid; e < nk * nk; e += kST) {
        const int r = e / nk, c = e - r * nk;
        double v = 0.0;
        for (int j = 0; j < m; ++j) v += Qk[j * nk + r] * tmp[j * nk + c];
        res[e] = v;
    }
    __syncthreads();
    for (int e = tid; e < nk * nk; e += kST) {
        const int r = e / nk, c = e - r * nk;
        M[(long long)r * S + c] = res[e];
    }
    __syncthreads();
}

__device__ inline void write_status(DavInst& I) {
    if (!I.status) return;
    double* st = I.status;
    st[0] = I.active;
    st[1] = I.converged;
    st[2] = I.it;
    st[3] = I.matvecs;
    st[4] = I.theta;
    st[5] = I.rnorm;
    st[6] = I.pnorm;
    st[7] = I.err;
}

__global__ __launch_bounds__(64) void k_bdav_start(DavInst* __restrict__ insts) {
    DavInst* I = insts + blockIdx.x;
    if (threadIdx.x != 0 || !I->active) return;
    I->Ht[0] = chunk_total(I->pg, I->nch, 2, 0);
    I->Nt[0] = chunk_total(I->pg, I->nch, 2, 1);
    I->m = 1;
    I->mr = 1;
    I->it = 0;
    I->matvecs = 1;
    I->converged = 0;
    I->restart = 0;
    I->last = 0;
    I->err = 0;
    I->ext = 1;
    I->from_t = 1;
    I->theta = I->rnorm = I->pnorm = 0.0;
    write_status(*I);
}

__global__ __launch_bounds__(kST) void k_bdav_solve(DavInst* __restrict__ insts) {
    extern __shared__ double lds_solve[];
    __shared__ double red[kST];
    DavInst* P = insts + blockIdx.x;
    if (!P->active) return;
    const int tid = threadIdx.x;
    const int m = P->m, S = P->S;
    const int it = P->it + 1;
    const bool last = it >= P->max_iter;
    const bool restart = !last && m >= P->max_sub;
    Work w = carve(lds_solve, m);
    for (int e = tid; e < m * m; e += kST) {
        const int i = e / m, j = e - i * m;
        w.H[e] = 0.5 * (P->Ht[(long long)i * S + j] + P->Ht[(long long)j * S + i]);
        w.N[e] = 0.5 * (P->Nt[(long long)i * S + j] + P->Nt[(long long)j * S + i]);
    }
    __syncthreads();
    solve_pencil(m, w, P->drop, restart, red);
    const int rk = int(w.misc[1]);
    const double theta = w.misc[0];
    int nk = 0;
    if (rk > 0 && restart) {
        nk = min(P->keep, rk);
        restart_basis(m, rk, nk, w.W, P->Qk, red);
        rotate_projected(m, nk, S, P->Ht, P->Qk, w.Z, w.B);
        rotate_projected(m, nk, S, P->Nt, P->Qk, w.Z, w.B);
    }
    if (rk > 0 && tid < m) P->aqd[tid] = w.v6[tid];
    __syncthreads();
    if (tid == 0) {
        P->it = it;
        if (rk == 0 || !isfinite(theta)) {
            P->err = rk == 0 ? kSpErrNorm : kSpErrNan;
            P->active = 0;
            P->ext = 0;
        } else {
            P->aqd[m] = theta;
            P->theta = theta;
            P->last = last;
            P->restart = restart;
            P->nk = nk;
            P->mr = m;
            P->m = restart ? nk : m;
            P->ext = last ? 0 : 1;
            if (!last) P->matvecs += 1;
        }
        write_status(*P);
    }
}

// rotate V, HV, NV (blockIdx.y) of every restarting instance (blockIdx.z)
// in place: row c < nk becomes sum_j Q[j][c] row j, j < mr
__global__ __launch_bounds__(256) void k_bdav_rotate(const DavInst* __restrict__ insts) {
    const DavInst I = insts[blockIdx.z];
    if (!I.active || !I.restart) return;
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= I.n) return;
    double* A = blockIdx.y == 0 ? I.V : (blockIdx.y == 1 ? I.HV : I.NV);
    double acc[kDevKeepMax];
#pragma unroll
    for (int c = 0; c < kDevKeepMax; ++c) acc[c] = 0.0;
    for (int j = 0; j < I.mr; ++j) {
        const double a = A[(long long)j * I.ld + e];
#pragma unroll
        for (int c = 0; c < kDevKeepMax; ++c)
            if (c < I.nk) acc[c] = fma(I.Qk[j * I.nk + c], a, acc[c]);
    }
#pragma unroll
    for (int c = 0; c < kDevKeepMax; ++c)
        if (c < I.nk) A[(long long)c * I.ld + e] = acc[c];
}

__global__ __launch_bounds__(kST) void k_bdav_update(DavInst* __restrict__ insts) {
    __shared__ double tot[4 * kDevSubMax + 8];
    __shared__ double sh[4];
    DavInst* P = insts + blockIdx.x;
    if (!P->active) return;
    const int tid = threadIdx.x;
    const int m = P->m, S = P->S, nch = P->nch;
    const int nd = 4 * m + 2;
    // every chunk total at once, one thread per quantity (each in ascending
    // chunk order): the three Ritz sums, then the nd Gram rows
    if (tid < 3) tot[tid] = chunk_total(P->part_x, nch, 3, tid);
    else if (tid < 3 + nd && P->ext) tot[tid] = chunk_total(P->pg, nch, nd, tid - 3);
    __syncthreads();
    if (tid == 0) {
        const double xx = tot[0], uu = tot[1], xn = tot[2];
        int grow = 0;
        if (!isfinite(xx) || !isfinite(uu) || !(xx > 0.0)) {
            P->err = kSpErrNan;
            P->active = 0;
        } else {
            P->rnorm = sqrt(uu / xx);
            P->pnorm = xn / xx;
            if (P->rnorm <= P->tol) {
                P->converged = 1;
                P->active = 0;
            } else if (P->last) {
                P->active = 0;
            } else if (!(*P->tnorm >= 1e-14)) {
                P->active = 0;
            } else {
                grow = 1;
            }
        }
        sh[0] = grow;
    }
    __syncthreads();
    if (sh[0] != 0.0) {
        const double* g = tot + 3;
        for (int j = tid; j <= m; j += kST) {
            const double hv_new = g[j], nv_new = g[m + 1 + j];
            const double hv_old = (j < m) ? g[2 * m + 2 + j] : hv_new;
            const double nv_old = (j < m) ? g[3 * m + 2 + j] : nv_new;
            P->Ht[(long long)j * S + m] = hv_new;
            P->Nt[(long long)j * S + m] = nv_new;
            P->Ht[(long long)m * S + j] = hv_old;
            P->Nt[(long long)m * S + j] = nv_old;
        }
        __syncthreads();
        if (tid == 0) P->m = m + 1;
    }
    if (tid == 0) {
        P->ext = 0;
        write_status(*P);
    }
}

// one instance's solve on device copies of H, N (tests)
__global__ __launch_bounds__(kST) void k_small_solve_test(int m, double* H, double* N, double drop, int need_all,
                                                           int keep, double* out, double* Qk) {
    extern __shared__ double lds_solve[];
    __shared__ double red[kST];
    const int tid = threadIdx.x;
    Work w = carve(lds_solve, m);
    for (int e = tid; e < m * m; e += kST) {
        const int i = e / m, j = e - i * m;
        w.H[e] = 0.5 * (H[i * m + j] + H[j * m + i]);
        w.N[e] = 0.5 * (N[i * m + j] + N[j * m + i]);
    }
    __syncthreads();
    solve_pencil(m, w, drop, need_all != 0, red);
    const int rk = int(w.misc[1]);
    if (tid == 0) {
        out[0] = w.misc[0];
        out[1] = rk;
    }
    if (rk > 0 && tid < m) out[2 + tid] = w.v6[tid];
    __syncthreads();
    if (rk > 0 && need_all) {
        const int nk = min(keep, rk);
        restart_basis(m, rk, nk, w.W, Qk, red);
        rotate_projected(m, nk, m, H, Qk, w.Z, w.B);
        rotate_projected(m, nk, m, N, Qk, w.Z, w.B);
        if (tid == 0) out[1] = nk;
    }
}

}  // namespace

void bdav_start(hipStream_t s, DavInst* insts, int ninst) {
    if (ninst > 0) hipLaunchKernelGGL(k_bdav_start, dim3(ninst), dim3(64), 0, s, insts);
}
void bdav_solve(hipStream_t s, DavInst* insts, int ninst, int max_m) {
    if (ninst > 0)
        hipLaunchKernelGGL(k_bdav_solve, dim3(ninst), dim3(kST), size_t(dev_solve_lds(max_m)), s, insts);
}
void bdav_rotate(hipStream_t s, const DavInst* insts, int ninst, int max_n) {
    if (ninst > 0) hipLaunchKernelGGL(k_bdav_rotate, dim3((max_n + 255) / 256, 3, ninst), dim3(256), 0, s, insts);
}
void bdav_update(hipStream_t s, DavInst* insts, int ninst) {
    if (ninst > 0) hipLaunchKernelGGL(k_bdav_update, dim3(ninst), dim3(kST), 0, s, insts);
}

int dev_small_solve(int m, double* H, double* N, double drop, int need_all, int keep, double* theta, double* a,
                    double* Qk) {
    if (m < 1 || m >= kDevSubMax || keep < 1 || keep > kDevKeepMax) return -1;
    double *dH = nullptr, *dN = nullptr, *dout = nullptr, *dQ = nullptr;
    const size_t mm = size_t(m) * m;
    if (hipMalloc(&dH, mm * 8) != hipSuccess || hipMalloc(&dN, mm * 8) != hipSuccess ||
        hipMalloc(&dout, (m + 2) * 8) != hipSuccess || hipMalloc(&dQ, mm * 8) != hipSuccess) {
        (void)hipFree(dH);
        (void)hipFree(dN);
        (void)hipFree(dout);
        (void)hipFree(dQ);
        return -2;
    }
    (void)hipMemcpy(dH, H, mm * 8, hipMemcpyHostToDevice);
    (void)hipMemcpy(dN, N, mm * 8, hipMemcpyHostToDevice);
    hipLaunchKernelGGL(k_small_solve_test, dim3(1), dim3(kST), size_t(dev_solve_lds(m)), 0, m, dH, dN, drop, need_all,
                       keep, dout, dQ);
    int rc = (hipDeviceSynchronize() == hipSuccess) ? 0 : -3;
    std::vector<double> out(m + 2);
    if (rc == 0) {
        (void)hipMemcpy(out.data(), dout, (m + 2) * 8, hipMemcpyDeviceToHost);
        *theta = out[0];
        const int rk = int(out[1]);
        for (int i = 0; i < m; ++i) a[i] = out[2 + i];
        if (need_all && rk > 0 && Qk) {
            (void)hipMemcpy(Qk, dQ, size_t(m) * rk * 8, hipMemcpyDeviceToHost);
            (void)hipMemcpy(H, dH, mm * 8, hipMemcpyDeviceToHost);
            (void)hipMemcpy(N, dN, mm * 8, hipMemcpyDeviceToHost);
        }
        rc = rk;
    }
    (void)hipFree(dH);
    (void)hipFree(dN);
    (void)hipFree(dout);
    (void)hipFree(dQ);
    return rc;
}

}  // namespace spk
