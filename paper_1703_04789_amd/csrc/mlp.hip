// Learned Davidson preconditioner: a two-layer perceptron applied to every
// element of the site tensor, its training pairs and its training.
//
// The paper leaves the local solver of Sec. 2.3 open; the library's solver
// is Davidson with the diagonal correction t = -r / (dh - theta dn).  The
// learned variant maps five features of each element,
//   f0 = |r_i| / rms(r), f1 = asinh(d_i), f2 = asinh(dn_i), f3 = asinh(-f0 / d_i'),
//   f4 = sign(r_i) t_i / rms(t)   (t = -r / d', the diagonal correction)
// (d = dh - theta dn, d' = d floored to |d'| >= floor) to
// t_i = sign(r_i) (w2 . relu(W1 f + b1) + b2): odd in r like a linear
// preconditioner, so the free sign of the Ritz vector does not matter.
// Davidson normalises t, so the scale is free.  Training targets are the
// solver's own exact corrections e_j = x*/(x_j . x*) - x_j (x_j the unit Ritz
// vector of iteration j, x* the converged one) divided by rms(e_j), times
// sign(r_i).
// Per-N-block scope: the root mean squares in f0 and f4 and in the targets
// are taken over the element's N-block of the site tensor (elements sharing
// both bond particle numbers), and the correction is scaled by the block's
// rms of the diagonal correction, so the model shapes the correction inside
// a block and the diagonal rule keeps the block's weight.
// Weights and recorded pairs are FP32 in memory; all arithmetic is FP64.
// Packed weights: W1 (H x 5, row-major) | b1 (H) | w2 (H) | b2.

#include <hip/hip_runtime.h>

#include "kernels.h"
#include "mlp.h"

namespace spk {

namespace {

constexpr int kMlpThreads = 256;

__device__ inline double wsum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// fixed-order sum over a work-group of blockDim.x (a multiple of 64) threads
__device__ inline double group_sum(double v, double* red) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    v = wsum(v);
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double r = 0.0;
    for (int w = 0; w < nw; ++w) r += red[w];
    return r;
}

__device__ inline double mlp_eval(const double* sw, int H, const double f[kMlpIn]) {
    const double* W1 = sw;
    const double* b1 = sw + H * kMlpIn;
    const double* w2 = b1 + H;
    double y = w2[H];  // b2
    for (int j = 0; j < H; ++j) {
        double z = b1[j];
#pragma unroll
        for (int c = 0; c < kMlpIn; ++c) z = fma(W1[j * kMlpIn + c], f[c], z);
        y = fma(w2[j], fmax(z, 0.0), y);
    }
    return y;
}

__device__ inline void load_weights(const float* __restrict__ w, int H, double* sw) {
    const int P = int(mlp_size(H));
    for (int p = threadIdx.x; p < P; p += blockDim.x) sw[p] = double(w[p]);
    __syncthreads();
}

__global__ __launch_bounds__(kMlpThreads) void k_sum_partials(const double* __restrict__ part, int nchunk, int stride,
                                                              int idx, double* __restrict__ out) {
    __shared__ double red[kMlpThreads / 64];
    double s = 0.0;
    for (int q = threadIdx.x; q < nchunk; q += kMlpThreads) s += part[(long long)q * stride + idx];
    s = group_sum(s, red);
    if (threadIdx.x == 0) *out = s;
}

// features of every element from the diagonal correction t = -r / d' (so
// r = -t d'), optionally recorded with sign(r_i) (feat, sgn), then optionally
// the model's correction in place of t
__global__ __launch_bounds__(kMlpThreads) void k_mlp_apply(const float* __restrict__ w, int H, double* __restrict__ t,
                                                           const double* __restrict__ dh,
                                                           const double* __restrict__ dn,
                                                           const double* __restrict__ theta,
                                                           const double* __restrict__ rr,
                                                           const double* __restrict__ tt, int n, double floor_,
                                                           float* __restrict__ feat, float* __restrict__ sgn,
                                                           const int* __restrict__ gid,
                                                           const double* __restrict__ grms) {
    extern __shared__ double sw[];
    if (w) load_weights(w, H, sw);
    const int i = blockIdx.x * kMlpThreads + threadIdx.x;
    if (i >= n) return;
    const double th = *theta;
    double rms, rmst;
    if (gid) {
        const int q = gid[i];
        rms = grms[2 * q];
        rmst = grms[2 * q + 1];
    } else {
        rms = sqrt(*rr / n);
        rmst = sqrt(*tt / n);
    }
    const double d = dh[i] - th * dn[i];
    const double dfl = fabs(d) < floor_ ? (d < 0.0 ? -floor_ : floor_) : d;
    const double r = -t[i] * dfl;
    const double sr = r > 0.0 ? 1.0 : (r < 0.0 ? -1.0 : 0.0);
    const double f0 = rms > 0.0 ? fabs(r) / rms : 0.0;
    double f[kMlpIn] = {f0, asinh(d), asinh(dn[i]), asinh(-f0 / dfl), rmst > 0.0 ? sr * t[i] / rmst : 0.0};
    if (feat) {
#pragma unroll
        for (int c = 0; c < kMlpIn; ++c) feat[(long long)i * kMlpIn + c] = float(f[c]);
        sgn[i] = float(sr);
    }
    if (w) t[i] = sr * mlp_eval(sw, H, f) * (gid ? rmst : 1.0);
}

// one work-group per group of element ranges: rms of r = -t d' and of t
__global__ __launch_bounds__(kMlpThreads) void k_mlp_group_rms(const double* __restrict__ t,
                                                               const double* __restrict__ dh,
                                                               const double* __restrict__ dn,
                                                               const double* __restrict__ theta, double floor_,
                                                               ElemGroups g, double* __restrict__ grms) {
    __shared__ double red[kMlpThreads / 64];
    const int q = blockIdx.x;
    const double th = *theta;
    double rr = 0.0, tt = 0.0;
    long long cnt = 0;
    for (int j = g.gptr[q]; j < g.gptr[q + 1]; ++j) {
        const long long o = g.roff[j];
        cnt += g.rlen[j];
        for (int e = threadIdx.x; e < g.rlen[j]; e += kMlpThreads) {
            const long long i = o + e;
            const double d = dh[i] - th * dn[i];
            const double dfl = fabs(d) < floor_ ? (d < 0.0 ? -floor_ : floor_) : d;
            const double r = -t[i] * dfl;
            rr = fma(r, r, rr);
            tt = fma(t[i], t[i], tt);
        }
    }
    rr = group_sum(rr, red);
    tt = group_sum(tt, red);
    if (threadIdx.x == 0) {
        grms[2 * q] = cnt > 0 ? sqrt(rr / double(cnt)) : 0.0;
        grms[2 * q + 1] = cnt > 0 ? sqrt(tt / double(cnt)) : 0.0;
    }
}

__global__ __launch_bounds__(1024) void k_sumsq(const double* __restrict__ v, int n, double* __restrict__ out) {
    __shared__ double red[16];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 1024) s = fma(v[i], v[i], s);
    s = group_sum(s, red);
    if (threadIdx.x == 0) *out = s;
}

__global__ __launch_bounds__(kMlpThreads) void k_mlp_forward(const float* __restrict__ w, int H,
                                                             const float* __restrict__ F, long long n,
                                                             float* __restrict__ y) {
    extern __shared__ double sw[];
    load_weights(w, H, sw);
    const long long i = (long long)blockIdx.x * kMlpThreads + threadIdx.x;
    if (i >= n) return;
    double f[kMlpIn];
#pragma unroll
    for (int c = 0; c < kMlpIn; ++c) f[c] = F[i * kMlpIn + c];
    y[i] = float(mlp_eval(sw, H, f));
}

// one work-group per recorded iteration j: Y_j = sign(r_j) e_j / rms(e_j),
// e_j = x*/(xh . x*) - xh, xh = x_j / |x_j|; Y_j holds sign(r_j) on entry
__global__ __launch_bounds__(1024) void k_mlp_targets(const double* __restrict__ X, long long ldx,
                                                      const double* __restrict__ xs, int n, float* __restrict__ Y) {
    __shared__ double red[16];
    const double* x = X + (long long)blockIdx.x * ldx;
    float* out = Y + (long long)blockIdx.x * n;
    double xx = 0.0, xy = 0.0;
    for (int i = threadIdx.x; i < n; i += 1024) {
        xx = fma(x[i], x[i], xx);
        xy = fma(x[i], xs[i], xy);
    }
    xx = group_sum(xx, red);
    xy = group_sum(xy, red);
    const double nx = sqrt(xx);
    const double c = xy / nx;  // xh . x*
    double ee = 0.0;
    for (int i = threadIdx.x; i < n; i += 1024) {
        const double e = xs[i] / c - x[i] / nx;
        ee = fma(e, e, ee);
    }
    ee = group_sum(ee, red);
    const double rms = sqrt(ee / n);
    const double inv = rms > 0.0 ? 1.0 / rms : 0.0;
    for (int i = threadIdx.x; i < n; i += 1024) out[i] = float(double(out[i]) * (xs[i] / c - x[i] / nx) * inv);
}

// grouped targets, first pass: one work-group per recorded iteration j,
// scal[2j] = |x_j|, scal[2j+1] = xh . x*
__global__ __launch_bounds__(1024) void k_mlp_target_dots(const double* __restrict__ X, long long ldx,
                                                          const double* __restrict__ xs, int n,
                                                          double* __restrict__ scal) {
    __shared__ double red[16];
    const double* x = X + (long long)blockIdx.x * ldx;
    double xx = 0.0, xy = 0.0;
    for (int i = threadIdx.x; i < n; i += 1024) {
        xx = fma(x[i], x[i], xx);
        xy = fma(x[i], xs[i], xy);
    }
    xx = group_sum(xx, red);
    xy = group_sum(xy, red);
    if (threadIdx.x == 0) {
        const double nx = sqrt(xx);
        scal[2 * blockIdx.x] = nx;
        scal[2 * blockIdx.x + 1] = xy / nx;
    }
}

// grouped targets, second pass: work-group (group q, iteration j) divides
// e_j on the group's ranges by its rms there; Y holds sign(r) on entry
__global__ __launch_bounds__(kMlpThreads) void k_mlp_targets_grouped(const double* __restrict__ X, long long ldx,
                                                                     const double* __restrict__ xs, int n,
                                                                     ElemGroups g, const double* __restrict__ scal,
                                                                     float* __restrict__ Y) {
    __shared__ double red[kMlpThreads / 64];
    const int q = blockIdx.x, j = blockIdx.y;
    const double* x = X + (long long)j * ldx;
    float* out = Y + (long long)j * n;
    const double nx = scal[2 * j], c = scal[2 * j + 1];
    double ee = 0.0;
    long long cnt = 0;
    for (int k = g.gptr[q]; k < g.gptr[q + 1]; ++k) {
        const long long o = g.roff[k];
        cnt += g.rlen[k];
        for (int e = threadIdx.x; e < g.rlen[k]; e += kMlpThreads) {
            const double v = xs[o + e] / c - x[o + e] / nx;
            ee = fma(v, v, ee);
        }
    }
    ee = group_sum(ee, red);
    const double rms = cnt > 0 ? sqrt(ee / double(cnt)) : 0.0;
    const double inv = rms > 0.0 ? 1.0 / rms : 0.0;
    for (int k = g.gptr[q]; k < g.gptr[q + 1]; ++k) {
        const long long o = g.roff[k];
        for (int e = threadIdx.x; e < g.rlen[k]; e += kMlpThreads) {
            const long long i = o + e;
            out[i] = float(double(out[i]) * (xs[i] / c - x[i] / nx) * inv);
        }
    }
}

// gradient partials of 0.5 * sum (y - Y)^2 over rows row0 + q*stride,
// q in this work-group's share of [0, count): thread j owns hidden unit j;
// four rows per reduction round
__global__ __launch_bounds__(kMlpThreads) void k_mlp_grad(const float* __restrict__ w, int H,
                                                          const float* __restrict__ F, const float* __restrict__ Y,
                                                          long long row0, long long stride, long long count,
                                                          double* __restrict__ gpart) {
    __shared__ double sf[4][kMlpIn + 1];
    __shared__ double sred[4][kMlpThreads / 64];
    __shared__ double sy[4];
    const int j = threadIdx.x;
    const bool own = j < H;
    double W1[kMlpIn] = {}, b1 = 0.0, w2 = 0.0;
    if (own) {
#pragma unroll
        for (int c = 0; c < kMlpIn; ++c) W1[c] = w[j * kMlpIn + c];
        b1 = w[H * kMlpIn + j];
        w2 = w[H * kMlpIn + H + j];
    }
    const double b2 = w[H * (kMlpIn + 2)];
    double gW1[kMlpIn] = {}, gb1 = 0.0, gw2 = 0.0, gb2 = 0.0, loss = 0.0;
    const long long per = (count + gridDim.x - 1) / gridDim.x;
    const long long q0 = (long long)blockIdx.x * per, q1 = min(count, q0 + per);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (long long q = q0; q < q1; q += 4) {
        const int ns = int(min(4LL, q1 - q));
        __syncthreads();
        if (threadIdx.x < 4 * (kMlpIn + 1)) {
            const int s = threadIdx.x / (kMlpIn + 1), c = threadIdx.x % (kMlpIn + 1);
            double v = 0.0;
            if (s < ns) {
                const long long row = row0 + (q + s) * stride;
                v = (c < kMlpIn) ? double(F[row * kMlpIn + c]) : double(Y[row]);
            }
            sf[s][c] = v;
        }
        __syncthreads();
        double z[4], h[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            double zz = b1;
#pragma unroll
            for (int c = 0; c < kMlpIn; ++c) zz = fma(W1[c], sf[s][c], zz);
            z[s] = zz;
            h[s] = own ? fmax(zz, 0.0) : 0.0;
            const double p = wsum(w2 * h[s]);
            if (lane == 0) sred[s][wave] = p;
        }
        __syncthreads();
        if (threadIdx.x < 4) {
            double y = b2;
            for (int v = 0; v < kMlpThreads / 64; ++v) y += sred[threadIdx.x][v];
            sy[threadIdx.x] = y;
        }
        __syncthreads();
        for (int s = 0; s < ns; ++s) {
            const double dy = sy[s] - sf[s][kMlpIn];
            if (own) {
                gw2 = fma(dy, h[s], gw2);
                if (z[s] > 0.0) {
                    const double dz = dy * w2;
                    gb1 += dz;
#pragma unroll
                    for (int c = 0; c < kMlpIn; ++c) gW1[c] = fma(dz, sf[s][c], gW1[c]);
                }
            }
            if (threadIdx.x == 0) {
                gb2 += dy;
                loss = fma(dy, dy, loss);
            }
        }
    }
    const long long P = mlp_size(H) + 1;
    double* g = gpart + (long long)blockIdx.x * P;
    if (own) {
#pragma unroll
        for (int c = 0; c < kMlpIn; ++c) g[j * kMlpIn + c] = gW1[c];
        g[H * kMlpIn + j] = gb1;
        g[H * kMlpIn + H + j] = gw2;
    }
    if (threadIdx.x == 0) {
        g[H * (kMlpIn + 2)] = gb2;
        g[P - 1] = loss;
    }
}

// Adam step: gradient = scale * (sum of the partials in work-group order)
__global__ __launch_bounds__(kMlpThreads) void k_mlp_adam(float* __restrict__ w, double* __restrict__ m,
                                                          double* __restrict__ v, int H,
                                                          const double* __restrict__ gpart, int nparts,
                                                          double scale, double lr, int step,
                                                          double* __restrict__ loss_out) {
    const long long P = mlp_size(H) + 1;
    const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
    const double c1 = 1.0 - pow(b1, step), c2 = 1.0 - pow(b2, step);
    for (long long p = threadIdx.x; p < P - 1; p += kMlpThreads) {
        double g = 0.0;
        for (int b = 0; b < nparts; ++b) g += gpart[b * P + p];
        g *= scale;
        const double mm = b1 * m[p] + (1.0 - b1) * g;
        const double vv = b2 * v[p] + (1.0 - b2) * g * g;
        m[p] = mm;
        v[p] = vv;
        w[p] = float(double(w[p]) - lr * (mm / c1) / (sqrt(vv / c2) + eps));
    }
    if (threadIdx.x == 0 && loss_out) {
        double l = 0.0;
        for (int b = 0; b < nparts; ++b) l += gpart[b * P + P - 1];
        *loss_out = 0.5 * l * scale;
    }
}

inline int blocks_for(long long n) { return int((n + kMlpThreads - 1) / kMlpThreads); }

}  // namespace

void sum_partials(hipStream_t s, const double* part, int nchunk, int stride, int idx, double* out) {
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kMlpThreads), 0, s, part, nchunk, stride, idx, out);
}

void mlp_apply(hipStream_t s, const float* w, int H, double* t, const double* dh, const double* dn,
               const double* theta, const double* rr, const double* tt, int n, double floor_, float* feat,
               float* sgn) {
    mlp_apply_grouped(s, w, H, t, dh, dn, theta, rr, tt, n, floor_, feat, sgn, nullptr, nullptr);
}

void mlp_apply_grouped(hipStream_t s, const float* w, int H, double* t, const double* dh, const double* dn,
                       const double* theta, const double* rr, const double* tt, int n, double floor_, float* feat,
                       float* sgn, const int* gid, const double* grms) {
    if (n <= 0) return;
    const size_t lds = w ? size_t(mlp_size(H)) * sizeof(double) : 0;
    hipLaunchKernelGGL(k_mlp_apply, dim3(blocks_for(n)), dim3(kMlpThreads), lds, s, w, H, t, dh, dn, theta, rr, tt,
                       n, floor_, feat, sgn, gid, grms);
}

void mlp_group_rms(hipStream_t s, const double* t, const double* dh, const double* dn, const double* theta,
                   double floor_, ElemGroups g, double* grms) {
    if (g.ng > 0)
        hipLaunchKernelGGL(k_mlp_group_rms, dim3(g.ng), dim3(kMlpThreads), 0, s, t, dh, dn, theta, floor_, g, grms);
}

void sumsq(hipStream_t s, const double* v, int n, double* out) {
    hipLaunchKernelGGL(k_sumsq, dim3(1), dim3(1024), 0, s, v, n, out);
}

void mlp_forward(hipStream_t s, const float* w, int H, const float* F, long long n, float* y) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_mlp_forward, dim3(blocks_for(n)), dim3(kMlpThreads), size_t(mlp_size(H)) * sizeof(double), s,
                       w, H, F, n, y);
}

void mlp_targets(hipStream_t s, const double* X, long long ldx, int nrec, const double* xstar, int n, float* Y) {
    if (nrec > 0 && n > 0) hipLaunchKernelGGL(k_mlp_targets, dim3(nrec), dim3(1024), 0, s, X, ldx, xstar, n, Y);
}

void mlp_targets_grouped(hipStream_t s, const double* X, long long ldx, int nrec, const double* xstar, int n,
                         ElemGroups g, double* scal, float* Y) {
    if (nrec <= 0 || n <= 0 || g.ng <= 0) return;
    hipLaunchKernelGGL(k_mlp_target_dots, dim3(nrec), dim3(1024), 0, s, X, ldx, xstar, n, scal);
    hipLaunchKernelGGL(k_mlp_targets_grouped, dim3(g.ng, nrec), dim3(kMlpThreads), 0, s, X, ldx, xstar, n, g, scal,
                       Y);
}

void mlp_grad(hipStream_t s, const float* w, int H, const float* F, const float* Y, long long row0, long long stride,
              long long count, double* gpart, int nparts) {
    hipLaunchKernelGGL(k_mlp_grad, dim3(nparts), dim3(kMlpThreads), 0, s, w, H, F, Y, row0, stride, count, gpart);
}

void mlp_adam(hipStream_t s, float* w, double* m, double* v, int H, const double* gpart, int nparts, double scale,
              double lr, int step, double* loss_out) {
    hipLaunchKernelGGL(k_mlp_adam, dim3(1), dim3(kMlpThreads), 0, s, w, m, v, H, gpart, nparts, scale, lr, step,
                       loss_out);
}

}  // namespace spk
