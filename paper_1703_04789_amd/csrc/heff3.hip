// The fused H_eff x / N_eff x kernel for gfx950 (FP64, or FP32 in the
// reduced-precision mode): one work-group per (quadrature point, bra
// particle-number block, chunk of rows) runs the left product, the W r
// mixing (Eq. [geproblem]) and the right product of its rows in one launch,
// through LDS, and writes per-g partial outputs that the g sum adds in a
// fixed order.  Kept in its own file so that its hardware-counter profiles
// are keyed to this source alone.
#include "kernels.h"

namespace spk {

namespace {

template <int RC, typename T, bool BATCH>
__global__ __launch_bounds__(kH3Threads) void k_heff3(const H3Task* __restrict__ tasks,
                                                        const H3Inst* __restrict__ insts, H3Inst one) {
    extern __shared__ double lds_raw[];
    T* lds = reinterpret_cast<T*>(lds_raw);
    const H3Task* __restrict__ tkp = tasks + blockIdx.x;
    const int blk = tkp->blk;
    if (blk < 0) return;
    const H3Inst I = BATCH ? insts[tkp->inst] : one;
    if (I.gate && *I.gate == 0) return;
    const H3Col* __restrict__ cols = I.cols;
    const H3LSrc* __restrict__ lsrc = I.lsrc;
    const H3Seg* __restrict__ segs = I.segs;
    const H3Term* __restrict__ terms = I.terms;
    const H3Piece* __restrict__ pieces = I.pieces;
    const double* __restrict__ x = I.x;
    double* __restrict__ ypart = I.ypart;
    double* __restrict__ nypart = I.nypart;
    const long long n = I.n;
    const int g = tkp->g, r0 = tkp->r0, rows = tkp->rows;
    const H3Blk* __restrict__ bp = I.blks + blk;
    const T* __restrict__ L = static_cast<const T*>(I.Lenv) + g * I.Lsz;
    const T* __restrict__ R = static_cast<const T*>(I.Renv) + g * I.Rsz;
    const double* __restrict__ cf = I.coef + (long long)g * I.nc;
    const int tid = threadIdx.x;

    // stage the chunk's rows of the left-environment blocks (zero rows past
    // the chunk so that every later loop runs over exactly RC rows)
    const int l0 = bp->l0, l1 = bp->l1;
    for (int q = l0; q < l1; ++q) {
        const H3LSrc src = lsrc[q];
        const int tot = RC * src.ld;
        const T* __restrict__ lrow = L + src.l_off + (long long)r0 * src.ld;
        for (int e = tid; e < tot; e += kH3Threads) lds[src.lds + e] = (e < rows * src.ld) ? lrow[e] : T(0);
    }
    __syncthreads();

    // phase A: T columns, two neighbours per thread; neighbours reading the
    // same x column (the plan sorts them together) load it once
    const int c0 = bp->c0, c1 = bp->c1;
    for (int ci = c0 + 2 * tid; ci + 1 < c1; ci += 2 * kH3Threads) {
        const H3Col ca = cols[ci], cb = cols[ci + 1];
        if (ca.K == 0 || ca.x_off != cb.x_off || ca.x_ld != cb.x_ld || ca.K != cb.K) {
            for (int h = 0; h < 2; ++h) {
                const H3Col c = h ? cb : ca;
                T acc[RC];
#pragma unroll
                for (int rr = 0; rr < RC; ++rr) acc[rr] = T(0);
                const double* __restrict__ xp = x + c.x_off;
                const T* lp = lds + c.l_lds;
                for (int kk = 0; kk < c.K; ++kk) {
                    const T xv = T(xp[kk * c.x_ld]);
#pragma unroll
                    for (int rr = 0; rr < RC; ++rr) acc[rr] = fma(lp[rr * c.l_ld + kk], xv, acc[rr]);
                }
#pragma unroll
                for (int rr = 0; rr < RC; ++rr) lds[c.t_pos + rr] = acc[rr];
            }
            continue;
        }
        T aa[RC], ab[RC];
#pragma unroll
        for (int rr = 0; rr < RC; ++rr) aa[rr] = ab[rr] = T(0);
        const double* __restrict__ xp = x + ca.x_off;
        const T* la = lds + ca.l_lds;
        const T* lb = lds + cb.l_lds;
        int kk = 0;
        for (; kk + 4 <= ca.K; kk += 4) {
            const T x0 = T(xp[kk * ca.x_ld]), x1 = T(xp[(kk + 1) * ca.x_ld]);
            const T x2 = T(xp[(kk + 2) * ca.x_ld]), x3 = T(xp[(kk + 3) * ca.x_ld]);
#pragma unroll
            for (int rr = 0; rr < RC; ++rr) {
                const T* l = la + rr * ca.l_ld + kk;
                aa[rr] = fma(l[3], x3, fma(l[2], x2, fma(l[1], x1, fma(l[0], x0, aa[rr]))));
                const T* m = lb + rr * cb.l_ld + kk;
                ab[rr] = fma(m[3], x3, fma(m[2], x2, fma(m[1], x1, fma(m[0], x0, ab[rr]))));
            }
        }
        for (; kk < ca.K; ++kk) {
            const T xv = T(xp[kk * ca.x_ld]);
#pragma unroll
            for (int rr = 0; rr < RC; ++rr) {
                aa[rr] = fma(la[rr * ca.l_ld + kk], xv, aa[rr]);
                ab[rr] = fma(lb[rr * cb.l_ld + kk], xv, ab[rr]);
            }
        }
#pragma unroll
        for (int rr = 0; rr < RC; ++rr) {
            lds[ca.t_pos + rr] = aa[rr];
            lds[cb.t_pos + rr] = ab[rr];
        }
    }
    // an odd count leaves the last column to one thread
    if (((c1 - c0) & 1) && tid == kH3Threads - 1) {
        const H3Col c = cols[c1 - 1];
        T acc[RC];
#pragma unroll
        for (int rr = 0; rr < RC; ++rr) acc[rr] = T(0);
        const double* __restrict__ xp = x + c.x_off;
        const T* lp = lds + c.l_lds;
        for (int kk = 0; kk < c.K; ++kk) {
            const T xv = T(xp[kk * c.x_ld]);
#pragma unroll
            for (int rr = 0; rr < RC; ++rr) acc[rr] = fma(lp[rr * c.l_ld + kk], xv, acc[rr]);
        }
#pragma unroll
        for (int rr = 0; rr < RC; ++rr) lds[c.t_pos + rr] = acc[rr];
    }
    __syncthreads();

    for (int sg = 0; sg < 4; ++sg) {
        const int p0 = tkp->p0[sg], p1 = tkp->p1[sg];
        if (p0 == p1) continue;
        const int s0 = bp->s0[sg], s1 = bp->s1[sg];
        // V of every right channel of sigma (the W r mixing)
        for (int si = s0; si < s1; ++si) {
            const H3Seg S = segs[si];
            const int ne = S.K * RC;
            for (int e = tid; e < ne; e += kH3Threads) {
                T v = T(0);
                for (int t = S.t0; t < S.t1; ++t) {
                    const H3Term tm = terms[t];
                    v = fma(T(cf[tm.cidx]), lds[tm.t_base + e], v);
                }
                lds[S.v_off + e] = v;
            }
        }
        __syncthreads();
        // outputs: one group of SL lanes per output column of a piece
        int items = 0;
        for (int p = p0; p < p1; ++p) items += pieces[p].nb;
        int SL = kH3SlMax;
        while (SL > 1 && items * SL > kH3Threads) SL >>= 1;
        const int sl = tid & (SL - 1);
        for (int it = tid / SL; it < items; it += kH3Threads / SL) {
            int p = p0, b = it;
            while (b >= pieces[p].nb) {
                b -= pieces[p].nb;
                ++p;
            }
            const H3Piece P = pieces[p];
            T ay[RC], an[RC];
#pragma unroll
            for (int rr = 0; rr < RC; ++rr) ay[rr] = an[rr] = T(0);
            for (int si = s0; si < s1; ++si) {
                const H3Seg S = segs[si];
                const T* __restrict__ rp = R + S.r_off + (long long)(P.b0 + b) * S.K;
                const T* vp = lds + S.v_off;
                const int K = S.K;
                if (S.is_ny) {
                    int k = sl;
                    for (; k + SL < K; k += 2 * SL) {
                        const T ra = rp[k], rb = rp[k + SL];
#pragma unroll
                        for (int rr = 0; rr < RC; ++rr)
                            an[rr] = fma(vp[(k + SL) * RC + rr], rb, fma(vp[k * RC + rr], ra, an[rr]));
                    }
                    for (; k < K; k += SL) {
                        const T r = rp[k];
#pragma unroll
                        for (int rr = 0; rr < RC; ++rr) an[rr] = fma(vp[k * RC + rr], r, an[rr]);
                    }
                } else {
                    int k = sl;
                    for (; k + 3 * SL < K; k += 4 * SL) {
                        const T ra = rp[k], rb = rp[k + SL], rc = rp[k + 2 * SL], rd = rp[k + 3 * SL];
#pragma unroll
                        for (int rr = 0; rr < RC; ++rr) {
                            T v = ay[rr];
                            v = fma(vp[k * RC + rr], ra, v);
                            v = fma(vp[(k + SL) * RC + rr], rb, v);
                            v = fma(vp[(k + 2 * SL) * RC + rr], rc, v);
                            ay[rr] = fma(vp[(k + 3 * SL) * RC + rr], rd, v);
                        }
                    }
                    for (; k < K; k += SL) {
                        const T r = rp[k];
#pragma unroll
                        for (int rr = 0; rr < RC; ++rr) ay[rr] = fma(vp[k * RC + rr], r, ay[rr]);
                    }
                }
            }
            for (int o = SL >> 1; o > 0; o >>= 1) {
#pragma unroll
                for (int rr = 0; rr < RC; ++rr) {
                    ay[rr] += __shfl_xor(ay[rr], o, 64);
                    an[rr] += __shfl_xor(an[rr], o, 64);
                }
            }
            if (sl == 0) {
                const long long base = g * n + P.out_off + b;
#pragma unroll
                for (int rr = 0; rr < RC; ++rr) {
                    if (rr >= P.rlo && rr < P.rhi) {
                        const long long o = base + (long long)(rr - P.rlo) * P.out_ld;
                        ypart[o] = double(ay[rr]);
                        nypart[o] = double(an[rr]);
                    }
                }
            }
        }
        __syncthreads();
    }
}

}  // namespace

template <typename T>
static void launch_heff3(hipStream_t s, int RC, int lds_elems, const H3Task* tasks, int ntasks, const H3Inst& I,
                         const H3Inst* insts) {
    if (ntasks <= 0) return;
    const size_t shm = size_t(lds_elems) * sizeof(T);
#define SPK_HEFF3(R)                                                                                               \
    case R:                                                                                                        \
        if (insts)                                                                                                 \
            hipLaunchKernelGGL((k_heff3<R, T, true>), dim3(ntasks), dim3(kH3Threads), shm, s, tasks, insts, I);    \
        else                                                                                                       \
            hipLaunchKernelGGL((k_heff3<R, T, false>), dim3(ntasks), dim3(kH3Threads), shm, s, tasks, insts, I);   \
        break;
    switch (RC) {
        SPK_HEFF3(1)
        SPK_HEFF3(2)
        SPK_HEFF3(3)
        SPK_HEFF3(4)
        SPK_HEFF3(5)
        SPK_HEFF3(6)
        SPK_HEFF3(7)
        SPK_HEFF3(8)
        default:
            break;
    }
#undef SPK_HEFF3
}
void heff3(hipStream_t s, int RC, int lds_elems, const H3Task* tasks, int ntasks, const H3Inst& I,
           const H3Inst* insts) {
    launch_heff3<double>(s, RC, lds_elems, tasks, ntasks, I, insts);
}
void heff3_f32(hipStream_t s, int RC, int lds_elems, const H3Task* tasks, int ntasks, const H3Inst& I,
               const H3Inst* insts) {
    launch_heff3<float>(s, RC, lds_elems, tasks, ntasks, I, insts);
}

}  // namespace spk
