// Per-N-block scope of the learned Davidson preconditioner (mlp.hip): groups
// of element ranges (the N-blocks of a site tensor) and the grouped
// variants of the feature and target kernels declared in kernels.h.
#pragma once

#include <hip/hip_runtime.h>

namespace spk {

// group q holds ranges gptr[q] .. gptr[q+1] - 1, range j the elements
// roff[j] .. roff[j] + rlen[j] - 1
struct ElemGroups {
    int ng;
    const int* gptr;
    const long long* roff;
    const int* rlen;
};

// mlp_apply with, for gid not null, element i in group gid[i]: the root mean
// squares are grms[2 gid[i]] (r) and grms[2 gid[i] + 1] (t) instead of
// those of rr, tt, and the correction is scaled by the group's rms of t
void mlp_apply_grouped(hipStream_t s, const float* w, int H, double* t, const double* dh, const double* dn,
                       const double* theta, const double* rr, const double* tt, int n, double floor_, float* feat,
                       float* sgn, const int* gid, const double* grms);
// grms[2q] = rms of r = -t d' and grms[2q+1] = rms of t over group q (one
// work-group per group, fixed order)
void mlp_group_rms(hipStream_t s, const double* t, const double* dh, const double* dn, const double* theta,
                   double floor_, ElemGroups g, double* grms);
// mlp_targets with e_j divided by its rms over each element's group; scal:
// 2 nrec doubles of device scratch
void mlp_targets_grouped(hipStream_t s, const double* X, long long ldx, int nrec, const double* xstar, int n,
                         ElemGroups g, double* scal, float* Y);

}  // namespace spk
