// Device kernels of the SP-MPS hot path (gfx950) and their launch wrappers.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace spk {

constexpr int kMaxBufs = 10;

// One output block C (M x N, row stride ldc) = sum over terms of
// coef[cidx] * A(M x K) B(K x N); accumulate != 0 adds to C.  A term with
// strides (a_rs, a_cs) reads A(r, k) = bufs[a_buf][a_off + r*a_rs + k*a_cs].
struct BTask {
    long long c_off;
    int c_buf, M, N, ldc;
    int t0, t1, accumulate, pad;
};
struct BTerm {
    long long a_off, b_off;
    int a_buf, b_buf;
    int a_rs, a_cs, b_rs, b_cs;
    int K, cidx;
};
// C[e] = sum_terms coef[cidx] * A[a_off + e], e < n.
struct CTask {
    long long c_off;
    int c_buf, n, t0, t1;
};
struct CTerm {
    long long a_off;
    int a_buf, cidx;
};
struct BufSet {
    double* p[kMaxBufs];
};

// diagonal of H_eff / N_eff for one packed block
struct DiagBlk {
    long long x_off;
    long long l_off0;  // offset of (row ro) diagonal start inside a left env block, per term
    int rows, cols, sigma, t0, t1;
    int pad;
};
struct DiagTerm {
    long long l_off;  // env block offset (per g) in the left env + ro*(ld+1)
    long long r_off;  // env block offset (per g) in the right env + co*(ld+1)
    int l_ld, r_ld;   // row length of the env blocks (diagonal stride ld+1)
    int cidx, pad;
};

// QR of one gathered sector matrix: pieces are row-major blocks of a packed
// site tensor; transposed pieces contribute their columns as rows.
struct QrTask {
    long long scratch_off;  // rows*cols doubles of scratch (column-major)
    long long r_off;        // cols*cols output (row-major)
    int rows, cols, p0, p1;
};
struct QrPiece {
    long long off;  // block offset in the site tensor
    int prow, pcol;  // stored block dims (row-major, ld = pcol)
    int transposed, row0;  // row offset in the gathered matrix
};

// Dense tile product: one 64x64 output tile C[r0:r0+64, c0:c0+64] of an
// M x N block = sum over segments of coef[cidx] * A[:, k0:k1] B[k0:k1, :].
// ta/tb = 1 read A (resp. B) transposed: A(r, k) = A[k*lda + r],
// B(k, c) = B[c*ldb + k].  mode 0 stores C[c_off + r*ldc + c]; mode 1 stores
// element (r, c) at C[c_off + map[pack_off + r*N + c]] when that index is
// >= 0 (scatter of a particle-number block into the packed (N, M) layout).
struct TTask {
    long long c_off, pack_off;
    int c_buf, ldc, M, N, r0, c0, s0, s1, mode, pad;
};
struct TSeg {
    long long a_off, b_off;
    int a_buf, b_buf, lda, ldb, ta, tb, k0, k1, cidx, pad;
};
constexpr int kTile = 64;  // the wide tile; 32 is the narrow one

// tile: 64 or 32 (the task grid of the list was built for that tile)
void tgemm(hipStream_t s, const TTask* tasks, int ntasks, const TSeg* segs, BufSet bufs, const double* coef,
           const int* map, int tile);
// the same products in split BF16 (hi + lo per operand, three matrix-core
// products, FP32 accumulation); relative error of order 1e-5
void tgemm_bf3(hipStream_t s, const TTask* tasks, int ntasks, const TSeg* segs, BufSet bufs, const double* coef,
               const int* map, int tile);
// dst[e] = map[e] >= 0 ? src[map[e]] : 0, e < n
void gather(hipStream_t s, const int* map, const double* src, double* dst, long long n);
// out[e] = sum_{g < G} part[g*stride + e] in ascending g, for two arrays at once
void gsum2(hipStream_t s, const double* pa, const double* pb, long long stride, int G, int n, double* outa,
           double* outb);

// Fused H_eff x / N_eff x (all quadrature points in one launch).  One
// work-group per (g, bra particle-number block i of the left bond, rows
// [r0, r0 + rows)), rows <= RC (a compile-time row count, 1..8).
//  phase A: the chunk's rows of every left-environment block L_g(c, i, .)
//           are staged in LDS; then every product T(c, s') = L_g(c, i) x[s']
//           (x block-sparse in M, so each T column runs over the ket rows of
//           one (N, M) sector) is formed one column per thread, all rows at
//           once, and kept in LDS column-major (RC rows per column);
//  per output sigma: V(c') = sum_terms coef * T for every right channel c'
//           of sigma (the W r mixing with coef_g; the identity channel gives
//           N_eff), then every allowed (N, M) output
//           y[sigma](r, b) = sum_c' sum_k V(c')(r, k) R_g(c')(b, k) is formed
//           by a group of lanes that split k and add their partial sums
//           with cross-lane shuffles (right environment read coalesced from
//           global memory).
// Per-g partials go to ypart/nypart[g*n + packed index].  All LDS offsets in
// the descriptors are in doubles and already include the RC factors.
struct H3Blk {
    int c0, c1;        // T columns (H3Col list)
    int l0, l1;        // left-environment blocks staged per chunk (H3LSrc list)
    int s0[4], s1[4];  // right-channel segments per output sigma (H3Seg list)
};
struct H3Col {
    int x_off, x_ld, K;  // x entries x_off + kk * x_ld, kk < K
    int l_lds, l_ld;     // staged L entry (rr, kk) at l_lds + rr * l_ld + kk
    int t_pos;           // T entry (rr) at t_pos + rr
    int pad0, pad1;
};
struct H3LSrc {
    int l_off, ld, lds, pad;  // rows of ld entries (within one g) -> LDS at lds + rr * ld
};
struct H3Seg {
    int r_off, K;  // right-environment block (within one g): row b at r_off + b * K
    int v_off;     // V entry (rr, k) at v_off + k * RC + rr
    int t0, t1;    // mixing terms
    int is_ny, pad0, pad1;
};
struct H3Term {
    int t_base, cidx;  // T block in LDS (entry (rr, k) at t_base + k * RC + rr), coefficient index
};
struct H3Piece {
    int rlo, rhi;         // chunk-relative rows of one left (N, M) sector
    int b0, nb;           // right-block rows of the output columns
    int out_off, out_ld;  // output (rr, b) at out_off + (rr - rlo) * out_ld + b
    int pad0, pad1;
};
struct H3Task {
    int g, blk, r0, rows;  // blk < 0: an empty task (padding)
    int p0[4], p1[4];      // output pieces per sigma
    int inst, pad0, pad1, pad2;  // instance of a batched launch (0 otherwise)
};
// Everything a task needs besides its own descriptor: the plan lists of its
// site, the environments, x and the outputs of one SP-MPS instance.  Lenv and
// Renv point to FP64 or FP32 data according to the launch.
struct H3Inst {
    const H3Blk* blks;
    const H3Col* cols;
    const H3LSrc* lsrc;
    const H3Seg* segs;
    const H3Term* terms;
    const H3Piece* pieces;
    const void* Lenv;
    const void* Renv;
    long long Lsz, Rsz;
    const double* x;
    const double* coef;
    double* ypart;
    double* nypart;
    long long n;
    int nc, pad;
    const int* gate;  // when set, tasks of this instance return at once while *gate == 0
};
constexpr int kH3MaxRC = 8;
constexpr int kH3Threads = 256;  // threads per work-group of the fused kernel
constexpr int kH3SlMax = 16;     // lanes per output column (at most)
// lds_elems: LDS elements (of the environment type) per work-group.  One
// instance (I, passed by value) or, with insts != nullptr, every task reads
// its instance from insts[task.inst] (many SP-MPS states in one launch; all
// tasks of a launch share RC).
void heff3(hipStream_t s, int RC, int lds_elems, const H3Task* tasks, int ntasks, const H3Inst& I,
           const H3Inst* insts = nullptr);
// the same contraction with FP32 environments, FP32 LDS tiles and FP32
// accumulation (x, the coefficients and the partial outputs stay FP64 in
// memory and are converted on the fly)
void heff3_f32(hipStream_t s, int RC, int lds_elems, const H3Task* tasks, int ntasks, const H3Inst& I,
               const H3Inst* insts = nullptr);
// out = float(in), n elements
void to_f32(hipStream_t s, const double* in, float* out, long long n);

void bgemm(hipStream_t s, const BTask* tasks, int ntasks, const BTerm* terms, BufSet bufs,
           const double* coef);
void combine(hipStream_t s, const CTask* tasks, int ntasks, const CTerm* terms, BufSet bufs,
             const double* coef);
// nsplit > 1: the (g, term) range of every block is cut into nsplit parts
// summed in a fixed order through part (nsplit x ntot doubles, ntot = the
// site size); nsplit = 1 sums straight into out
constexpr int kDiagSplitMax = 8;
void heff_diag(hipStream_t s, const DiagBlk* blks, int nblk, const DiagTerm* terms,
               const double* lenv, long long lsize, const double* renv, long long rsize,
               const double* coef, int ncoef, int G, double* out, int nsplit = 1, double* part = nullptr,
               long long ntot = 0);
// Per-sector positive-diagonal QR.  Tasks whose two rows x cols matrices
// fit kQrLdsMax doubles run in LDS (lds_doubles = the largest 2 rows cols
// of the list); otherwise they use the scratch buffer in global memory.
constexpr int kQrLdsMax = 12288;
void qr_sectors(hipStream_t s, const QrTask* tasks, int ntasks, const QrPiece* pieces, double* site,
                double* scratch, double* rout, int lds_doubles);

// Davidson vector kernels (n = vector length, ld = stride between vectors)
void normalize(hipStream_t s, const double* in, double* out, int n, double* norm_out);
// p[0..n) = value
void fill(hipStream_t s, double* p, long long n, double value);
void multidot(hipStream_t s, const double* A, long long ld, int m, const double* u, int n,
              double* out);
void basis_rotate(hipStream_t s, const double* A, long long ld, int m, const double* Q, int keep,
                  double* out, int n);
// Grid-parallel Davidson passes.  Each work-group owns kDavChunk consecutive
// elements and writes per-chunk partial sums; consumers add the partials of
// all chunks in ascending chunk order (deterministic).  m <= kDavMaxVec.
constexpr int kDavChunk = 256;
constexpr int kGramGroup = 16;  // dots per work-group of the Gram pass
constexpr int kDavMaxVec = 256;
__host__ __device__ inline int dav_chunks(int n) { return (n + kDavChunk - 1) / kDavChunk; }
// aq = (a_0 .. a_{m-1}, theta) (device or mapped host memory); x = V a,
// u = HV a - theta NV a, t = -u / floor(dh - theta dn); part_x[3 per chunk] =
// (x.x, u.u, x.(NV a)); part_c[m per chunk] = V_j . t
void dav_ritz(hipStream_t s, const double* V, const double* HV, const double* NV, long long ld, int m,
              const double* aq, const double* dh, const double* dn, int n, double floor_, double* x, double* t,
              double* part_x, double* part_c);
// c = sum of part_in over chunks; t -= V c; then part_out = V_j . t (mode 0)
// or part_out = t.t per chunk (mode 1)
void dav_cgs(hipStream_t s, const double* V, long long ld, int m_sub, int m_dot, const double* part_in,
             int nchunk, double* t, int n, double* part_out, int mode);
// vout = t / sqrt(sum part), tnorm = sqrt(sum part)
void dav_normalize(hipStream_t s, const double* part, int nchunk, const double* t, double* vout, int n,
                   double* tnorm);
// Gram rows of the new vector m, per chunk: V_j.HV_m (j<=m), V_j.NV_m (j<=m),
// HV_j.V_m (j<m), NV_j.V_m (j<m).  With t != nullptr, V_m = t / |t| where
// |t|^2 = the sum of the npn partials pn (|t| -> *tnorm) and H_eff t, N_eff t
// are scaled by 1/|t| (t needs ypart); with ypart != nullptr they are the
// sums over the G quadrature partials (stride gstride) and V_m (if t), HV_m
// and NV_m are stored, else they are read from HV_m, NV_m.
void dav_gram(hipStream_t s, double* V, double* HV, double* NV, long long ld, int m, int n, const double* t,
              const double* pn, int npn, double* tnorm, const double* ypart, const double* nypart, long long gstride,
              int G, double* part);

// One instance of the batched Davidson passes (many SP-MPS states advanced
// together): the arguments of the single-instance passes above, with the
// partial-sum buffers pc1 (Ritz -> first CGS), pc2 (first -> second CGS)
// and pn (second CGS -> Gram).  The Gram pass forms V_m from t when
// from_t != 0 (then ypart must be set).
struct DavInst {
    double* V;
    double* HV;
    double* NV;
    long long ld;
    const double* aq;  // (a_0 .. a_{m-1}, theta), mapped host memory
    const double* dh;
    const double* dn;
    double floor_;
    double* x;
    double* t;
    double* part_x;  // 3 per chunk (mapped host memory)
    double* pc1;
    double* pc2;
    double* pn;
    double* pg;     // Gram rows, 4m+2 per chunk (mapped host memory)
    double* tnorm;  // (mapped host memory)
    const double* ypart;
    const double* nypart;
    long long gstride;
    int G, m, n, active, from_t, mr;  // mr: subspace size of the Ritz pass
    int ext;  // the search space grows this iteration (CGS, H_eff and Gram passes run)
    // device-resident iteration (davdev.hip): the state the host-driven
    // solver keeps on the host, here in this record on the device
    int it, max_iter, max_sub, keep, nk, restart, last, converged, matvecs, err, S, nch;
    double tol, drop, theta, rnorm, pnorm;
    double* Ht;      // S x S projected H_eff (device)
    double* Nt;      // S x S projected N_eff (device)
    double* Qk;      // restart rotation, m x nk (device)
    double* aqd;     // where the subspace solve writes (a, theta); aq reads it
    double* status;  // 8 doubles per instance for the host (mapped memory)
};
void bdav_ritz(hipStream_t s, const DavInst* insts, int ninst, int max_n);
// mode 0, 1: the two CGS passes; mode 2: after a restart, the dots of the
// correction with the rotated basis (instances without a restart skip it)
void bdav_cgs(hipStream_t s, const DavInst* insts, int ninst, int max_n, int mode);
void bdav_gram(hipStream_t s, const DavInst* insts, int ninst, int max_n, int max_m);

// Device-resident Davidson iteration (davdev.hip).  Subspace sizes up to
// kDevSubMax - 1 vectors and restarts keeping up to kDevKeepMax.
constexpr int kDevSubMax = 48;
constexpr int kDevKeepMax = 16;
// LDS bytes of the subspace solve for m vectors
__host__ __device__ inline int dev_solve_lds(int m) { return (7 * m * m + 8 * m + 512) * 8; }
// after the first product and Gram pass of a local solve: Ht[0], Nt[0] from
// the Gram partials, m = 1, iteration counters reset
void bdav_start(hipStream_t s, DavInst* insts, int ninst);
// one subspace solve per active instance (one work-group each): lowest pair
// of the projected pencil by canonical orthogonalisation, the restart
// rotation when the space is full, the fields the passes of the iteration read
void bdav_solve(hipStream_t s, DavInst* insts, int ninst, int max_m);
// restart: V, HV, NV rotated in place by Qk (instances without a restart skip)
void bdav_rotate(hipStream_t s, const DavInst* insts, int ninst, int max_n);
// end of an iteration: residual norm, convergence, the new Gram row, status
void bdav_update(hipStream_t s, DavInst* insts, int ninst);
// one instance's subspace solve on host data (tests): H, N m x m row-major;
// need_all != 0 also forms the restart rotation of `keep` vectors into Qk
// (m x keep) and the rotated H, N (keep x keep, into H and N); returns the
// rank kept (0: the metric vanishes)
int dev_small_solve(int m, double* H, double* N, double drop, int need_all, int keep, double* theta, double* a,
                    double* Qk);

// Learned Davidson preconditioner (mlp.hip): two-layer perceptron on five
// features per element; packed weights W1 (H x 5) | b1 (H) | w2 (H) | b2
constexpr int kMlpIn = 5;
constexpr int kMlpMaxHidden = 256;
__host__ __device__ inline long long mlp_size(int H) { return (long long)H * (kMlpIn + 2) + 1; }
// *out = sum over chunks of part[q * stride + idx] (fixed order)
void sum_partials(hipStream_t s, const double* part, int nchunk, int stride, int idx, double* out);
// features of every element from t = -r / d' (rr = |r|^2, tt = |t|^2,
// theta device scalars); feat (n x 5 FP32) and sgn (n, sign(r_i)) if feat is not null;
// t replaced by the model's correction if w is not null
void mlp_apply(hipStream_t s, const float* w, int H, double* t, const double* dh, const double* dn,
               const double* theta, const double* rr, const double* tt, int n, double floor_, float* feat,
               float* sgn);
// *out = v . v (one work-group, fixed order)
void sumsq(hipStream_t s, const double* v, int n, double* out);
void mlp_forward(hipStream_t s, const float* w, int H, const float* F, long long n, float* y);
// targets of nrec recorded iterations (Ritz vectors ldx apart) against the
// unit vector xstar, n per iteration; Y holds sign(r) on entry
void mlp_targets(hipStream_t s, const double* X, long long ldx, int nrec, const double* xstar, int n, float* Y);
// per-work-group gradient partials (mlp_size(H) + 1 doubles each, the last
// the summed squared error) over rows row0 + q * stride, q < count
void mlp_grad(hipStream_t s, const float* w, int H, const float* F, const float* Y, long long row0, long long stride,
              long long count, double* gpart, int nparts);
void mlp_adam(hipStream_t s, float* w, double* m, double* v, int H, const double* gpart, int nparts, double scale,
              double lr, int step, double* loss_out);

}  // namespace spk
