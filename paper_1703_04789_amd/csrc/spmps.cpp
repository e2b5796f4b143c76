// Host runtime and C ABI of the SP-MPS hot path (one MI355X, FP64).
//
// Holds the block structure of an (N, 2M)-symmetric MPS, the quadrature of
// the spin projector (Eqs. [PSMM], [pmpo]), the rotated MPO W[k] r(beta_g)
// (Eq. [expSy]), the environments of every quadrature point, and for every
// site the precomputed task lists that the device kernels execute:
//
//   left  pass:  T_g = L_g[k-1] x            (env blocks (N_bra, N_ket) times
//                                             (N, M) blocks of the site)
//                V_g = sum W~_g T_g           (W~_g = W[k] r_g, the rotation
//                                             acting on the ket index)
//   y   = P_NM sum_g coef_g V_g R_g[k+1]^T    (H_eff x)
//   ny  = P_NM sum_g coef_g r_g T_g R^I_g^T   (N_eff x, identity channels)
//   L_g[k] = A^T V_g                          (left environment update)
//   right pass mirrors it for R_g[k].
//
// The environments are blocked by particle number only: the rotation
// exp(-i beta S_y) mixes M, so every (N_bra, N_ket) block is dense in M
// (the subduction described in Sec. 2.3).  Site tensors and H_eff vectors
// keep the (N, M) blocks.
#include "spmps.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <condition_variable>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

#include "host_linalg.h"
#include "kernels.h"
#include "mlp.h"

namespace {

thread_local std::string g_last_error;

struct SpError : std::runtime_error {
    int code;
    SpError(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define SP_REQUIRE(cond, msg)                                  \
    do {                                                       \
        if (!(cond)) throw SpError(SP_EINVAL, std::string(msg)); \
    } while (0)

inline void hip_check(hipError_t e, const char* what) {
    if (e != hipSuccess) {
        if (e == hipErrorOutOfMemory) throw SpError(SP_ENOMEM, std::string(what) + ": out of device memory");
        throw SpError(SP_EHIP, std::string(what) + ": " + hipGetErrorString(e));
    }
}
#define HIPCK(x) hip_check((x), #x)

constexpr int kSigmaN[4] = {0, 1, 1, 2};
constexpr int kSigma2M[4] = {0, -1, 1, 0};

template <class T>
struct DArr {  // owned device array
    T* p = nullptr;
    size_t n = 0;
    DArr() = default;
    DArr(const DArr&) = delete;
    DArr& operator=(const DArr&) = delete;
    DArr(DArr&& o) noexcept : p(o.p), n(o.n) {
        o.p = nullptr;
        o.n = 0;
    }
    DArr& operator=(DArr&& o) noexcept {
        if (this != &o) {
            release();
            p = o.p;
            n = o.n;
            o.p = nullptr;
            o.n = 0;
        }
        return *this;
    }
    ~DArr() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
    void alloc(size_t count) {
        release();
        n = count;
        if (count) HIPCK(hipMalloc(&p, count * sizeof(T)));
    }
    void upload(const std::vector<T>& v, hipStream_t s) {
        alloc(v.size());
        if (!v.empty()) HIPCK(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
    }
};

template <class T>
struct DRef {  // view of device memory owned elsewhere
    T* p = nullptr;
};

struct Sector {
    int n, m2, dim, off, nb, ro;
};
struct NBlock {
    int n, dim, off, s0, s1;
};
struct Bond {
    std::vector<Sector> sec;
    std::vector<NBlock> nb;
    int D = 0;
    std::map<std::pair<int, int>, int> sidx;
    std::map<int, int> nidx;
    int sector(int n, int m2) const {
        auto it = sidx.find({n, m2});
        return it == sidx.end() ? -1 : it->second;
    }
    int nblock(int n) const {
        auto it = nidx.find(n);
        return it == nidx.end() ? -1 : it->second;
    }
};
struct XBlk {
    int sa, s, sb, rows, cols;
    long long off;
};
struct SiteInfo {
    std::vector<XBlk> blk;
    long long size = 0, goff = 0;
    std::map<std::pair<int, int>, int> by_sa_s;  // (left sector, sigma) -> block
    int find(int sa, int s) const {
        auto it = by_sa_s.find({sa, s});
        return it == by_sa_s.end() ? -1 : it->second;
    }
};
// N-blocks of one site tensor (elements sharing both bond particle numbers)
// as groups of contiguous block ranges, and the group of every element; the
// host vectors stay alive as the sources of the uploads
struct NBlocks {
    int ng = 0;
    std::vector<int> gptr_h, rlen_h, gid_h;
    std::vector<long long> roff_h;
    DArr<int> gptr, rlen, gid;
    DArr<long long> roff;
    spk::ElemGroups groups() const { return spk::ElemGroups{ng, gptr.p, roff.p, rlen.p}; }
};
struct EnvBlk {
    int c, i, j, rows, cols;
    long long off;
};
struct EnvLayout {
    int nc = 0, nnb = 0;
    std::vector<EnvBlk> blk;
    std::vector<int> idx;  // c * nnb + i -> block
    long long size = 0;    // per quadrature point
    int find(int c, int i) const { return idx[size_t(c) * nnb + i]; }
};

// task list of one launch (host copy + device copy)
struct BList {
    std::vector<spk::BTask> tasks;
    std::vector<spk::BTerm> terms;
    DArr<spk::BTask> dtasks;
    DArr<spk::BTerm> dterms;
    double flops = 0.0;
    void add_task(int c_buf, long long c_off, int M, int N, int ldc, int accumulate = 0) {
        spk::BTask t{};
        t.c_off = c_off;
        t.c_buf = c_buf;
        t.M = M;
        t.N = N;
        t.ldc = ldc;
        t.t0 = t.t1 = int(terms.size());
        t.accumulate = accumulate;
        tasks.push_back(t);
    }
    void add_term(int a_buf, long long a_off, int a_rs, int a_cs, int b_buf, long long b_off, int b_rs,
                  int b_cs, int K, int cidx) {
        spk::BTerm m{};
        m.a_off = a_off;
        m.b_off = b_off;
        m.a_buf = a_buf;
        m.b_buf = b_buf;
        m.a_rs = a_rs;
        m.a_cs = a_cs;
        m.b_rs = b_rs;
        m.b_cs = b_cs;
        m.K = K;
        m.cidx = cidx;
        terms.push_back(m);
        tasks.back().t1 = int(terms.size());
        flops += 2.0 * tasks.back().M * tasks.back().N * K;
    }
    void upload(hipStream_t s) {
        dtasks.upload(tasks, s);
        dterms.upload(terms, s);
    }
    void launch(hipStream_t s, const spk::BufSet& b, const double* coef) const {
        spk::bgemm(s, dtasks.p, int(tasks.size()), dterms.p, b, coef);
    }
};
struct CList {
    std::vector<spk::CTask> tasks;
    std::vector<spk::CTerm> terms;
    DArr<spk::CTask> dtasks;
    DArr<spk::CTerm> dterms;
    double flops = 0.0;
    void add_task(int c_buf, long long c_off, int n) {
        spk::CTask t{};
        t.c_off = c_off;
        t.c_buf = c_buf;
        t.n = n;
        t.t0 = t.t1 = int(terms.size());
        tasks.push_back(t);
    }
    void add_term(int a_buf, long long a_off, int cidx) {
        spk::CTerm m{};
        m.a_off = a_off;
        m.a_buf = a_buf;
        m.cidx = cidx;
        terms.push_back(m);
        tasks.back().t1 = int(terms.size());
        flops += 2.0 * tasks.back().n;
    }
    void upload(hipStream_t s) {
        dtasks.upload(tasks, s);
        dterms.upload(terms, s);
    }
    void launch(hipStream_t s, const spk::BufSet& b, const double* coef) const {
        spk::combine(s, dtasks.p, int(tasks.size()), dterms.p, b, coef);
    }
};

struct TList {
    std::vector<spk::TTask> tasks;
    std::vector<spk::TSeg> segs;
    int tile = spk::kTile;  // output tile of every task (64 or 32)
    DArr<spk::TTask> dtasks;
    DArr<spk::TSeg> dsegs;
    void add_task(int c_buf, long long c_off, int ldc, int M, int N, int r0, int c0, int mode, long long pack_off) {
        spk::TTask t{};
        t.c_off = c_off;
        t.pack_off = pack_off;
        t.c_buf = c_buf;
        t.ldc = ldc;
        t.M = M;
        t.N = N;
        t.r0 = r0;
        t.c0 = c0;
        t.s0 = t.s1 = int(segs.size());
        t.mode = mode;
        tasks.push_back(t);
    }
    void add_seg(int a_buf, long long a_off, int lda, int ta, int b_buf, long long b_off, int ldb, int tb, int k0,
                 int k1, int cidx) {
        spk::TSeg g{};
        g.a_off = a_off;
        g.b_off = b_off;
        g.a_buf = a_buf;
        g.b_buf = b_buf;
        g.lda = lda;
        g.ldb = ldb;
        g.ta = ta;
        g.tb = tb;
        g.k0 = k0;
        g.k1 = k1;
        g.cidx = cidx;
        segs.push_back(g);
        tasks.back().s1 = int(segs.size());
    }
    void upload(hipStream_t s) {
        dtasks.upload(tasks, s);
        dsegs.upload(segs, s);
    }
    void launch(hipStream_t s, const spk::BufSet& b, const double* coef, const int* map, bool bf3 = false) const {
        if (bf3) spk::tgemm_bf3(s, dtasks.p, int(tasks.size()), dsegs.p, b, coef, map, tile);
        else spk::tgemm(s, dtasks.p, int(tasks.size()), dsegs.p, b, coef, map, tile);
    }
};

// buffer slots of a launch; B_BRA is the site tensor on the bra side of the
// plain-path environment updates (the same as B_X except for the mixed
// environments of an orthogonality constraint)
enum Buf { B_ENVL = 0, B_ENVR = 1, B_X = 2, B_T = 3, B_V = 4, B_Y = 5, B_NY = 6, B_OUT = 7, B_BRA = 8, B_LT = 9 };

struct SitePlan {
    // coefficient table [G][nc]
    int nW = 0, nc = 0;
    std::vector<std::array<int, 4>> went;  // (a, b, s, u) of the rotated MPO pattern
    std::vector<double> coef_h;
    DArr<double> coef;
    int c_wt(int e) const { return e; }
    int c_cwt(int e) const { return nW + e; }
    int c_g() const { return 2 * nW; }
    int c_gr(int s, int u) const { return 2 * nW + 1 + 4 * s + u; }
    int c_one() const { return 2 * nW + 17; }
    // unrotated MPO entries W[a, b, s, s'] (block-product path) and the
    // rotation r_g(s, u) itself
    int nWr = 0;
    int c_wr(int e) const { return 2 * nW + 18 + e; }
    int c_r(int s, int u) const { return 2 * nW + 18 + nWr + 4 * s + u; }
    // scratch sizes per quadrature point
    long long Tsize = 0, Vsize = 0, Zsize = 0, Ztsize = 0;
    BList p1, yout, envl_out, p1r, envr_out;
    CList mixl, mixr;
    double heff_flops = 0.0;
    // diagonal
    std::vector<spk::DiagBlk> dblk_h, dblk_n;
    std::vector<spk::DiagTerm> dterm_h, dterm_n;
    DArr<spk::DiagBlk> ddblk_h, ddblk_n;
    DArr<spk::DiagTerm> ddterm_h, ddterm_n;
    // gauge moves
    std::vector<spk::QrTask> qr_tasks, lq_tasks;
    std::vector<spk::QrPiece> qr_pieces, lq_pieces;
    DArr<spk::QrTask> dqr_tasks, dlq_tasks;
    DArr<spk::QrPiece> dqr_pieces, dlq_pieces;
    long long qr_scratch = 0, lq_scratch = 0, qr_rsize = 0, lq_rsize = 0;
    int qr_lds = 0, lq_lds = 0;  // largest 2 * rows * cols of a task (doubles)
    std::vector<long long> qr_roff;  // per right sector of bond k
    std::vector<long long> lq_roff;  // per left sector of bond k-1
    BList absorb_right;  // R of site k into site k+1
    BList absorb_left;   // L of site k into site k-1
    // tiled path: dense particle-number layout of the site and its tile lists
    long long Xd_size = 0;
    std::vector<int> xmap_h;  // dense element -> packed index or -1
    DArr<int> xmap;
    TList t_left, t_right, t_envl, t_zr, t_envr;
    // H_eff x of the tiled block products from the pre-mixed left
    // environment Lt(sigma, c', sigma', i) = sum_c W~_g[c, c', sigma, sigma'] L_g(c, i)
    // (premix, once per local problem), V = sum_sigma' Lt Xd(sigma') (t_leftv)
    // and the identity-channel products T(0, i, sigma') for N_eff (t_left0)
    CList premix, xrmix;
    TList t_leftv, t_left0;
    long long LTsize = 0;
    int tr_split = 1;  // channel chunks of the tiled right product (partials: tr_split * G)
    // fused H_eff x
    int h_rows = 0;         // rows per task (RC); 0: no fused plan
    int h_lds = 0;          // dynamic LDS per work-group (doubles)
    std::vector<spk::H3Task> h_tasks;
    std::vector<spk::H3Blk> h_blks;
    std::vector<spk::H3Col> h_cols;
    std::vector<spk::H3LSrc> h_lsrc;
    std::vector<spk::H3Seg> h_segs;
    std::vector<spk::H3Term> h_terms;
    std::vector<spk::H3Piece> h_pieces;
    DArr<spk::H3Task> dh_tasks;
    DArr<spk::H3Blk> dh_blks;
    DArr<spk::H3Col> dh_cols;
    DArr<spk::H3LSrc> dh_lsrc;
    DArr<spk::H3Seg> dh_segs;
    DArr<spk::H3Term> dh_terms;
    DArr<spk::H3Piece> dh_pieces;
};

}  // namespace

struct sp_handle {
    hipStream_t stream = nullptr;
    int device = 0;
    int L = 0, N = 0, twoS = 0, twoM = 0, G = 0;
    bool inexact = false;
    std::vector<double> qx, qw, qc, qs, qcoef;
    std::vector<int> w;                    // MPO bond dimensions
    std::vector<std::vector<int>> dn;      // per bond, per channel: particle change
    std::vector<std::vector<double>> W;    // per site (index k-1)
    std::vector<Bond> bonds;
    std::vector<SiteInfo> sites;           // index k-1
    std::vector<EnvLayout> env;            // per bond
    // Environments per bond, G * size each.  An interior bond keeps one
    // buffer for both sides: a sweep builds L[k] only after its last use of
    // R[k] and the other way round, so at most one of the two is valid at a
    // time (Lvalid/Rvalid); the boundary bonds 0 and L keep both.
    std::vector<DArr<double>> envmem;
    std::vector<DArr<float>> envmem32;     // FP32 copies (reduced precisions)
    std::vector<DRef<double>> envL, envR;
    std::vector<DRef<float>> envL32, envR32;
    std::vector<int> tab_nsec, tab_n, tab_2m, tab_dim;  // the block table as given
    int precision = SP_FP64;
    std::vector<char> Lvalid, Rvalid;
    DArr<double> mps;
    long long mps_size = 0, max_site = 0;
    std::vector<SitePlan> plan;            // index k-1
    int path = SP_PATH_TILED;
    DArr<double> T, V, qr_scratch, qr_r, tmp_site, Xd, ypart, nypart;
    // pre-mixed left environment of one site (tiled block products); valid
    // for site lt_site while the generation of L[lt_site - 1] is lt_gen
    DArr<double> LT;
    long long LT_cap = 0;
    DArr<double> diag_part;  // partial sums of the split diagonal (kDiagSplitMax x max_site)
    std::vector<long long> Lgen;
    int lt_site = -1;
    long long lt_gen = -1;
    long long Xd_cap = 0;
    int tr_split_max = 1;  // partial slots per quadrature point (tiled lists)
    long long T_cap = 0, V_cap = 0, qr_scratch_cap = 0, qr_r_cap = 0;
    int center = 1;
    // Davidson workspace
    int dav_sub = 0;
    long long ld = 0;
    DArr<double> dV, dHV, dNV, dRot, dx, dt, ddh, ddn, dpart, dsmall, dy, dny;
    DArr<double> dHt, dNt;  // projected H_eff, N_eff of the device-resident solve ((dav_sub+1)^2)
    double* pin = nullptr;  // pinned host staging (device -> host)
    double* pin_dev = nullptr;  // the same memory as kernels address it
    size_t pin_n = 0;
    double* pin_up = nullptr;  // pinned host staging (host -> device)
    double* pin_up_dev = nullptr;
    size_t pin_up_n = 0;
    // orthogonality constraints (excited states): one identity-MPO handle per
    // lower state whose environments are mixed (bra: this state, ket: the
    // lower state), the orthonormalised constraint vectors of the current
    // site (cld apart) and their projection partials
    std::vector<std::unique_ptr<sp_handle>> cons;
    DArr<double> conB, conPart;
    long long cld = 0;
    int con_active = 0;
    double* con_pin = nullptr;  // mapped: norm partials read by the host
    double* con_pin_dev = nullptr;
    // learned preconditioner: the model used for corrections and the one
    // collecting training pairs (either may be null), Ritz vectors of the
    // current solve for the targets, device scalars
    sp_mlp* mlp_use = nullptr;
    sp_mlp* mlp_rec = nullptr;
    DArr<double> xrec, mlp_scal, mlp_grms, mlp_tscal;
    std::vector<NBlocks> nblocks;  // per site (index k-1), built on first use
    ~sp_handle() {
        if (pin) (void)hipHostFree(pin);
        if (pin_up) (void)hipHostFree(pin_up);
        if (con_pin) (void)hipHostFree(con_pin);
    }
};

// reduced-precision local solves (SP_FP32 or SP_BF16X3): FP32 fused products,
// FP64 Rayleigh quotient per site step, looser canonical orthogonalisation
inline bool reduced(const sp_handle* h) { return h->precision != SP_FP64; }
// canonical orthogonalisation of the projected metric: eigenvalues below
// drop x the largest are discarded; the threshold sits above the relative
// noise of the products (FP64 ~1e-15, FP32 ~1e-7, split BF16 ~5e-6) by two
// orders, one order for split BF16 (1e-3 there slowed the descent of the
// sweeps by discarding directions of small spin-S weight)
inline double metric_drop(const sp_handle* h) {
    return h->precision == SP_FP64 ? 1e-10 : (h->precision == SP_FP32 ? 1e-5 : 1e-4);
}

// a learned Davidson preconditioner and its training pairs (one device)
struct sp_mlp {
    int hidden = 0, device = 0;
    DArr<float> w;       // packed weights
    DArr<double> m, v;   // Adam moments
    int step = 0;
    long long cap = 0, rows = 0;
    DArr<float> F, Y;    // recorded pairs: cap x 5 features, cap targets
    DArr<double> gpart, scal;
    int nparts = 0;
    int scope = SP_MLP_VECTOR;  // rms over the site vector or per N-block
};

namespace {

// ---------------------------------------------------------------------------
// setup

void build_bonds(sp_handle* h, const sp_block_table* bt) {
    const int L = h->L;
    h->bonds.assign(L + 1, Bond{});
    long long pos = 0;
    for (int k = 0; k <= L; ++k) {
        Bond& b = h->bonds[k];
        const int ns = bt->nsec[k];
        SP_REQUIRE(ns >= 1, "every bond needs at least one sector");
        int off = 0;
        for (int i = 0; i < ns; ++i, ++pos) {
            Sector s{bt->sec_n[pos], bt->sec_2m[pos], bt->sec_dim[pos], off, -1, 0};
            SP_REQUIRE(s.dim >= 1, "sector dimensions must be positive");
            if (i > 0) {
                const Sector& p = b.sec.back();
                SP_REQUIRE(p.n < s.n || (p.n == s.n && p.m2 < s.m2), "sectors must be sorted by (N, 2M)");
            }
            off += s.dim;
            b.sec.push_back(s);
        }
        b.D = off;
        for (int i = 0; i < ns; ++i) {
            Sector& s = b.sec[i];
            if (b.nb.empty() || b.nb.back().n != s.n) b.nb.push_back(NBlock{s.n, 0, s.off, i, i});
            NBlock& nb = b.nb.back();
            s.nb = int(b.nb.size()) - 1;
            s.ro = nb.dim;
            nb.dim += s.dim;
            nb.s1 = i + 1;
            b.sidx[{s.n, s.m2}] = i;
        }
        for (int i = 0; i < int(b.nb.size()); ++i) b.nidx[b.nb[i].n] = i;
    }
    SP_REQUIRE(h->bonds[0].sec.size() == 1 && h->bonds[0].sec[0].n == 0 && h->bonds[0].sec[0].m2 == 0 &&
                   h->bonds[0].sec[0].dim == 1,
               "bond 0 must be the single sector (0, 0) of dimension 1");
    SP_REQUIRE(h->bonds[L].sec.size() == 1 && h->bonds[L].sec[0].n == h->N &&
                   h->bonds[L].sec[0].m2 == h->twoM && h->bonds[L].sec[0].dim == 1,
               "bond L must be the single sector (N, 2M) of dimension 1");
    // reachability: a sector cannot hold more states than its neighbours reach
    for (int k = 1; k < L; ++k) {
        for (const Sector& s : h->bonds[k].sec) {
            int left = 0, right = 0;
            for (int q = 0; q < 4; ++q) {
                int a = h->bonds[k - 1].sector(s.n - kSigmaN[q], s.m2 - kSigma2M[q]);
                if (a >= 0) left += h->bonds[k - 1].sec[a].dim;
                int c = h->bonds[k + 1].sector(s.n + kSigmaN[q], s.m2 + kSigma2M[q]);
                if (c >= 0) right += h->bonds[k + 1].sec[c].dim;
            }
            SP_REQUIRE(s.dim <= left && s.dim <= right,
                       "block table: a sector is wider than its support in a neighbouring bond");
        }
    }
    // site blocks in canonical order
    h->sites.assign(L, SiteInfo{});
    long long goff = 0;
    for (int k = 1; k <= L; ++k) {
        SiteInfo& si = h->sites[k - 1];
        si.goff = goff;
        const Bond& bl = h->bonds[k - 1];
        const Bond& br = h->bonds[k];
        long long off = 0;
        for (int a = 0; a < int(bl.sec.size()); ++a) {
            for (int q = 0; q < 4; ++q) {
                const int b = br.sector(bl.sec[a].n + kSigmaN[q], bl.sec[a].m2 + kSigma2M[q]);
                if (b < 0) continue;
                XBlk x{a, q, b, bl.sec[a].dim, br.sec[b].dim, off};
                si.by_sa_s[{a, q}] = int(si.blk.size());
                si.blk.push_back(x);
                off += (long long)x.rows * x.cols;
            }
        }
        si.size = off;
        SP_REQUIRE(off > 0, "a site has no allowed block");
        goff += off;
        h->max_site = std::max(h->max_site, off);
    }
    h->mps_size = goff;
}

void build_mpo(sp_handle* h, const sp_mpo* Wm) {
    const int L = h->L;
    h->w.assign(Wm->w, Wm->w + L + 1);
    SP_REQUIRE(h->w[0] == 1 && h->w[L] == 1, "MPO: w[0] and w[L] must be 1");
    for (int k = 0; k <= L; ++k) SP_REQUIRE(h->w[k] >= 1 && h->w[k] <= 4096, "MPO: bad bond dimension");
    h->W.assign(L, {});
    long long pos = 0;
    for (int k = 1; k <= L; ++k) {
        const long long n = (long long)h->w[k - 1] * h->w[k] * 16;
        h->W[k - 1].assign(Wm->data + pos, Wm->data + pos + n);
        pos += n;
    }
    // particle change of every channel, propagated from bond 0
    h->dn.assign(L + 1, {});
    h->dn[0] = {0};
    for (int k = 1; k <= L; ++k) {
        const int wl = h->w[k - 1], wr = h->w[k];
        std::vector<int> d(wr, INT32_MIN);
        const auto& Wk = h->W[k - 1];
        for (int a = 0; a < wl; ++a)
            for (int b = 0; b < wr; ++b)
                for (int s = 0; s < 4; ++s)
                    for (int t = 0; t < 4; ++t) {
                        const double v = Wk[((size_t(a) * wr + b) * 4 + s) * 4 + t];
                        if (v == 0.0) continue;
                        const int val = h->dn[k - 1][a] + kSigmaN[s] - kSigmaN[t];
                        if (d[b] == INT32_MIN) d[b] = val;
                        SP_REQUIRE(d[b] == val, "MPO: an operator entry changes the particle number inconsistently");
                    }
        for (int b = 0; b < wr; ++b)
            if (d[b] == INT32_MIN) d[b] = 0;  // channel never reached: unused
        h->dn[k] = d;
    }
    SP_REQUIRE(h->dn[L][0] == 0, "MPO: the full operator must conserve the particle number");
    // identity channels: column 0 (k < L) and the last row (k > 1)
    auto op = [&](int k, int a, int b, int s, int t) {
        return h->W[k - 1][((size_t(a) * h->w[k] + b) * 4 + s) * 4 + t];
    };
    for (int k = 1; k <= L; ++k) {
        const int wl = h->w[k - 1], wr = h->w[k];
        if (k < L)
            for (int a = 0; a < wl; ++a)
                for (int s = 0; s < 4; ++s)
                    for (int t = 0; t < 4; ++t)
                        SP_REQUIRE(op(k, a, 0, s, t) == ((a == 0 && s == t) ? 1.0 : 0.0),
                                   "MPO: channel 0 must be the left identity string");
        if (k > 1)
            for (int b = 0; b < wr; ++b)
                for (int s = 0; s < 4; ++s)
                    for (int t = 0; t < 4; ++t)
                        SP_REQUIRE(op(k, wl - 1, b, s, t) == ((b == wr - 1 && s == t) ? 1.0 : 0.0),
                                   "MPO: the last channel must be the right identity string");
    }
}

void build_env_layouts(sp_handle* h) {
    const int L = h->L;
    h->env.assign(L + 1, EnvLayout{});
    for (int k = 0; k <= L; ++k) {
        EnvLayout& e = h->env[k];
        const Bond& b = h->bonds[k];
        e.nc = h->w[k];
        e.nnb = int(b.nb.size());
        e.idx.assign(size_t(e.nc) * e.nnb, -1);
        long long off = 0;
        for (int c = 0; c < e.nc; ++c)
            for (int i = 0; i < e.nnb; ++i) {
                const int j = b.nblock(b.nb[i].n - h->dn[k][c]);
                if (j < 0) continue;
                e.idx[size_t(c) * e.nnb + i] = int(e.blk.size());
                e.blk.push_back(EnvBlk{c, i, j, b.nb[i].dim, b.nb[j].dim, off});
                off += (long long)b.nb[i].dim * b.nb[j].dim;
            }
        e.size = off;
    }
    SP_REQUIRE(h->env[0].size == 1 && h->env[L].size == 1, "boundary environments must be 1x1");
    h->Lvalid.assign(L + 1, 0);
    h->Rvalid.assign(L + 1, 0);
    h->Lgen.assign(L + 1, 0);
}

// Interior bonds 1..L-1 hold one buffer shared by L[k] and R[k]; bonds 0
// and L hold two (the boundary ones and the full contractions).
template <class T>
void alloc_env_set(const sp_handle* h, std::vector<DArr<T>>& mem, std::vector<DRef<T>>& l,
                   std::vector<DRef<T>>& r) {
    const int L = h->L;
    mem.clear();
    mem.resize(L + 3);
    l.assign(L + 1, {});
    r.assign(L + 1, {});
    for (int k = 0; k <= L; ++k) {
        mem[k].alloc(size_t(h->G) * h->env[k].size);
        l[k].p = r[k].p = mem[k].p;
    }
    mem[L + 1].alloc(size_t(h->G) * h->env[0].size);
    mem[L + 2].alloc(size_t(h->G) * h->env[L].size);
    r[0].p = mem[L + 1].p;
    r[L].p = mem[L + 2].p;
}

// an interior bond's two environments share storage
inline bool env_shared(const sp_handle* h, int k) { return k > 0 && k < h->L; }

void alloc_envs(sp_handle* h) {
    const int L = h->L;
    alloc_env_set(h, h->envmem, h->envL, h->envR);
    // boundary environments: one 1x1 block equal to 1 for every g
    std::vector<double> ones(h->G, 1.0);
    HIPCK(hipMemcpyAsync(h->envL[0].p, ones.data(), h->G * sizeof(double), hipMemcpyHostToDevice, h->stream));
    HIPCK(hipMemcpyAsync(h->envR[L].p, ones.data(), h->G * sizeof(double), hipMemcpyHostToDevice, h->stream));
    if (reduced(h)) {
        alloc_env_set(h, h->envmem32, h->envL32, h->envR32);
        spk::to_f32(h->stream, h->envL[0].p, h->envL32[0].p, h->G);
        spk::to_f32(h->stream, h->envR[L].p, h->envR32[L].p, h->G);
    }
    HIPCK(hipStreamSynchronize(h->stream));
    h->Lvalid[0] = 1;
    h->Rvalid[L] = 1;
    ++h->Lgen[0];
}

// rotated MPO W[k] r(beta_g): pattern and values
bool rot_nonzero(int t, int u) { return (t == u) || ((t == 1 || t == 2) && (u == 1 || u == 2)); }
double rot_value(int t, int u, double c, double s) {
    if (t == 0 || t == 3) return t == u ? 1.0 : 0.0;
    if (u == 0 || u == 3) return 0.0;
    if (t == u) return c;
    return (t == 1) ? s : -s;  // r[1][2] = s, r[2][1] = -s  (Eq. [expSy])
}

void build_plan(sp_handle* h, int k) {
    SitePlan& P = h->plan[k - 1];
    const int G = h->G;
    const Bond& bl = h->bonds[k - 1];
    const Bond& br = h->bonds[k];
    const SiteInfo& si = h->sites[k - 1];
    const EnvLayout& el = h->env[k - 1];  // L env at bond k-1 (also output of the right pass)
    const EnvLayout& er = h->env[k];      // R env at bond k (also output of the left pass)
    const int wl = h->w[k - 1], wr = h->w[k];
    const auto& Wk = h->W[k - 1];
    // ---- rotated MPO pattern and coefficient table
    for (int a = 0; a < wl; ++a)
        for (int b = 0; b < wr; ++b) {
            const double* op = &Wk[(size_t(a) * wr + b) * 16];
            bool any = false;
            for (int e = 0; e < 16; ++e) any = any || op[e] != 0.0;
            if (!any) continue;
            for (int s = 0; s < 4; ++s)
                for (int u = 0; u < 4; ++u) {
                    bool nz = false;
                    for (int t = 0; t < 4; ++t)
                        if (op[s * 4 + t] != 0.0 && rot_nonzero(t, u)) nz = true;
                    if (nz) P.went.push_back({a, b, s, u});
                }
        }
    P.nW = int(P.went.size());
    // the rotated-MPO entries by (sigma, right channel) as (left channel,
    // sigma', entry), by (sigma, left channel) as (right channel, sigma',
    // entry), and the diagonal ones (sigma' = sigma) by sigma as (left
    // channel, right channel, entry), each in ascending order (the order of
    // the entry list)
    std::vector<std::vector<std::array<int, 3>>> byL(size_t(4) * wr), byR(size_t(4) * wl), byD(4);
    for (int e = 0; e < P.nW; ++e) {
        const auto& q = P.went[e];
        byL[size_t(q[2]) * wr + q[1]].push_back({q[0], q[3], e});
        byR[size_t(q[2]) * wl + q[0]].push_back({q[1], q[3], e});
        if (q[2] == q[3]) byD[q[2]].push_back({q[0], q[1], e});
    }
    // the unrotated entries W[a, b, s, s'] of the blocks in the pattern, by
    // (s, b) as (a, s', entry) in ascending order: the block products
    // pre-mix the left environment with them and apply the rotation to the
    // site vector instead (Eq. [expSy] acts on s' only)
    std::vector<std::vector<std::array<int, 3>>> byWr(size_t(4) * wr);
    std::vector<double> wr_val;
    {
        std::set<std::pair<int, int>> blocks;
        for (const auto& q : P.went) blocks.insert({q[0], q[1]});
        for (const auto& ab : blocks) {
            const double* op = &Wk[(size_t(ab.first) * wr + ab.second) * 16];
            for (int s2 = 0; s2 < 4; ++s2)
                for (int v = 0; v < 4; ++v)
                    if (op[s2 * 4 + v] != 0.0) {
                        byWr[size_t(s2) * wr + ab.second].push_back({ab.first, v, int(wr_val.size())});
                        wr_val.push_back(op[s2 * 4 + v]);
                    }
        }
    }
    P.nWr = int(wr_val.size());
    P.nc = 2 * P.nW + 18 + P.nWr + 16;
    P.coef_h.assign(size_t(G) * P.nc, 0.0);
    for (int g = 0; g < G; ++g) {
        double* cf = &P.coef_h[size_t(g) * P.nc];
        for (int e = 0; e < P.nW; ++e) {
            const auto& q = P.went[e];
            double v = 0.0;
            for (int t = 0; t < 4; ++t)
                v += Wk[((size_t(q[0]) * wr + q[1]) * 4 + q[2]) * 4 + t] * rot_value(t, q[3], h->qc[g], h->qs[g]);
            cf[P.c_wt(e)] = v;
            cf[P.c_cwt(e)] = h->qcoef[g] * v;
        }
        cf[P.c_g()] = h->qcoef[g];
        for (int s = 0; s < 4; ++s)
            for (int u = 0; u < 4; ++u) cf[P.c_gr(s, u)] = h->qcoef[g] * rot_value(s, u, h->qc[g], h->qs[g]);
        cf[P.c_one()] = 1.0;
        for (int e = 0; e < P.nWr; ++e) cf[P.c_wr(e)] = wr_val[e];
        for (int s = 0; s < 4; ++s)
            for (int u = 0; u < 4; ++u) cf[P.c_r(s, u)] = rot_value(s, u, h->qc[g], h->qs[g]);
    }
    const long long Lsz = el.size, Rsz = er.size;

    // ---- left pass, phase 1: T(eb, sigma') = L(eb) X(j, sigma', jb)
    std::vector<long long> Toff(el.blk.size() * 4, -1);
    std::vector<int> Tcols(el.blk.size() * 4, 0);
    long long toff = 0;
    for (size_t e = 0; e < el.blk.size(); ++e)
        for (int q = 0; q < 4; ++q) {
            const EnvBlk& eb = el.blk[e];
            const int jb = br.nblock(bl.nb[eb.j].n + kSigmaN[q]);
            if (jb < 0) continue;
            Toff[e * 4 + q] = toff;
            Tcols[e * 4 + q] = br.nb[jb].dim;
            toff += (long long)eb.rows * br.nb[jb].dim;
        }
    P.Tsize = toff;
    for (int g = 0; g < G; ++g) {
        for (size_t e = 0; e < el.blk.size(); ++e)
            for (int q = 0; q < 4; ++q) {
                if (Toff[e * 4 + q] < 0) continue;
                const EnvBlk& eb = el.blk[e];
                const int jb = br.nblock(bl.nb[eb.j].n + kSigmaN[q]);
                const NBlock& NB = br.nb[jb];
                for (int sb = NB.s0; sb < NB.s1; ++sb) {
                    const Sector& SB = br.sec[sb];
                    const long long coff = g * P.Tsize + Toff[e * 4 + q] + SB.ro;
                    P.p1.add_task(B_T, coff, eb.rows, SB.dim, NB.dim);
                    const int sa = bl.sector(SB.n - kSigmaN[q], SB.m2 - kSigma2M[q]);
                    if (sa < 0) continue;
                    const int xb = si.find(sa, q);
                    if (xb < 0) continue;
                    const XBlk& X = si.blk[xb];
                    P.p1.add_term(B_ENVL, g * Lsz + eb.off + bl.sec[sa].ro, eb.cols, 1, B_X, X.off, X.cols, 1,
                                  X.rows, g * P.nc + P.c_one());
                }
            }
    }
    // ---- left pass, mixing: V(sigma, c', i) = sum W~[c, c', sigma, sigma'] T(eb(c, i), sigma')
    std::map<std::array<int, 3>, long long> Voff;  // (sigma, c', i) -> offset
    std::map<std::array<int, 3>, int> Vcols;
    long long voff = 0;
    struct VTerm { int sig, cp, i; long long toffv; int widx, e, q; };
    std::vector<VTerm> vterms;
    for (int sig = 0; sig < 4; ++sig)
        for (int cp = 0; cp < wr; ++cp)
            for (int i = 0; i < int(bl.nb.size()); ++i) {
                const int nbk = br.nblock(bl.nb[i].n + kSigmaN[sig]);
                if (nbk < 0) continue;
                const int nbp = br.nblock(br.nb[nbk].n - h->dn[k][cp]);
                if (nbp < 0) continue;
                bool any = false;
                for (const auto& ent : byL[size_t(sig) * wr + cp]) {
                    const int c = ent[0], q = ent[1];
                    const int e = el.find(c, i);
                    if (e < 0 || Toff[size_t(e) * 4 + q] < 0) continue;
                    const int jb = br.nblock(bl.nb[el.blk[e].j].n + kSigmaN[q]);
                    SP_REQUIRE(jb == nbp, "internal: inconsistent particle numbers in the MPO mixing");
                    vterms.push_back({sig, cp, i, Toff[size_t(e) * 4 + q], ent[2], e, q});
                    any = true;
                }
                if (!any) continue;
                Voff[{sig, cp, i}] = voff;
                Vcols[{sig, cp, i}] = br.nb[nbp].dim;
                voff += (long long)bl.nb[i].dim * br.nb[nbp].dim;
            }
    P.Vsize = voff;
    for (int g = 0; g < G; ++g) {
        size_t t = 0;
        while (t < vterms.size()) {
            const VTerm& v0 = vterms[t];
            const long long vo = Voff[{v0.sig, v0.cp, v0.i}];
            const int n = bl.nb[v0.i].dim * Vcols[{v0.sig, v0.cp, v0.i}];
            P.mixl.add_task(B_V, g * P.Vsize + vo, n);
            while (t < vterms.size() && vterms[t].sig == v0.sig && vterms[t].cp == v0.cp && vterms[t].i == v0.i) {
                P.mixl.add_term(B_T, g * P.Tsize + vterms[t].toffv, g * P.nc + P.c_wt(vterms[t].widx));
                ++t;
            }
        }
    }
    // ---- y = sum_g coef_g V R^T  and  ny = sum_g coef_g r T0 R_last^T, per (N, M) block
    const int lastR = wr - 1;
    for (const XBlk& X : si.blk) {
        const Sector& SA = bl.sec[X.sa];
        const Sector& SB = br.sec[X.sb];
        P.yout.add_task(B_Y, X.off, X.rows, X.cols, X.cols);
        for (int g = 0; g < G; ++g)
            for (int cp = 0; cp < wr; ++cp) {
                auto it = Voff.find({X.s, cp, SA.nb});
                if (it == Voff.end()) continue;
                const int re = er.find(cp, SB.nb);
                if (re < 0) continue;
                const EnvBlk& RB = er.blk[re];
                const int K = Vcols[{X.s, cp, SA.nb}];
                SP_REQUIRE(K == RB.cols, "internal: V and R blocks disagree");
                P.yout.add_term(B_V, g * P.Vsize + it->second + (long long)SA.ro * K, K, 1, B_ENVR,
                                g * Rsz + RB.off + (long long)SB.ro * RB.cols, 1, RB.cols, K, g * P.nc + P.c_g());
            }
    }
    for (const XBlk& X : si.blk) {
        const Sector& SA = bl.sec[X.sa];
        const Sector& SB = br.sec[X.sb];
        P.yout.add_task(B_NY, X.off, X.rows, X.cols, X.cols);
        const int e0 = el.find(0, SA.nb);
        const int re = er.find(lastR, SB.nb);
        if (e0 < 0 || re < 0) continue;
        SP_REQUIRE(el.blk[e0].j == SA.nb && er.blk[re].j == SB.nb, "internal: identity channels must conserve N");
        for (int g = 0; g < G; ++g)
            for (int q = 0; q < 4; ++q) {
                if (!rot_nonzero(X.s, q)) continue;
                const long long to = Toff[size_t(e0) * 4 + q];
                if (to < 0) continue;
                const int K = Tcols[size_t(e0) * 4 + q];
                const EnvBlk& RB = er.blk[re];
                SP_REQUIRE(K == RB.cols, "internal: T and R identity blocks disagree");
                P.yout.add_term(B_T, g * P.Tsize + to + (long long)SA.ro * K, K, 1, B_ENVR,
                                g * Rsz + RB.off + (long long)SB.ro * RB.cols, 1, RB.cols, K,
                                g * P.nc + P.c_gr(X.s, q));
            }
    }
    // ---- left environment update: L[k](c', b, b') rows of sector s_b = sum_sigma A^T V
    for (int g = 0; g < G; ++g)
        for (const EnvBlk& OB : er.blk) {
            const NBlock& NB = br.nb[OB.i];
            for (int sb = NB.s0; sb < NB.s1; ++sb) {
                const Sector& SB = br.sec[sb];
                P.envl_out.add_task(B_OUT, g * Rsz + OB.off + (long long)SB.ro * OB.cols, SB.dim, OB.cols, OB.cols);
                for (int q = 0; q < 4; ++q) {
                    const int sa = bl.sector(SB.n - kSigmaN[q], SB.m2 - kSigma2M[q]);
                    if (sa < 0) continue;
                    const int xb = si.find(sa, q);
                    if (xb < 0) continue;
                    const XBlk& X = si.blk[xb];
                    auto it = Voff.find({q, OB.c, bl.sec[sa].nb});
                    if (it == Voff.end()) continue;
                    SP_REQUIRE((Vcols[{q, OB.c, bl.sec[sa].nb}] == OB.cols), "internal: V and L blocks disagree");
                    P.envl_out.add_term(B_BRA, X.off, 1, X.cols, B_V,
                                        g * P.Vsize + it->second + (long long)bl.sec[sa].ro * OB.cols, OB.cols, 1,
                                        X.rows, g * P.nc + P.c_one());
                }
            }
        }
    // ---- right pass, phase 1: Z(rb, sigma') rows of sector s_a' = X R(rb)^T
    std::vector<long long> Zoff(er.blk.size() * 4, -1);
    long long zoff = 0;
    for (size_t e = 0; e < er.blk.size(); ++e)
        for (int q = 0; q < 4; ++q) {
            const EnvBlk& rb = er.blk[e];
            const int i = bl.nblock(br.nb[rb.j].n - kSigmaN[q]);
            if (i < 0) continue;
            Zoff[e * 4 + q] = zoff;
            zoff += (long long)bl.nb[i].dim * rb.rows;
        }
    P.Zsize = zoff;
    for (int g = 0; g < G; ++g)
        for (size_t e = 0; e < er.blk.size(); ++e)
            for (int q = 0; q < 4; ++q) {
                if (Zoff[e * 4 + q] < 0) continue;
                const EnvBlk& rb = er.blk[e];
                const int i = bl.nblock(br.nb[rb.j].n - kSigmaN[q]);
                const NBlock& NA = bl.nb[i];
                for (int sa = NA.s0; sa < NA.s1; ++sa) {
                    const Sector& SA = bl.sec[sa];
                    P.p1r.add_task(B_T, g * P.Zsize + Zoff[e * 4 + q] + (long long)SA.ro * rb.rows, SA.dim, rb.rows,
                                   rb.rows);
                    const int xb = si.find(sa, q);
                    if (xb < 0) continue;
                    const XBlk& X = si.blk[xb];
                    const Sector& SB = br.sec[X.sb];
                    P.p1r.add_term(B_X, X.off, X.cols, 1, B_ENVR, g * Rsz + rb.off + SB.ro, 1, rb.cols, X.cols,
                                   g * P.nc + P.c_one());
                }
            }
    // ---- right pass, mixing: Zt(sigma, c, i') = sum W~[c, c', sigma, sigma'] Z(rb(c', b), sigma')
    std::map<std::array<int, 3>, long long> Ztoff;
    std::map<std::array<int, 3>, int> Ztcols;
    long long ztoff = 0;
    std::vector<VTerm> zterms;
    for (int sig = 0; sig < 4; ++sig)
        for (int c = 0; c < wl; ++c)
            for (int ip = 0; ip < int(bl.nb.size()); ++ip) {
                const int ia = bl.nblock(bl.nb[ip].n + h->dn[k - 1][c]);
                if (ia < 0) continue;
                const int nbb = br.nblock(bl.nb[ia].n + kSigmaN[sig]);
                if (nbb < 0) continue;
                bool any = false;
                for (const auto& ent : byR[size_t(sig) * wl + c]) {
                    const int cp = ent[0], q = ent[1];
                    const int e = er.find(cp, nbb);
                    if (e < 0 || Zoff[size_t(e) * 4 + q] < 0) continue;
                    const int irow = bl.nblock(br.nb[er.blk[e].j].n - kSigmaN[q]);
                    SP_REQUIRE(irow == ip, "internal: inconsistent particle numbers in the right mixing");
                    zterms.push_back({sig, c, ip, Zoff[size_t(e) * 4 + q], ent[2]});
                    any = true;
                }
                if (!any) continue;
                Ztoff[{sig, c, ip}] = ztoff;
                Ztcols[{sig, c, ip}] = br.nb[nbb].dim;
                ztoff += (long long)bl.nb[ip].dim * br.nb[nbb].dim;
            }
    P.Ztsize = ztoff;
    for (int g = 0; g < G; ++g) {
        size_t t = 0;
        while (t < zterms.size()) {
            const VTerm& v0 = zterms[t];
            const long long zo = Ztoff[{v0.sig, v0.cp, v0.i}];
            const int n = bl.nb[v0.i].dim * Ztcols[{v0.sig, v0.cp, v0.i}];
            P.mixr.add_task(B_V, g * P.Ztsize + zo, n);
            while (t < zterms.size() && zterms[t].sig == v0.sig && zterms[t].cp == v0.cp && zterms[t].i == v0.i) {
                P.mixr.add_term(B_T, g * P.Zsize + zterms[t].toffv, g * P.nc + P.c_wt(zterms[t].widx));
                ++t;
            }
        }
    }
    // ---- right environment update: R(c, a, a') rows of sector s_a = sum_sigma A Zt^T
    for (int g = 0; g < G; ++g)
        for (const EnvBlk& OB : el.blk) {
            const NBlock& NA = bl.nb[OB.i];
            for (int sa = NA.s0; sa < NA.s1; ++sa) {
                const Sector& SA = bl.sec[sa];
                P.envr_out.add_task(B_OUT, g * Lsz + OB.off + (long long)SA.ro * OB.cols, SA.dim, OB.cols, OB.cols);
                for (int q = 0; q < 4; ++q) {
                    const int xb = si.find(sa, q);
                    if (xb < 0) continue;
                    const XBlk& X = si.blk[xb];
                    const Sector& SB = br.sec[X.sb];
                    auto it = Ztoff.find({q, OB.c, OB.j});
                    if (it == Ztoff.end()) continue;
                    const int nbcols = Ztcols[{q, OB.c, OB.j}];
                    P.envr_out.add_term(B_BRA, X.off, X.cols, 1, B_V, g * P.Ztsize + it->second + SB.ro, 1, nbcols,
                                        X.cols, g * P.nc + P.c_one());
                }
            }
        }
    // ---- diagonal of H_eff and N_eff
    for (const XBlk& X : si.blk) {
        const Sector& SA = bl.sec[X.sa];
        const Sector& SB = br.sec[X.sb];
        spk::DiagBlk db{};
        db.x_off = X.off;
        db.rows = X.rows;
        db.cols = X.cols;
        db.sigma = X.s;
        db.t0 = int(P.dterm_h.size());
        for (const auto& ent : byD[X.s]) {
            const int c = ent[0], cp = ent[1];
            const int e = el.find(c, SA.nb);
            if (e < 0 || el.blk[e].j != SA.nb) continue;
            {
                const int re = er.find(cp, SB.nb);
                if (re < 0 || er.blk[re].j != SB.nb) continue;
                spk::DiagTerm dt{};
                dt.l_off = el.blk[e].off + (long long)SA.ro * (el.blk[e].cols + 1);
                dt.r_off = er.blk[re].off + (long long)SB.ro * (er.blk[re].cols + 1);
                dt.l_ld = el.blk[e].cols;
                dt.r_ld = er.blk[re].cols;
                dt.cidx = P.c_cwt(ent[2]);
                P.dterm_h.push_back(dt);
            }
        }
        db.t1 = int(P.dterm_h.size());
        P.dblk_h.push_back(db);
        db.t0 = int(P.dterm_n.size());
        const int e0 = el.find(0, SA.nb);
        const int re = er.find(lastR, SB.nb);
        if (e0 >= 0 && re >= 0) {
            spk::DiagTerm dt{};
            dt.l_off = el.blk[e0].off + (long long)SA.ro * (el.blk[e0].cols + 1);
            dt.r_off = er.blk[re].off + (long long)SB.ro * (er.blk[re].cols + 1);
            dt.l_ld = el.blk[e0].cols;
            dt.r_ld = er.blk[re].cols;
            dt.cidx = P.c_gr(X.s, X.s);
            P.dterm_n.push_back(dt);
        }
        db.t1 = int(P.dterm_n.size());
        P.dblk_n.push_back(db);
    }
    // ---- QR per right sector (left-orthonormalise) and LQ per left sector
    P.qr_roff.assign(br.sec.size(), -1);
    long long sc = 0, ro = 0;
    for (int sb = 0; sb < int(br.sec.size()); ++sb) {
        spk::QrTask t{};
        t.p0 = int(P.qr_pieces.size());
        int rows = 0;
        for (const XBlk& X : si.blk)
            if (X.sb == sb) {
                P.qr_pieces.push_back(spk::QrPiece{X.off, X.rows, X.cols, 0, rows});
                rows += X.rows;
            }
        t.p1 = int(P.qr_pieces.size());
        t.rows = rows;
        t.cols = br.sec[sb].dim;
        SP_REQUIRE(t.cols <= 256, "a sector wider than 256 states is not supported");
        if (rows == 0) continue;
        SP_REQUIRE(rows >= t.cols, "block table: a sector is wider than its left support");
        t.scratch_off = sc;
        t.r_off = ro;
        P.qr_roff[sb] = ro;
        sc += 2LL * rows * t.cols;
        ro += (long long)t.cols * t.cols;
        P.qr_lds = int(std::min<long long>(INT32_MAX, std::max<long long>(P.qr_lds, 2LL * rows * t.cols)));
        P.qr_tasks.push_back(t);
    }
    P.qr_scratch = sc;
    P.qr_rsize = ro;
    P.lq_roff.assign(bl.sec.size(), -1);
    sc = 0;
    ro = 0;
    for (int sa = 0; sa < int(bl.sec.size()); ++sa) {
        spk::QrTask t{};
        t.p0 = int(P.lq_pieces.size());
        int rows = 0;
        for (const XBlk& X : si.blk)
            if (X.sa == sa) {
                P.lq_pieces.push_back(spk::QrPiece{X.off, X.rows, X.cols, 1, rows});
                rows += X.cols;
            }
        t.p1 = int(P.lq_pieces.size());
        t.rows = rows;
        t.cols = bl.sec[sa].dim;
        SP_REQUIRE(t.cols <= 256, "a sector wider than 256 states is not supported");
        if (rows == 0) continue;
        SP_REQUIRE(rows >= t.cols, "block table: a sector is wider than its right support");
        t.scratch_off = sc;
        t.r_off = ro;
        P.lq_roff[sa] = ro;
        sc += 2LL * rows * t.cols;
        ro += (long long)t.cols * t.cols;
        P.lq_lds = int(std::min<long long>(INT32_MAX, std::max<long long>(P.lq_lds, 2LL * rows * t.cols)));
        P.lq_tasks.push_back(t);
    }
    P.lq_scratch = sc;
    P.lq_rsize = ro;
    // absorb R of this site into site k+1: A[k+1](sb, ., .) <- R_sb A[k+1](sb, ., .)
    if (k < h->L) {
        const SiteInfo& sn = h->sites[k];
        for (const XBlk& X : sn.blk) {
            P.absorb_right.add_task(B_OUT, X.off, X.rows, X.cols, X.cols);
            const long long r = P.qr_roff[X.sa];
            SP_REQUIRE(r >= 0, "internal: missing R factor");
            P.absorb_right.add_term(B_V, r, X.rows, 1, B_X, X.off, X.cols, 1, X.rows, P.c_one());
        }
    }
    // absorb L of this site into site k-1: A[k-1](., ., sa) <- A[k-1](., ., sa) L_sa, L = R'^T
    if (k > 1) {
        const SiteInfo& sp = h->sites[k - 2];
        for (const XBlk& X : sp.blk) {
            P.absorb_left.add_task(B_OUT, X.off, X.rows, X.cols, X.cols);
            const long long r = P.lq_roff[X.sb];
            SP_REQUIRE(r >= 0, "internal: missing L factor");
            P.absorb_left.add_term(B_X, X.off, X.cols, 1, B_V, r, 1, X.cols, X.cols, P.c_one());
        }
    }
    // algorithmic flops of one H_eff x: per g the left product, the mixing and
    // the right product for y, and the right product of ny
    P.heff_flops = P.p1.flops + P.mixl.flops + P.yout.flops;

    // ================= tiled path =================
    // dense particle-number blocks Xd(j, sigma, jb) of the site (zero outside
    // the (N, M) blocks) and the map from dense elements to packed indices
    std::vector<long long> Xdoff(bl.nb.size() * 4, -1);
    long long xd = 0;
    for (int j = 0; j < int(bl.nb.size()); ++j)
        for (int q = 0; q < 4; ++q) {
            const int jb = br.nblock(bl.nb[j].n + kSigmaN[q]);
            if (jb < 0) continue;
            Xdoff[size_t(j) * 4 + q] = xd;
            xd += (long long)bl.nb[j].dim * br.nb[jb].dim;
        }
    P.Xd_size = xd;
    P.xmap_h.assign(size_t(std::max(1LL, xd)), -1);
    for (const XBlk& X : si.blk) {
        const Sector& SA = bl.sec[X.sa];
        const Sector& SB = br.sec[X.sb];
        const int ldb = br.nb[SB.nb].dim;
        const long long base = Xdoff[size_t(SA.nb) * 4 + X.s];
        for (int r = 0; r < X.rows; ++r)
            for (int c = 0; c < X.cols; ++c)
                P.xmap_h[base + (long long)(SA.ro + r) * ldb + SB.ro + c] = int(X.off + (long long)r * X.cols + c);
    }
    auto xdoff = [&](int j, int q) { return Xdoff[size_t(j) * 4 + q]; };
    // rows of N-block j (bond k-1) that columns [c0, c1) of N-block jb (bond k)
    // reach through sigma, as one contiguous range
    auto k_from_cols = [&](int jb, int q, int c0, int c1, int& k0, int& k1) {
        k0 = INT32_MAX;
        k1 = -1;
        const NBlock& NB = br.nb[jb];
        for (int sb = NB.s0; sb < NB.s1; ++sb) {
            const Sector& SB = br.sec[sb];
            if (SB.ro + SB.dim <= c0 || SB.ro >= c1) continue;
            const int sa = bl.sector(SB.n - kSigmaN[q], SB.m2 - kSigma2M[q]);
            if (sa < 0) continue;
            k0 = std::min(k0, bl.sec[sa].ro);
            k1 = std::max(k1, bl.sec[sa].ro + bl.sec[sa].dim);
        }
        return k1 > k0;
    };
    // columns of N-block jb (bond k) that rows [r0, r1) of N-block j reach
    auto k_from_rows = [&](int j, int q, int r0, int r1, int& k0, int& k1) {
        k0 = INT32_MAX;
        k1 = -1;
        const NBlock& NA = bl.nb[j];
        for (int sa = NA.s0; sa < NA.s1; ++sa) {
            const Sector& SA = bl.sec[sa];
            if (SA.ro + SA.dim <= r0 || SA.ro >= r1) continue;
            const int sb = br.sector(SA.n + kSigmaN[q], SA.m2 + kSigma2M[q]);
            if (sb < 0) continue;
            k0 = std::min(k0, br.sec[sb].ro);
            k1 = std::max(k1, br.sec[sb].ro + br.sec[sb].dim);
        }
        return k1 > k0;
    };
    // output tile of the site's lists: 32 when the particle-number blocks of
    // both bonds are narrow (dimension-weighted mean <= 32), else 64
    int TT = spk::kTile;
    {
        double wsum = 0.0, dsum = 0.0;
        for (const Bond* bd : {&bl, &br})
            for (const NBlock& nb : bd->nb) {
                wsum += double(nb.dim) * nb.dim;
                dsum += nb.dim;
            }
        if (dsum > 0 && wsum / dsum <= 32.0) TT = 32;
    }
    for (TList* tl : {&P.t_left, &P.t_right, &P.t_envl, &P.t_zr, &P.t_envr}) tl->tile = TT;
    // left product: T(eb, sigma') = L_g(eb) Xd(j, sigma', jb)
    for (int g = 0; g < G; ++g)
        for (size_t e = 0; e < el.blk.size(); ++e)
            for (int q = 0; q < 4; ++q) {
                if (Toff[e * 4 + q] < 0) continue;
                const EnvBlk& eb = el.blk[e];
                const int jb = br.nblock(bl.nb[eb.j].n + kSigmaN[q]);
                const int ncol = br.nb[jb].dim;
                for (int r0 = 0; r0 < eb.rows; r0 += TT)
                    for (int c0 = 0; c0 < ncol; c0 += TT) {
                        P.t_left.add_task(B_T, g * P.Tsize + Toff[e * 4 + q], ncol, eb.rows, ncol, r0, c0, 0, 0);
                        int k0, k1;
                        if (k_from_cols(jb, q, c0, std::min(ncol, c0 + TT), k0, k1))
                            P.t_left.add_seg(B_ENVL, g * Lsz + eb.off, eb.cols, 0, B_X, xdoff(eb.j, q), ncol, 0, k0, k1,
                                             g * P.nc + P.c_one());
                    }
            }
    // Pre-mixed left environment with the unrotated MPO, Lt(sigma, c', i,
    // sigma'') = sum_c W[c, c', sigma, sigma''] L(c, i) (rows of bra N-block i
    // x ket N-block j, the same j for every channel c of the group), and the
    // rotated site vector Xr(sigma'', j) = sum_sigma' r_g(sigma'', sigma')
    // Xd(j, sigma') (Eq. [expSy]: it mixes the two singly occupied states
    // only, so Xr = Xd for the empty and doubly occupied states), so that
    // V(sigma, c', i) = sum_sigma'' Lt(sigma, c', i, sigma'') Xr(sigma'', j).
    // The rotation acts on the site vector, which is small, instead of
    // multiplying the environment blocks: fewer and smaller Lt blocks.  The
    // Lt blocks are built once per local problem, the Xr blocks with every
    // product; both live in the pre-mixed scratch (Lt first, then Xr).
    for (TList* tl : {&P.t_leftv, &P.t_left0}) tl->tile = TT;
    {
        struct LtBlk {
            int j;
            long long off;
            std::vector<std::pair<int, int>> terms;  // (env block e, unrotated entry)
        };
        std::vector<LtBlk> lts;
        std::map<std::array<int, 4>, int> ltidx;  // (sigma, c', i, sigma'')
        long long lto = 0;
        for (int sig = 0; sig < 4; ++sig)
            for (int cp = 0; cp < wr; ++cp)
                for (int i = 0; i < int(bl.nb.size()); ++i) {
                    if (!Voff.count({sig, cp, i})) continue;
                    for (const auto& ent : byWr[size_t(sig) * wr + cp]) {
                        const int c = ent[0], s2 = ent[1];
                        const int e = el.find(c, i);
                        if (e < 0) continue;
                        const EnvBlk& eb = el.blk[e];
                        if (xdoff(eb.j, s2) < 0) continue;
                        auto it = ltidx.find({sig, cp, i, s2});
                        if (it == ltidx.end()) {
                            it = ltidx.emplace(std::array<int, 4>{sig, cp, i, s2}, int(lts.size())).first;
                            lts.push_back(LtBlk{eb.j, lto, {}});
                            lto += (long long)eb.rows * eb.cols;
                        }
                        LtBlk& lb = lts[it->second];
                        SP_REQUIRE(lb.j == eb.j, "internal: inconsistent particle numbers in the pre-mixed environment");
                        lb.terms.push_back({e, ent[2]});
                    }
                }
        // rotated site-vector blocks of the singly occupied states
        std::map<std::array<int, 2>, long long> xroff;  // (sigma'' in {1, 2}, j)
        long long xro = lto;
        for (int j = 0; j < int(bl.nb.size()); ++j)
            for (int s2 = 1; s2 <= 2; ++s2) {
                if (xdoff(j, s2) < 0) continue;
                xroff[{s2, j}] = xro;
                xro += (long long)bl.nb[j].dim * br.nb[br.nblock(bl.nb[j].n + kSigmaN[s2])].dim;
            }
        P.LTsize = xro;
        for (int g = 0; g < G; ++g)
            for (const LtBlk& lb : lts) {
                const EnvBlk& e0 = el.blk[lb.terms[0].first];
                P.premix.add_task(B_LT, g * P.LTsize + lb.off, e0.rows * e0.cols);
                for (const auto& tm : lb.terms)
                    P.premix.add_term(B_ENVL, g * Lsz + el.blk[tm.first].off, g * P.nc + P.c_wr(tm.second));
            }
        for (int g = 0; g < G; ++g)
            for (const auto& kv : xroff) {
                const int s2 = kv.first[0], j = kv.first[1];
                const int ncol = br.nb[br.nblock(bl.nb[j].n + kSigmaN[s2])].dim;
                P.xrmix.add_task(B_LT, g * P.LTsize + kv.second, bl.nb[j].dim * ncol);
                for (int q = 1; q <= 2; ++q) P.xrmix.add_term(B_X, xdoff(j, q), g * P.nc + P.c_r(s2, q));
            }
        // V(sigma, c', i) = sum over sigma'' (ascending) of Lt(sigma, c', i, sigma'') Xr(sigma'', j)
        for (int g = 0; g < G; ++g)
            for (int sig = 0; sig < 4; ++sig)
                for (int cp = 0; cp < wr; ++cp)
                    for (int i = 0; i < int(bl.nb.size()); ++i) {
                        auto vo = Voff.find({sig, cp, i});
                        if (vo == Voff.end()) continue;
                        const int ncol = Vcols[{sig, cp, i}];
                        const int nbk = br.nblock(bl.nb[i].n + kSigmaN[sig]);
                        const int nbp = br.nblock(br.nb[nbk].n - h->dn[k][cp]);
                        const int M = bl.nb[i].dim;
                        for (int r0 = 0; r0 < M; r0 += TT)
                            for (int c0 = 0; c0 < ncol; c0 += TT) {
                                P.t_leftv.add_task(B_V, g * P.Vsize + vo->second, ncol, M, ncol, r0, c0, 0, 0);
                                for (int s2 = 0; s2 < 4; ++s2) {
                                    auto li = ltidx.find({sig, cp, i, s2});
                                    if (li == ltidx.end()) continue;
                                    const LtBlk& lb = lts[li->second];
                                    SP_REQUIRE(br.nblock(bl.nb[lb.j].n + kSigmaN[s2]) == nbp,
                                               "internal: pre-mixed product columns");
                                    // rows of Xr reached by the tile's columns: those of
                                    // every state the rotation mixes into sigma''
                                    int k0 = INT32_MAX, k1 = -1;
                                    for (int q = 0; q < 4; ++q) {
                                        int a0, a1;
                                        if (rot_nonzero(s2, q) && k_from_cols(nbp, q, c0, std::min(ncol, c0 + TT), a0, a1)) {
                                            k0 = std::min(k0, a0);
                                            k1 = std::max(k1, a1);
                                        }
                                    }
                                    if (k1 <= k0) continue;
                                    if (s2 == 1 || s2 == 2)
                                        P.t_leftv.add_seg(B_LT, g * P.LTsize + lb.off, bl.nb[lb.j].dim, 0, B_LT,
                                                          g * P.LTsize + xroff.at({s2, lb.j}), ncol, 0, k0, k1,
                                                          g * P.nc + P.c_one());
                                    else
                                        P.t_leftv.add_seg(B_LT, g * P.LTsize + lb.off, bl.nb[lb.j].dim, 0, B_X,
                                                          xdoff(lb.j, s2), ncol, 0, k0, k1, g * P.nc + P.c_one());
                                }
                            }
                    }
        // T of the identity channel (c = 0) only, for N_eff
        for (int g = 0; g < G; ++g)
            for (size_t e = 0; e < el.blk.size(); ++e) {
                if (el.blk[e].c != 0) continue;
                for (int q = 0; q < 4; ++q) {
                    if (Toff[e * 4 + q] < 0) continue;
                    const EnvBlk& eb = el.blk[e];
                    const int jb = br.nblock(bl.nb[eb.j].n + kSigmaN[q]);
                    const int ncol = br.nb[jb].dim;
                    for (int r0 = 0; r0 < eb.rows; r0 += TT)
                        for (int c0 = 0; c0 < ncol; c0 += TT) {
                            P.t_left0.add_task(B_T, g * P.Tsize + Toff[e * 4 + q], ncol, eb.rows, ncol, r0, c0, 0, 0);
                            int k0, k1;
                            if (k_from_cols(jb, q, c0, std::min(ncol, c0 + TT), k0, k1))
                                P.t_left0.add_seg(B_ENVL, g * Lsz + eb.off, eb.cols, 0, B_X, xdoff(eb.j, q), ncol, 0, k0,
                                                  k1, g * P.nc + P.c_one());
                        }
                }
            }
    }
    // right product: per g partial y and ny, scattered into the packed layout.
    // An output tile sums over every right channel; wide MPOs have hundreds,
    // so the channel list of a tile is cut into up to tr_split chunks, each
    // its own work-group writing partial slot (chunk * G + g): the consumers
    // add all tr_split * G slots in a fixed order (slots a tile has no chunk
    // for are zero-filled before the launch).  tr_split aims at about 16384
    // work-groups (two per wave slot of the GPU for the 64-thread tiles: a
    // work-group's channels run as a chain of dependent chunk loads, so the
    // chains are cut short; 8192 was 9% and 32768 1% slower at the K = 12
    // ab-initio centre), each with at least 4 channels, so that the extra
    // partial slots stay few.
    const long long xs = si.size;
    struct TSegD {
        int a_buf;
        long long a_off;
        int lda, ta, b_buf;
        long long b_off;
        int ldb, tb, k0, k1, cidx;
    };
    struct TOut {
        int c_buf, g, Nn, M, r0, c0;
        long long pack;
        std::vector<TSegD> segs;
    };
    std::vector<TOut> outs;
    for (int g = 0; g < G; ++g)
        for (int i = 0; i < int(bl.nb.size()); ++i)
            for (int sig = 0; sig < 4; ++sig) {
                const int nbb = br.nblock(bl.nb[i].n + kSigmaN[sig]);
                if (nbb < 0) continue;
                const int M = bl.nb[i].dim, Nn = br.nb[nbb].dim;
                for (int r0 = 0; r0 < M; r0 += TT)
                    for (int c0 = 0; c0 < Nn; c0 += TT) {
                        int k0, k1;
                        if (!k_from_rows(i, sig, r0, std::min(M, r0 + TT), k0, k1)) continue;
                        if (k1 <= c0 || k0 >= std::min(Nn, c0 + TT)) continue;  // no (N, M) block in the tile
                        TOut oy{B_Y, g, Nn, M, r0, c0, xdoff(i, sig), {}};
                        for (int cp = 0; cp < wr; ++cp) {
                            auto it = Voff.find({sig, cp, i});
                            if (it == Voff.end()) continue;
                            const int re = er.find(cp, nbb);
                            if (re < 0) continue;
                            const EnvBlk& RB = er.blk[re];
                            oy.segs.push_back(TSegD{B_V, g * P.Vsize + it->second, RB.cols, 0, B_ENVR,
                                                    g * Rsz + RB.off, RB.cols, 1, 0, RB.cols, g * P.nc + P.c_g()});
                        }
                        outs.push_back(std::move(oy));
                        TOut on{B_NY, g, Nn, M, r0, c0, xdoff(i, sig), {}};
                        const int e0 = el.find(0, i);
                        const int re = er.find(lastR, nbb);
                        if (e0 >= 0 && re >= 0)
                            for (int q = 0; q < 4; ++q) {
                                if (!rot_nonzero(sig, q)) continue;
                                const long long to = Toff[size_t(e0) * 4 + q];
                                if (to < 0) continue;
                                const EnvBlk& RB = er.blk[re];
                                on.segs.push_back(TSegD{B_T, g * P.Tsize + to, Tcols[size_t(e0) * 4 + q], 0, B_ENVR,
                                                        g * Rsz + RB.off, RB.cols, 1, 0, RB.cols,
                                                        g * P.nc + P.c_gr(sig, q)});
                            }
                        outs.push_back(std::move(on));
                    }
            }
    size_t max_segs = 1;
    for (const TOut& o : outs) max_segs = std::max(max_segs, o.segs.size());
    const int want = int(std::max<size_t>(1, (16384 + outs.size() - 1) / std::max<size_t>(1, outs.size())));
    const int kSegChunk = int(std::max<size_t>(4, (max_segs + want - 1) / want));
    P.tr_split = 1;
    for (const TOut& o : outs)
        P.tr_split = std::max(P.tr_split, int((o.segs.size() + kSegChunk - 1) / kSegChunk));
    for (const TOut& o : outs) {
        const int nchunk = std::max(1, int((o.segs.size() + kSegChunk - 1) / kSegChunk));
        for (int c = 0; c < nchunk; ++c) {
            P.t_right.add_task(o.c_buf, ((long long)c * G + o.g) * xs, o.Nn, o.M, o.Nn, o.r0, o.c0, 1, o.pack);
            const size_t s0 = size_t(c) * kSegChunk, s1 = std::min(o.segs.size(), s0 + kSegChunk);
            for (size_t q = s0; q < s1; ++q) {
                const TSegD& d = o.segs[q];
                P.t_right.add_seg(d.a_buf, d.a_off, d.lda, d.ta, d.b_buf, d.b_off, d.ldb, d.tb, d.k0, d.k1, d.cidx);
            }
        }
    }
    // left environment: L[k](c', b, b') = sum_sigma Xd(a, sigma, b)^T V(sigma, c', a)
    for (int g = 0; g < G; ++g)
        for (const EnvBlk& OB : er.blk)
            for (int r0 = 0; r0 < OB.rows; r0 += TT)
                for (int c0 = 0; c0 < OB.cols; c0 += TT) {
                    P.t_envl.add_task(B_OUT, g * Rsz + OB.off, OB.cols, OB.rows, OB.cols, r0, c0, 0, 0);
                    for (int q = 0; q < 4; ++q) {
                        const int a = bl.nblock(br.nb[OB.i].n - kSigmaN[q]);
                        if (a < 0) continue;
                        auto it = Voff.find({q, OB.c, a});
                        if (it == Voff.end()) continue;
                        int k0, k1;
                        if (!k_from_cols(OB.i, q, r0, std::min(OB.rows, r0 + TT), k0, k1)) continue;
                        P.t_envl.add_seg(B_X, xdoff(a, q), OB.rows, 1, B_V, g * P.Vsize + it->second, OB.cols, 0, k0,
                                         k1, g * P.nc + P.c_one());
                    }
                }
    // right pass: Z(rb, sigma') = Xd(i, sigma', b') R_g(rb)^T
    for (int g = 0; g < G; ++g)
        for (size_t e = 0; e < er.blk.size(); ++e)
            for (int q = 0; q < 4; ++q) {
                if (Zoff[e * 4 + q] < 0) continue;
                const EnvBlk& rb = er.blk[e];
                const int i = bl.nblock(br.nb[rb.j].n - kSigmaN[q]);
                const int M = bl.nb[i].dim;
                for (int r0 = 0; r0 < M; r0 += TT)
                    for (int c0 = 0; c0 < rb.rows; c0 += TT) {
                        P.t_zr.add_task(B_T, g * P.Zsize + Zoff[e * 4 + q], rb.rows, M, rb.rows, r0, c0, 0, 0);
                        int k0, k1;
                        if (k_from_rows(i, q, r0, std::min(M, r0 + TT), k0, k1))
                            P.t_zr.add_seg(B_X, xdoff(i, q), rb.cols, 0, B_ENVR, g * Rsz + rb.off, rb.cols, 1, k0, k1,
                                           g * P.nc + P.c_one());
                    }
            }
    // right environment: R(c, a, a') = sum_sigma Xd(a, sigma, b) Zt(sigma, c, a')^T
    for (int g = 0; g < G; ++g)
        for (const EnvBlk& OB : el.blk)
            for (int r0 = 0; r0 < OB.rows; r0 += TT)
                for (int c0 = 0; c0 < OB.cols; c0 += TT) {
                    P.t_envr.add_task(B_OUT, g * Lsz + OB.off, OB.cols, OB.rows, OB.cols, r0, c0, 0, 0);
                    for (int q = 0; q < 4; ++q) {
                        auto it = Ztoff.find({q, OB.c, OB.j});
                        if (it == Ztoff.end()) continue;
                        const int nbb = br.nblock(bl.nb[OB.i].n + kSigmaN[q]);
                        int k0, k1;
                        if (!k_from_rows(OB.i, q, r0, std::min(OB.rows, r0 + TT), k0, k1)) continue;
                        P.t_envr.add_seg(B_X, xdoff(OB.i, q), br.nb[nbb].dim, 0, B_V, g * P.Ztsize + it->second,
                                         br.nb[nbb].dim, 1, k0, k1, g * P.nc + P.c_one());
                    }
                }
}

// fused H_eff x plan: column descriptors, products per bra block, channels
// per output sigma, output lists and row-chunk tasks
// LDS budget of the fused H_eff kernel per work-group (doubles): the default,
// and the largest the autotuner tries (the 160 KB of a CU less the static
// arrays)
constexpr int kHeffLdsBudget = 9216;
constexpr int kHeffLdsMax = 18432;

// Returns false (and leaves the site without a fused plan, h_rows = 0) when
// a particle-number block is too wide for the budget: the site then runs
// the LDS-tiled block-product lists.
bool build_fused(sp_handle* h, int k, int lds_budget = kHeffLdsBudget) {
    SitePlan& P = h->plan[k - 1];
    const int G = h->G;
    const Bond& bl = h->bonds[k - 1];
    const Bond& br = h->bonds[k];
    const SiteInfo& si = h->sites[k - 1];
    const EnvLayout& el = h->env[k - 1];
    const EnvLayout& er = h->env[k];
    const int wl = h->w[k - 1], wr = h->w[k];
    const int lastR = wr - 1;
    // rotated-MPO entries by (sigma, right channel): (left channel, sigma', entry)
    std::vector<std::vector<std::array<int, 3>>> byL(size_t(4) * wr);
    for (int e = 0; e < P.nW; ++e) {
        const auto& q = P.went[e];
        byL[size_t(q[2]) * wr + q[1]].push_back({q[0], q[3], e});
    }
    const int nb = int(bl.nb.size());

    // RC-independent description of one bra block
    struct TCol {
        int x_off, x_ld, K, src, ro;  // src: local L source, ro: its first column
    };
    struct TBlk {
        int ncol;
        std::vector<TCol> cols;
    };
    struct SegD {
        long long r_off;
        int K, is_ny;
        std::vector<std::pair<int, int>> terms;  // (local T block, coefficient)
    };
    struct BlkD {
        std::vector<std::pair<long long, int>> lsrc;  // (L offset, ld)
        std::vector<TBlk> T;
        std::array<std::vector<SegD>, 4> seg;
        int lsum = 0, tsum = 0, vmax = 0;
    };
    std::vector<BlkD> bd(nb);
    for (int i = 0; i < nb; ++i) {
        const NBlock& NA = bl.nb[i];
        BlkD& D = bd[i];
        std::map<std::pair<int, int>, int> tloc;  // (c, s') -> local T block
        for (int c = 0; c < wl; ++c) {
            const int e = el.find(c, i);
            if (e < 0) continue;
            const EnvBlk& EB = el.blk[e];
            const int src = int(D.lsrc.size());
            D.lsrc.push_back({EB.off, EB.cols});
            D.lsum += EB.cols;
            const int j = EB.j;
            for (int q = 0; q < 4; ++q) {
                const int jb = br.nblock(bl.nb[j].n + kSigmaN[q]);
                if (jb < 0) continue;
                const NBlock& NB = br.nb[jb];
                TBlk T;
                T.ncol = NB.dim;
                for (int sb = NB.s0; sb < NB.s1; ++sb) {
                    const Sector& SB = br.sec[sb];
                    const int sa = bl.sector(SB.n - kSigmaN[q], SB.m2 - kSigma2M[q]);
                    const int xb = sa >= 0 ? si.find(sa, q) : -1;
                    for (int c2 = 0; c2 < SB.dim; ++c2) {
                        if (xb < 0) {
                            T.cols.push_back(TCol{0, 0, 0, src, 0});
                        } else {
                            const XBlk& X = si.blk[xb];
                            SP_REQUIRE(bl.sec[sa].n == bl.nb[j].n, "internal: fused ket sector");
                            T.cols.push_back(TCol{int(X.off + c2), X.cols, X.rows, src, bl.sec[sa].ro});
                        }
                    }
                }
                tloc[{c, q}] = int(D.T.size());
                D.tsum += T.ncol;
                D.T.push_back(std::move(T));
            }
        }
        for (int sig = 0; sig < 4; ++sig) {
            const int nbb = br.nblock(NA.n + kSigmaN[sig]);
            if (nbb < 0) continue;
            auto add_seg = [&](int re, int is_ny, const std::vector<std::pair<int, int>>& tl) {
                if (tl.empty()) return;
                const EnvBlk& RB = er.blk[re];
                for (auto& pr : tl)
                    SP_REQUIRE(D.T[pr.first].ncol == RB.cols, "internal: fused H_eff particle numbers");
                D.seg[sig].push_back(SegD{RB.off, RB.cols, is_ny, tl});
            };
            for (int cp = 0; cp < wr; ++cp) {
                const int re = er.find(cp, nbb);
                if (re < 0) continue;
                std::vector<std::pair<int, int>> tl;
                for (const auto& ent : byL[size_t(sig) * wr + cp]) {  // ascending (c, s'), as tloc
                    auto it = tloc.find({ent[0], ent[1]});
                    if (it != tloc.end()) tl.push_back({it->second, P.c_cwt(ent[2])});
                }
                add_seg(re, 0, tl);
            }
            const int re = er.find(lastR, nbb);
            if (re >= 0) {
                std::vector<std::pair<int, int>> tl;
                for (int q = 0; q < 4; ++q) {
                    if (!rot_nonzero(sig, q)) continue;
                    auto it = tloc.find({0, q});
                    if (it == tloc.end()) continue;
                    SP_REQUIRE(el.blk[el.find(0, i)].j == i, "internal: identity channel must conserve N");
                    tl.push_back({it->second, P.c_gr(sig, q)});
                }
                add_seg(re, 1, tl);
            }
            int v = 0;
            for (auto& sd : D.seg[sig]) v += sd.K;
            D.vmax = std::max(D.vmax, v);
        }
    }
    // rows per task: the largest RC <= 8 whose LDS fits the budget
    int need1 = 1;
    for (auto& D : bd) need1 = std::max(need1, D.lsum + D.tsum + D.vmax);
    const int RC = std::min(spk::kH3MaxRC, lds_budget / need1);
    P.h_blks.clear();
    P.h_cols.clear();
    P.h_lsrc.clear();
    P.h_segs.clear();
    P.h_terms.clear();
    P.h_pieces.clear();
    P.h_tasks.clear();
    if (RC < 1) {
        P.h_rows = 0;
        P.h_lds = 0;
        return false;
    }
    P.h_rows = RC;
    P.h_lds = RC * need1;
    for (int i = 0; i < nb; ++i) {
        BlkD& D = bd[i];
        spk::H3Blk B{};
        B.l0 = int(P.h_lsrc.size());
        std::vector<int> lds_src(D.lsrc.size());
        int pos = 0;
        for (size_t q = 0; q < D.lsrc.size(); ++q) {
            SP_REQUIRE(D.lsrc[q].first < INT32_MAX, "environment too large for 32-bit offsets");
            lds_src[q] = pos;
            P.h_lsrc.push_back(spk::H3LSrc{int(D.lsrc[q].first), D.lsrc[q].second, pos, 0});
            pos += RC * D.lsrc[q].second;
        }
        B.l1 = int(P.h_lsrc.size());
        B.c0 = int(P.h_cols.size());
        std::vector<int> tbase(D.T.size());
        for (size_t t = 0; t < D.T.size(); ++t) {
            tbase[t] = pos;
            for (int c2 = 0; c2 < D.T[t].ncol; ++c2) {
                const TCol& tc = D.T[t].cols[c2];
                P.h_cols.push_back(spk::H3Col{tc.x_off, tc.x_ld, tc.K, lds_src[tc.src] + tc.ro,
                                              D.lsrc[tc.src].second, pos + c2 * RC, 0, 0});
            }
            pos += RC * D.T[t].ncol;
        }
        B.c1 = int(P.h_cols.size());
        // columns that read the same x column (channels with the same ket
        // block) next to each other: the kernel pairs neighbours and loads a
        // shared x column once; empty columns last
        std::stable_sort(P.h_cols.begin() + B.c0, P.h_cols.begin() + B.c1,
                         [](const spk::H3Col& a, const spk::H3Col& b) {
                             if ((a.K == 0) != (b.K == 0)) return b.K == 0;
                             return std::tie(a.x_off, a.x_ld, a.K) < std::tie(b.x_off, b.x_ld, b.K);
                         });
        const int vbase = pos;
        for (int sig = 0; sig < 4; ++sig) {
            B.s0[sig] = int(P.h_segs.size());
            int v = vbase;
            for (auto& sd : D.seg[sig]) {
                SP_REQUIRE(sd.r_off < INT32_MAX, "environment too large for 32-bit offsets");
                spk::H3Seg S{};
                S.r_off = int(sd.r_off);
                S.K = sd.K;
                S.v_off = v;
                S.t0 = int(P.h_terms.size());
                for (auto& pr : sd.terms) P.h_terms.push_back(spk::H3Term{tbase[pr.first], pr.second});
                S.t1 = int(P.h_terms.size());
                S.is_ny = sd.is_ny;
                P.h_segs.push_back(S);
                v += RC * sd.K;
            }
            B.s1[sig] = int(P.h_segs.size());
        }
        P.h_blks.push_back(B);
    }
    // tasks of one quadrature point: chunks of RC rows per bra block, with the
    // output pieces (rows of one left sector x the columns its sigma allows)
    std::vector<spk::H3Task> one;
    for (int i = 0; i < nb; ++i) {
        const NBlock& NA = bl.nb[i];
        for (int r0 = 0; r0 < NA.dim; r0 += RC) {
            spk::H3Task t{};
            t.g = 0;
            t.blk = i;
            t.r0 = r0;
            t.rows = std::min(RC, NA.dim - r0);
            bool any = false;
            for (int sig = 0; sig < 4; ++sig) {
                t.p0[sig] = t.p1[sig] = int(P.h_pieces.size());
                if (br.nblock(NA.n + kSigmaN[sig]) < 0) continue;
                for (int sa = NA.s0; sa < NA.s1; ++sa) {
                    const Sector& SA = bl.sec[sa];
                    const int lo = std::max(r0, SA.ro), hi = std::min(r0 + t.rows, SA.ro + SA.dim);
                    if (lo >= hi) continue;
                    const int sb = br.sector(SA.n + kSigmaN[sig], SA.m2 + kSigma2M[sig]);
                    if (sb < 0) continue;
                    const int xb = si.find(sa, sig);
                    SP_REQUIRE(xb >= 0, "internal: missing site block");
                    const XBlk& X = si.blk[xb];
                    spk::H3Piece pc{};
                    pc.rlo = lo - r0;
                    pc.rhi = hi - r0;
                    pc.b0 = br.sec[sb].ro;
                    pc.nb = br.sec[sb].dim;
                    pc.out_off = int(X.off + (long long)(lo - SA.ro) * X.cols);
                    pc.out_ld = X.cols;
                    P.h_pieces.push_back(pc);
                }
                t.p1[sig] = int(P.h_pieces.size());
                any = any || t.p1[sig] > t.p0[sig];
            }
            if (any) one.push_back(t);
        }
    }
    // all quadrature points, dealt to the eight XCDs in contiguous runs of the
    // g-ordered list (work-group w runs on XCD w mod 8), so that each XCD's L2
    // holds the environments of about G/8 quadrature points
    std::vector<spk::H3Task> all;
    for (int g = 0; g < G; ++g)
        for (spk::H3Task t : one) {
            t.g = g;
            all.push_back(t);
        }
    const int T = int(all.size()), nq = 8;
    const int rounds = (T + nq - 1) / nq;
    P.h_tasks.assign(size_t(rounds) * nq, spk::H3Task{0, -1, 0, 0, {0, 0, 0, 0}, {0, 0, 0, 0}});
    for (int q = 0; q < nq; ++q) {
        const int a0 = int((long long)T * q / nq), a1 = int((long long)T * (q + 1) / nq);
        for (int r = 0; r < a1 - a0; ++r) P.h_tasks[size_t(r) * nq + q] = all[a0 + r];
    }
    while (!P.h_tasks.empty() && P.h_tasks.back().blk < 0) P.h_tasks.pop_back();
    return true;
}

void upload_fused(sp_handle* h, int k) {
    SitePlan& P = h->plan[k - 1];
    hipStream_t s = h->stream;
    P.dh_tasks.upload(P.h_tasks, s);
    P.dh_blks.upload(P.h_blks, s);
    P.dh_cols.upload(P.h_cols, s);
    P.dh_lsrc.upload(P.h_lsrc, s);
    P.dh_segs.upload(P.h_segs, s);
    P.dh_terms.upload(P.h_terms, s);
    P.dh_pieces.upload(P.h_pieces, s);
    // every list the fused kernel reads must be on the device, whole
    SP_REQUIRE(P.dh_tasks.n == P.h_tasks.size() && P.dh_blks.n == P.h_blks.size() &&
                   P.dh_cols.n == P.h_cols.size() && P.dh_lsrc.n == P.h_lsrc.size() &&
                   P.dh_segs.n == P.h_segs.size() && P.dh_terms.n == P.h_terms.size() &&
                   P.dh_pieces.n == P.h_pieces.size(),
               "internal: fused plan upload");
    SP_REQUIRE(P.h_tasks.empty() || (P.dh_tasks.p && P.dh_blks.p && P.dh_cols.p && P.dh_lsrc.p && P.dh_pieces.p),
               "internal: fused plan upload");
}

void upload_plan(sp_handle* h, int k) {
    SitePlan& P = h->plan[k - 1];
    hipStream_t s = h->stream;
    P.coef.upload(P.coef_h, s);
    P.p1.upload(s);
    P.mixl.upload(s);
    P.yout.upload(s);
    P.envl_out.upload(s);
    P.p1r.upload(s);
    P.mixr.upload(s);
    P.envr_out.upload(s);
    P.ddblk_h.upload(P.dblk_h, s);
    P.ddblk_n.upload(P.dblk_n, s);
    P.ddterm_h.upload(P.dterm_h, s);
    P.ddterm_n.upload(P.dterm_n, s);
    P.dqr_tasks.upload(P.qr_tasks, s);
    P.dlq_tasks.upload(P.lq_tasks, s);
    P.dqr_pieces.upload(P.qr_pieces, s);
    P.dlq_pieces.upload(P.lq_pieces, s);
    P.absorb_right.upload(s);
    P.absorb_left.upload(s);
    P.xmap.upload(P.xmap_h, s);
    P.t_left.upload(s);
    P.t_leftv.upload(s);
    P.t_left0.upload(s);
    P.premix.upload(s);
    P.xrmix.upload(s);
    P.t_right.upload(s);
    P.t_envl.upload(s);
    P.t_zr.upload(s);
    P.t_envr.upload(s);
    upload_fused(h, k);
}

// ---------------------------------------------------------------------------
// bounds validation of every task list against the buffers it will touch
// (host side, at init): a descriptor error becomes SP_EINVAL, never a device
// memory fault

using Sizes = std::array<long long, spk::kMaxBufs>;

void check_span(long long off, long long last, long long size, const char* what) {
    if (off < 0 || last < off || last >= size) throw SpError(SP_EINVAL, std::string("internal bounds check: ") + what);
}

void validate(const BList& b, const Sizes& sz, long long ncoef, const char* what) {
    for (const spk::BTask& t : b.tasks) {
        if (t.M <= 0 || t.N <= 0) continue;
        check_span(t.c_off, t.c_off + (long long)(t.M - 1) * t.ldc + (t.N - 1), sz[t.c_buf], what);
        for (int i = t.t0; i < t.t1; ++i) {
            const spk::BTerm& m = b.terms[i];
            if (m.K <= 0) throw SpError(SP_EINVAL, std::string("internal: empty term in ") + what);
            check_span(m.a_off, m.a_off + (long long)(t.M - 1) * m.a_rs + (long long)(m.K - 1) * m.a_cs,
                       sz[m.a_buf], what);
            check_span(m.b_off, m.b_off + (long long)(m.K - 1) * m.b_rs + (long long)(t.N - 1) * m.b_cs,
                       sz[m.b_buf], what);
            check_span(m.cidx, m.cidx, ncoef, what);
        }
    }
}

void validate(const CList& b, const Sizes& sz, long long ncoef, const char* what) {
    for (const spk::CTask& t : b.tasks) {
        check_span(t.c_off, t.c_off + t.n - 1, sz[t.c_buf], what);
        for (int i = t.t0; i < t.t1; ++i) {
            check_span(b.terms[i].a_off, b.terms[i].a_off + t.n - 1, sz[b.terms[i].a_buf], what);
            check_span(b.terms[i].cidx, b.terms[i].cidx, ncoef, what);
        }
    }
}

void validate(const TList& b, const Sizes& sz, long long ncoef, long long map_size, long long packed_max,
              const char* what) {
    const int TT = b.tile;
    if (TT != 32 && TT != 64) throw SpError(SP_EINVAL, std::string("internal tile size: ") + what);
    for (const spk::TTask& t : b.tasks) {
        if (t.r0 < 0 || t.c0 < 0 || t.r0 >= t.M || t.c0 >= t.N) throw SpError(SP_EINVAL, std::string("internal tile: ") + what);
        const int rl = std::min(t.M, t.r0 + TT) - 1, cl = std::min(t.N, t.c0 + TT) - 1;
        if (t.mode == 0) {
            check_span(t.c_off + (long long)t.r0 * t.ldc + t.c0, t.c_off + (long long)rl * t.ldc + cl, sz[t.c_buf], what);
        } else {
            check_span(t.pack_off, t.pack_off + (long long)(t.M - 1) * t.N + (t.N - 1), map_size, what);
            check_span(t.c_off, t.c_off + packed_max - 1, sz[t.c_buf], what);
        }
        for (int i = t.s0; i < t.s1; ++i) {
            const spk::TSeg& g = b.segs[i];
            if (g.k0 < 0 || g.k1 <= g.k0) throw SpError(SP_EINVAL, std::string("internal segment: ") + what);
            const long long a_first = g.ta ? g.a_off + (long long)g.k0 * g.lda + t.r0 : g.a_off + (long long)t.r0 * g.lda + g.k0;
            const long long a_last = g.ta ? g.a_off + (long long)(g.k1 - 1) * g.lda + rl : g.a_off + (long long)rl * g.lda + (g.k1 - 1);
            const long long b_first = g.tb ? g.b_off + (long long)t.c0 * g.ldb + g.k0 : g.b_off + (long long)g.k0 * g.ldb + t.c0;
            const long long b_last = g.tb ? g.b_off + (long long)cl * g.ldb + (g.k1 - 1) : g.b_off + (long long)(g.k1 - 1) * g.ldb + cl;
            check_span(a_first, a_last, sz[g.a_buf], what);
            check_span(b_first, b_last, sz[g.b_buf], what);
            check_span(g.cidx, g.cidx, ncoef, what);
        }
    }
}

// bounds of every list of the fused H_eff plan of site k (host side)
void validate_fused(sp_handle* h, int k) {
    const SitePlan& P = h->plan[k - 1];
    const long long xs = h->sites[k - 1].size;
    if (P.h_rows == 0) {  // no fused plan: the site runs the plain lists
        if (!P.h_tasks.empty() || P.h_lds != 0) throw SpError(SP_EINVAL, "internal: fused plan state");
        return;
    }
    const long long Lg = h->env[k - 1].size, Rg = h->env[k].size;
    const int RC = P.h_rows, lmax = P.h_lds;
    const int nblk = int(P.h_blks.size());
    auto in_lds = [&](long long a0, long long a1, const char* what) { check_span(a0, a1, lmax, what); };
    if (RC < 1 || RC > spk::kH3MaxRC || lmax > kHeffLdsMax) throw SpError(SP_EINVAL, "internal: fused shape");
    std::vector<int> seen(size_t(xs) * h->G, 0);
    for (const spk::H3Task& t : P.h_tasks) {
        if (t.blk < 0) continue;
        if (t.g < 0 || t.g >= h->G || t.blk >= nblk || t.rows < 1 || t.rows > RC)
            throw SpError(SP_EINVAL, "internal: fused task");
        const spk::H3Blk& B = P.h_blks[t.blk];
        check_span(B.l0, B.l1 - 1, (long long)P.h_lsrc.size(), "fused L sources");
        for (int q = B.l0; q < B.l1; ++q) {
            const spk::H3LSrc& L = P.h_lsrc[q];
            check_span(L.l_off + (long long)t.r0 * L.ld, L.l_off + (long long)(t.r0 + t.rows) * L.ld - 1, Lg,
                       "fused L rows");
            in_lds(L.lds, L.lds + (long long)RC * L.ld - 1, "fused staged L");
        }
        if (B.c1 > B.c0) check_span(B.c0, B.c1 - 1, (long long)P.h_cols.size(), "fused columns");
        for (int ci = B.c0; ci < B.c1; ++ci) {
            const spk::H3Col& c = P.h_cols[ci];
            if (c.K > 0) {
                check_span(c.x_off, c.x_off + (long long)(c.K - 1) * c.x_ld, xs, "fused x column");
                in_lds(c.l_lds, c.l_lds + (long long)(RC - 1) * c.l_ld + c.K - 1, "fused L entries");
            }
            in_lds(c.t_pos, c.t_pos + RC - 1, "fused T column");
        }
        for (int sig = 0; sig < 4; ++sig) {
            if (B.s1[sig] > B.s0[sig]) check_span(B.s0[sig], B.s1[sig] - 1, (long long)P.h_segs.size(), "fused segments");
            if (t.p1[sig] > t.p0[sig]) check_span(t.p0[sig], t.p1[sig] - 1, (long long)P.h_pieces.size(), "fused pieces");
            for (int p = t.p0[sig]; p < t.p1[sig]; ++p) {
                const spk::H3Piece& pc = P.h_pieces[p];
                if (pc.rlo < 0 || pc.rhi > t.rows || pc.rlo >= pc.rhi || pc.nb < 1)
                    throw SpError(SP_EINVAL, "internal: fused piece");
                for (int rr = pc.rlo; rr < pc.rhi; ++rr)
                    for (int b = 0; b < pc.nb; ++b) {
                        const long long o = pc.out_off + (long long)(rr - pc.rlo) * pc.out_ld + b;
                        check_span(o, o, xs, "fused output");
                        if (seen[size_t(t.g) * xs + o]++) throw SpError(SP_EINVAL, "internal: fused output written twice");
                    }
                for (int si = B.s0[sig]; si < B.s1[sig]; ++si) {
                    const spk::H3Seg& S = P.h_segs[si];
                    check_span(S.r_off + (long long)pc.b0 * S.K, S.r_off + (long long)(pc.b0 + pc.nb) * S.K - 1, Rg,
                               "fused R rows");
                }
            }
            for (int si = B.s0[sig]; si < B.s1[sig]; ++si) {
                const spk::H3Seg& S = P.h_segs[si];
                in_lds(S.v_off, S.v_off + (long long)RC * S.K - 1, "fused V");
                if (S.t1 > S.t0) check_span(S.t0, S.t1 - 1, (long long)P.h_terms.size(), "fused terms");
                for (int tm = S.t0; tm < S.t1; ++tm) {
                    in_lds(P.h_terms[tm].t_base, P.h_terms[tm].t_base + (long long)RC * S.K - 1, "fused T block");
                    check_span(P.h_terms[tm].cidx, P.h_terms[tm].cidx, P.nc, "fused coefficient");
                }
            }
        }
    }
    for (long long o = 0; o < (long long)xs * h->G; ++o)
        if (seen[o] != 1) throw SpError(SP_EINVAL, "internal: fused outputs do not cover the site");
}

void validate_plans(sp_handle* h) {
    const long long G = h->G;
    for (int k = 1; k <= h->L; ++k) {
        const SitePlan& P = h->plan[k - 1];
        const long long nco = G * P.nc;
        const long long xs = h->sites[k - 1].size;
        const long long Lb = G * h->env[k - 1].size, Rb = G * h->env[k].size;
        const long long Tb = h->T_cap, Vb = h->V_cap;
        Sizes z{};
        z.fill(0);
        z[B_ENVL] = Lb;
        z[B_ENVR] = Rb;
        z[B_X] = xs;
        z[B_T] = Tb;
        z[B_V] = Vb;
        z[B_Y] = xs;
        z[B_NY] = xs;
        z[B_BRA] = xs;
        if (G * P.Tsize > Tb || G * P.Vsize > Vb || G * P.Zsize > Tb || G * P.Ztsize > Vb)
            throw SpError(SP_EINVAL, "internal: scratch too small");
        validate(P.p1, z, nco, "left product");
        validate(P.mixl, z, nco, "left mixing");
        validate(P.yout, z, nco, "H_eff output");
        validate(P.p1r, z, nco, "right product");
        validate(P.mixr, z, nco, "right mixing");
        z[B_OUT] = Rb;
        validate(P.envl_out, z, nco, "left environment");
        z[B_OUT] = Lb;
        validate(P.envr_out, z, nco, "right environment");
        // tiled lists: B_X is the dense site layout, B_Y/B_NY the per-g partials
        {
            Sizes t = z;
            t[B_X] = h->Xd_cap;
            t[B_Y] = G * h->tr_split_max * h->max_site;
            t[B_NY] = G * h->tr_split_max * h->max_site;
            for (int e : P.xmap_h)
                if (e >= xs) throw SpError(SP_EINVAL, "internal: packed map out of range");
            const long long ms = (long long)P.xmap_h.size();
            validate(P.t_left, t, nco, ms, xs, "tiled left product");
            if (h->path == SP_PATH_TILED) {  // the plain path has no pre-mixed environment buffer
                t[B_LT] = h->LT_cap;
                if (G * P.LTsize > h->LT_cap)
                    throw SpError(SP_EINVAL, "internal: pre-mixed environment scratch too small");
                validate(P.t_leftv, t, nco, ms, xs, "tiled product of the pre-mixed environment");
                validate(P.t_left0, t, nco, ms, xs, "tiled identity-channel product");
                validate(P.premix, t, nco, "pre-mixed left environment");
                validate(P.xrmix, t, nco, "rotated site vector");
            }
            validate(P.t_right, t, nco, ms, xs, "tiled right product");
            validate(P.t_zr, t, nco, ms, xs, "tiled right-pass product");
            t[B_OUT] = Rb;
            validate(P.t_envl, t, nco, ms, xs, "tiled left environment");
            t[B_OUT] = Lb;
            validate(P.t_envr, t, nco, ms, xs, "tiled right environment");
            if (P.Xd_size > h->Xd_cap) throw SpError(SP_EINVAL, "internal: dense site scratch too small");
        }
        validate_fused(h, k);
        if (k < h->L) {
            Sizes a{};
            a.fill(0);
            a[B_V] = h->qr_r_cap;
            a[B_X] = h->sites[k].size;
            a[B_OUT] = std::min<long long>(h->sites[k].size, h->max_site);
            validate(P.absorb_right, a, P.nc, "absorb right");
        }
        if (k > 1) {
            Sizes a{};
            a.fill(0);
            a[B_V] = h->qr_r_cap;
            a[B_X] = h->sites[k - 2].size;
            a[B_OUT] = std::min<long long>(h->sites[k - 2].size, h->max_site);
            validate(P.absorb_left, a, P.nc, "absorb left");
        }
        for (int pass = 0; pass < 2; ++pass) {
            const auto& tasks = pass ? P.lq_tasks : P.qr_tasks;
            const auto& pieces = pass ? P.lq_pieces : P.qr_pieces;
            for (const spk::QrTask& t : tasks) {
                if (t.cols > 256 || t.rows < t.cols) throw SpError(SP_EINVAL, "internal: bad QR task");
                check_span(t.scratch_off, t.scratch_off + 2LL * t.rows * t.cols - 1, h->qr_scratch_cap, "QR scratch");
                check_span(t.r_off, t.r_off + (long long)t.cols * t.cols - 1, h->qr_r_cap, "QR factor");
                int rows = 0;
                for (int i = t.p0; i < t.p1; ++i) {
                    const spk::QrPiece& pc = pieces[i];
                    check_span(pc.off, pc.off + (long long)pc.prow * pc.pcol - 1, xs, "QR piece");
                    if ((pc.transposed ? pc.prow : pc.pcol) != t.cols || pc.row0 != rows)
                        throw SpError(SP_EINVAL, "internal: QR piece shape");
                    rows += pc.transposed ? pc.pcol : pc.prow;
                }
                if (rows != t.rows) throw SpError(SP_EINVAL, "internal: QR rows");
            }
        }
        for (int pass = 0; pass < 2; ++pass) {
            const auto& blks = pass ? P.dblk_n : P.dblk_h;
            const auto& terms = pass ? P.dterm_n : P.dterm_h;
            for (const spk::DiagBlk& d : blks) {
                check_span(d.x_off, d.x_off + (long long)d.rows * d.cols - 1, xs, "diagonal block");
                for (int i = d.t0; i < d.t1; ++i) {
                    const spk::DiagTerm& t = terms[i];
                    check_span(t.l_off, t.l_off + (long long)(d.rows - 1) * (t.l_ld + 1), h->env[k - 1].size, "diag L");
                    check_span(t.r_off, t.r_off + (long long)(d.cols - 1) * (t.r_ld + 1), h->env[k].size, "diag R");
                    check_span(t.cidx, t.cidx, P.nc, "diag coefficient");
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// operations

double* site_ptr(sp_handle* h, int k) { return h->mps.p + h->sites[k - 1].goff; }

// the N-blocks of site k's tensor: its (left sector, sigma) blocks grouped by
// the left bond's particle number and that of sigma (hence also the right
// bond's), whatever their M
const NBlocks& site_nblocks(sp_handle* h, int k) {
    if (h->nblocks.size() != size_t(h->L)) h->nblocks.resize(h->L);
    NBlocks& nb = h->nblocks[k - 1];
    if (nb.ng > 0) return nb;
    const SiteInfo& si = h->sites[k - 1];
    const Bond& bl = h->bonds[k - 1];
    std::map<std::pair<int, int>, int> key;
    std::vector<int> grp(si.blk.size());
    for (size_t b = 0; b < si.blk.size(); ++b) {
        const XBlk& x = si.blk[b];
        grp[b] = key.emplace(std::make_pair(bl.sec[x.sa].n, kSigmaN[x.s]), int(key.size())).first->second;
    }
    const int ng = int(key.size());
    nb.gptr_h.assign(ng + 1, 0);
    for (int g : grp) ++nb.gptr_h[g + 1];
    for (int g = 0; g < ng; ++g) nb.gptr_h[g + 1] += nb.gptr_h[g];
    nb.roff_h.assign(si.blk.size(), 0);
    nb.rlen_h.assign(si.blk.size(), 0);
    nb.gid_h.assign(size_t(si.size), 0);
    std::vector<int> fill(nb.gptr_h.begin(), nb.gptr_h.end() - 1);
    for (size_t b = 0; b < si.blk.size(); ++b) {  // site order inside a group
        const XBlk& x = si.blk[b];
        const long long len = (long long)x.rows * x.cols;
        const int j = fill[grp[b]]++;
        nb.roff_h[j] = x.off;
        nb.rlen_h[j] = int(len);
        std::fill(nb.gid_h.begin() + x.off, nb.gid_h.begin() + x.off + len, grp[b]);
    }
    nb.gptr.upload(nb.gptr_h, h->stream);
    nb.roff.upload(nb.roff_h, h->stream);
    nb.rlen.upload(nb.rlen_h, h->stream);
    nb.gid.upload(nb.gid_h, h->stream);
    nb.ng = ng;
    return nb;
}

spk::BufSet bufset(sp_handle* h, int k, const double* x, double* y, double* ny, double* out) {
    spk::BufSet b{};
    b.p[B_ENVL] = h->envL[k - 1].p;
    b.p[B_ENVR] = h->envR[k].p;
    b.p[B_X] = const_cast<double*>(x);
    b.p[B_T] = h->T.p;
    b.p[B_V] = h->V.p;
    b.p[B_Y] = y;
    b.p[B_NY] = ny;
    b.p[B_OUT] = out;
    b.p[B_BRA] = const_cast<double*>(x);
    b.p[B_LT] = h->LT.p;
    return b;
}

void check_site(const sp_handle* h, int k) { SP_REQUIRE(k >= 1 && k <= h->L, "site out of range"); }

// the fused-kernel instance descriptor of site k applied to x
// (yp, nyp: the per-g partial slots; null = the handle's own)
spk::H3Inst heff_inst(sp_handle* h, int k, const double* x, bool f32, double* yp = nullptr, double* nyp = nullptr) {
    SitePlan& P = h->plan[k - 1];
    spk::H3Inst I{};
    I.blks = P.dh_blks.p;
    I.cols = P.dh_cols.p;
    I.lsrc = P.dh_lsrc.p;
    I.segs = P.dh_segs.p;
    I.terms = P.dh_terms.p;
    I.pieces = P.dh_pieces.p;
    if (f32) {
        I.Lenv = h->envL32[k - 1].p;
        I.Renv = h->envR32[k].p;
    } else {
        I.Lenv = h->envL[k - 1].p;
        I.Renv = h->envR[k].p;
    }
    I.Lsz = h->env[k - 1].size;
    I.Rsz = h->env[k].size;
    I.x = x;
    I.coef = P.coef.p;
    I.ypart = yp ? yp : h->ypart.p;
    I.nypart = nyp ? nyp : h->nypart.p;
    I.n = h->sites[k - 1].size;
    I.nc = P.nc;
    return I;
}

// H_eff x at a tiled-path site without a fused plan (a particle-number block
// too wide for its LDS): the LDS-tiled block-product lists (FP64, or split
// BF16 in that mode), leaving the same per-g partials as the fused kernel.
// The MPO is mixed into the left environment instead of into the products
// L_g x, and the rotation r_g into the site vector: the pre-mixed
// environment depends only on L[k-1] and is built once per local problem
// (the first product after L[k-1] changes), the rotated site vector (two
// small blocks per particle-number block) with every product, so each
// product is one small mixing launch and two block-product launches.
void heff_tiled(sp_handle* h, int k, const double* x, bool bf3 = false, double* yp = nullptr,
                double* nyp = nullptr) {
    SitePlan& P = h->plan[k - 1];
    hipStream_t s = h->stream;
    if (!yp) yp = h->ypart.p;
    if (!nyp) nyp = h->nypart.p;
    const spk::BufSet b = bufset(h, k, h->Xd.p, yp, nyp, nullptr);
    spk::gather(s, P.xmap.p, x, h->Xd.p, P.Xd_size);
    if (h->lt_site != k || h->lt_gen != h->Lgen[k - 1]) {  // once per left environment and site
        P.premix.launch(s, b, P.coef.p);
        h->lt_site = k;
        h->lt_gen = h->Lgen[k - 1];
    }
    P.xrmix.launch(s, b, P.coef.p);
    P.t_left0.launch(s, b, P.coef.p, P.xmap.p, bf3);
    P.t_leftv.launch(s, b, P.coef.p, P.xmap.p, bf3);
    if (P.tr_split > 1) {  // slots without a chunk of some tile stay zero
        const long long nslot = (long long)P.tr_split * h->G * h->sites[k - 1].size;
        spk::fill(s, yp, nslot, 0.0);
        spk::fill(s, nyp, nslot, 0.0);
    }
    P.t_right.launch(s, b, P.coef.p, P.xmap.p, bf3);
}

// number of per-site partial outputs H_eff x leaves (in G * n blocks of n)
int heff_parts(const sp_handle* h, int k) {
    return (h->path == SP_PATH_TILED && h->plan[k - 1].h_rows == 0) ? h->G * h->plan[k - 1].tr_split : h->G;
}

// With defer_gsum on the tiled path only the per-quadrature-point partials
// (h->ypart, h->nypart) are produced and the function returns true: the
// caller adds them (the Davidson Gram pass does).
// yp, nyp: where the partials go (null = the handle's own slots)
bool heff_apply(sp_handle* h, int k, const double* x, double* y, double* ny, bool defer_gsum = false,
                bool force_fp64 = false, double* yp = nullptr, double* nyp = nullptr) {
    if (!h->Lvalid[k - 1] || !h->Rvalid[k])
        throw SpError(SP_ESTATE, "H_eff needs L[site-1] and R[site+1]; build them with sp_env_update");
    SitePlan& P = h->plan[k - 1];
    hipStream_t s = h->stream;
    if (h->path == SP_PATH_PLAIN) {
        const spk::BufSet b = bufset(h, k, x, y, ny, nullptr);
        P.p1.launch(s, b, P.coef.p);
        P.mixl.launch(s, b, P.coef.p);
        P.yout.launch(s, b, P.coef.p);
        return false;
    }
    const int n = int(h->sites[k - 1].size);
    if (!yp) yp = h->ypart.p;
    if (!nyp) nyp = h->nypart.p;
    if (P.h_rows == 0) {
        heff_tiled(h, k, x, h->precision == SP_BF16X3 && !force_fp64, yp, nyp);
    } else {
        const bool f32 = reduced(h) && !force_fp64;
        const spk::H3Inst I = heff_inst(h, k, x, f32, yp, nyp);
        if (f32) spk::heff3_f32(s, P.h_rows, P.h_lds, P.dh_tasks.p, int(P.h_tasks.size()), I);
        else spk::heff3(s, P.h_rows, P.h_lds, P.dh_tasks.p, int(P.h_tasks.size()), I);
    }
    if (defer_gsum) return true;
    spk::gsum2(s, yp, nyp, n, heff_parts(h, k), n, y, ny);
    return false;
}

void env_left(sp_handle* h, int k) {
    if (!h->Lvalid[k - 1]) throw SpError(SP_ESTATE, "left environment of the previous bond is not built");
    SitePlan& P = h->plan[k - 1];
    hipStream_t s = h->stream;
    if (h->path == SP_PATH_PLAIN) {
        const spk::BufSet b = bufset(h, k, site_ptr(h, k), nullptr, nullptr, h->envL[k].p);
        P.p1.launch(s, b, P.coef.p);
        P.mixl.launch(s, b, P.coef.p);
        P.envl_out.launch(s, b, P.coef.p);
    } else {
        const spk::BufSet b = bufset(h, k, h->Xd.p, nullptr, nullptr, h->envL[k].p);
        spk::gather(s, P.xmap.p, site_ptr(h, k), h->Xd.p, P.Xd_size);
        P.t_left.launch(s, b, P.coef.p, P.xmap.p);
        P.mixl.launch(s, b, P.coef.p);
        P.t_envl.launch(s, b, P.coef.p, P.xmap.p);
    }
    if (reduced(h))
        spk::to_f32(s, h->envL[k].p, h->envL32[k].p, (long long)h->G * h->env[k].size);
    h->Lvalid[k] = 1;
    ++h->Lgen[k];
    if (env_shared(h, k)) h->Rvalid[k] = 0;
    for (int q = k + 1; q <= h->L; ++q) h->Lvalid[q] = 0;
}

void env_right(sp_handle* h, int k) {
    if (!h->Rvalid[k]) throw SpError(SP_ESTATE, "right environment of the next bond is not built");
    SitePlan& P = h->plan[k - 1];
    hipStream_t s = h->stream;
    if (h->path == SP_PATH_PLAIN) {
        const spk::BufSet b = bufset(h, k, site_ptr(h, k), nullptr, nullptr, h->envR[k - 1].p);
        P.p1r.launch(s, b, P.coef.p);
        P.mixr.launch(s, b, P.coef.p);
        P.envr_out.launch(s, b, P.coef.p);
    } else {
        const spk::BufSet b = bufset(h, k, h->Xd.p, nullptr, nullptr, h->envR[k - 1].p);
        spk::gather(s, P.xmap.p, site_ptr(h, k), h->Xd.p, P.Xd_size);
        P.t_zr.launch(s, b, P.coef.p, P.xmap.p);
        P.mixr.launch(s, b, P.coef.p);
        P.t_envr.launch(s, b, P.coef.p, P.xmap.p);
    }
    if (reduced(h))
        spk::to_f32(s, h->envR[k - 1].p, h->envR32[k - 1].p, (long long)h->G * h->env[k - 1].size);
    h->Rvalid[k - 1] = 1;
    if (env_shared(h, k - 1)) h->Lvalid[k - 1] = 0;
    for (int q = 0; q < k - 1; ++q) h->Rvalid[q] = 0;
}

void diag(sp_handle* h, int k, double* dh, double* dn) {
    if (!h->Lvalid[k - 1] || !h->Rvalid[k]) throw SpError(SP_ESTATE, "environments for the diagonal are not built");
    SitePlan& P = h->plan[k - 1];
    const EnvLayout& el = h->env[k - 1];
    const EnvLayout& er = h->env[k];
    // wide MPOs: cut each block's (g, term) range into parts summed in a
    // fixed order, so that a block's thousands of terms run in parallel
    auto split = [&](const std::vector<spk::DiagBlk>& bl) {
        int tmax = 0;
        for (const spk::DiagBlk& d : bl) tmax = std::max(tmax, d.t1 - d.t0);
        const long long u = (long long)h->G * tmax / 1024;
        return int(std::min<long long>(std::max<long long>(u, 1), spk::kDiagSplitMax));
    };
    const long long ntot = h->sites[k - 1].size;
    spk::heff_diag(h->stream, P.ddblk_h.p, int(P.dblk_h.size()), P.ddterm_h.p, h->envL[k - 1].p, el.size,
                   h->envR[k].p, er.size, P.coef.p, P.nc, h->G, dh, split(P.dblk_h), h->diag_part.p, ntot);
    spk::heff_diag(h->stream, P.ddblk_n.p, int(P.dblk_n.size()), P.ddterm_n.p, h->envL[k - 1].p, el.size,
                   h->envR[k].p, er.size, P.coef.p, P.nc, h->G, dn, split(P.dblk_n), h->diag_part.p, ntot);
}

// positive-diagonal QR per right sector of site k, R pushed into site k+1
void move_right(sp_handle* h, int k) {
    SitePlan& P = h->plan[k - 1];
    spk::qr_sectors(h->stream, P.dqr_tasks.p, int(P.qr_tasks.size()), P.dqr_pieces.p, site_ptr(h, k),
                    h->qr_scratch.p, h->qr_r.p, P.qr_lds);
    if (k < h->L) {
        spk::BufSet b{};
        b.p[B_V] = h->qr_r.p;
        b.p[B_X] = site_ptr(h, k + 1);
        b.p[B_OUT] = h->tmp_site.p;
        P.absorb_right.launch(h->stream, b, P.coef.p);
        HIPCK(hipMemcpyAsync(site_ptr(h, k + 1), h->tmp_site.p, h->sites[k].size * sizeof(double),
                             hipMemcpyDeviceToDevice, h->stream));
    }
}

// positive-diagonal LQ per left sector of site k, L pushed into site k-1
void move_left(sp_handle* h, int k) {
    SitePlan& P = h->plan[k - 1];
    spk::qr_sectors(h->stream, P.dlq_tasks.p, int(P.lq_tasks.size()), P.dlq_pieces.p, site_ptr(h, k),
                    h->qr_scratch.p, h->qr_r.p, P.lq_lds);
    if (k > 1) {
        spk::BufSet b{};
        b.p[B_V] = h->qr_r.p;
        b.p[B_X] = site_ptr(h, k - 1);
        b.p[B_OUT] = h->tmp_site.p;
        P.absorb_left.launch(h->stream, b, P.coef.p);
        HIPCK(hipMemcpyAsync(site_ptr(h, k - 1), h->tmp_site.p, h->sites[k - 2].size * sizeof(double),
                             hipMemcpyDeviceToDevice, h->stream));
    }
}

void invalidate_for_site(sp_handle* h, int k) {
    for (int q = k; q <= h->L; ++q) h->Lvalid[q] = 0;
    for (int q = 0; q <= k - 1; ++q) h->Rvalid[q] = 0;
}

// ---------------------------------------------------------------------------
// Davidson for the singular pencil H_eff x = theta N_eff x (Eq. [geproblem])

// Pinned, mapped and coherent host memory: the Davidson kernels read the
// subspace coefficients from it and write their per-chunk partial sums into
// it directly, so an iteration needs no copy in either direction.
// ---------------------------------------------------------------------------
// Orthogonality constraints (Sec. 2.3, Eq. [orthoB]).  A constraint handle
// holds a lower state Psi_0 with the identity MPO on the plain path; its
// environments are rebuilt with this state on the bra side, so that its
// N_eff applied to Psi_0's site tensor k gives B[k] = d<Psi|P|Psi_0>/dA[k]
// in this state's packed layout.

constexpr int kMaxConstraints = 8;

void env_left_mixed(sp_handle* a, int k, const double* bra) {
    SitePlan& P = a->plan[k - 1];
    spk::BufSet b = bufset(a, k, site_ptr(a, k), nullptr, nullptr, a->envL[k].p);
    b.p[B_BRA] = const_cast<double*>(bra);
    P.p1.launch(a->stream, b, P.coef.p);
    P.mixl.launch(a->stream, b, P.coef.p);
    P.envl_out.launch(a->stream, b, P.coef.p);
    a->Lvalid[k] = 1;
    ++a->Lgen[k];
    if (env_shared(a, k)) a->Rvalid[k] = 0;
}

void env_right_mixed(sp_handle* a, int k, const double* bra) {
    SitePlan& P = a->plan[k - 1];
    spk::BufSet b = bufset(a, k, site_ptr(a, k), nullptr, nullptr, a->envR[k - 1].p);
    b.p[B_BRA] = const_cast<double*>(bra);
    P.p1r.launch(a->stream, b, P.coef.p);
    P.mixr.launch(a->stream, b, P.coef.p);
    P.envr_out.launch(a->stream, b, P.coef.p);
    a->Rvalid[k - 1] = 1;
    if (env_shared(a, k - 1)) a->Lvalid[k - 1] = 0;
}

// B[k] of constraint handle a into out (ny: scratch of the site's size)
void constraint_vector(sp_handle* a, int k, double* out, double* ny) {
    SitePlan& P = a->plan[k - 1];
    const spk::BufSet b = bufset(a, k, site_ptr(a, k), out, ny, nullptr);
    P.p1.launch(a->stream, b, P.coef.p);
    P.mixl.launch(a->stream, b, P.coef.p);
    P.yout.launch(a->stream, b, P.coef.p);
}

// u -= C (C^T u) for the con_active orthonormal constraint vectors, twice
// (classical Gram-Schmidt with one reorthogonalisation)
void project_out(sp_handle* h, double* u, int n) {
    const int m = h->con_active;
    if (m == 0) return;
    hipStream_t s = h->stream;
    const int nch = spk::dav_chunks(n);
    double* P1 = h->conPart.p;
    double* P2 = P1 + (size_t)nch * m;
    spk::dav_cgs(s, h->conB.p, h->cld, 0, m, P1, nch, u, n, P1, 0);  // dots only
    spk::dav_cgs(s, h->conB.p, h->cld, m, m, P1, nch, u, n, P2, 0);  // subtract, dots again
    spk::dav_cgs(s, h->conB.p, h->cld, m, 0, P2, nch, u, n, P1, 0);  // subtract
}

// the orthonormal constraint vectors at site k: B[k] of every constraint in
// order, each orthogonalised against the ones kept before it and dropped
// when its remainder is below 1e-10 of its own norm
void prepare_constraints(sp_handle* h, int k) {
    h->con_active = 0;
    if (h->cons.empty()) return;
    hipStream_t s = h->stream;
    const int n = int(h->sites[k - 1].size);
    const int nch = spk::dav_chunks(n);
    double* p0 = h->con_pin_dev;  // raw norm partials
    double* p1 = p0 + nch;        // norm partials after the projection
    for (auto& a : h->cons) {
        double* row = h->conB.p + (size_t)h->con_active * h->cld;
        constraint_vector(a.get(), k, row, h->tmp_site.p);
        spk::dav_cgs(s, h->conB.p, h->cld, 0, 0, p0, nch, row, n, p0, 1);  // |B|^2 partials
        project_out(h, row, n);
        spk::dav_cgs(s, h->conB.p, h->cld, 0, 0, p1, nch, row, n, p1, 1);
        HIPCK(hipStreamSynchronize(s));
        double n0 = 0.0, n1 = 0.0;
        for (int q = 0; q < nch; ++q) {
            n0 += h->con_pin[q];
            n1 += h->con_pin[nch + q];
        }
        if (!(n0 > 0.0) || !(n1 > 1e-20 * n0)) continue;  // dependent on the kept vectors
        spk::dav_normalize(s, p1, nch, row, row, n, p0 + 2 * nch);
        h->con_active++;
    }
}

void ensure_pinned(sp_handle* h, size_t n, size_t n_up) {
    const unsigned flags = hipHostMallocMapped | hipHostMallocCoherent;
    if (h->pin_n < n) {
        if (h->pin) HIPCK(hipHostFree(h->pin));
        h->pin = nullptr;
        h->pin_dev = nullptr;
        HIPCK(hipHostMalloc(&h->pin, n * sizeof(double), flags));
        HIPCK(hipHostGetDevicePointer((void**)&h->pin_dev, h->pin, 0));
        h->pin_n = n;
    }
    if (h->pin_up_n < n_up) {
        if (h->pin_up) HIPCK(hipHostFree(h->pin_up));
        h->pin_up = nullptr;
        h->pin_up_dev = nullptr;
        HIPCK(hipHostMalloc(&h->pin_up, n_up * sizeof(double), flags));
        HIPCK(hipHostGetDevicePointer((void**)&h->pin_up_dev, h->pin_up, 0));
        h->pin_up_n = n_up;
    }
}

// device small area of the Davidson solve (offsets in doubles)
struct DavLayout {
    long long a, theta, q, pc1, pc2, pn, out, tn, px, pg, total;
    DavLayout(int max_sub, int nch) {
        a = 0;
        theta = max_sub + 2;
        q = max_sub + 4;
        pc1 = q + (long long)max_sub * max_sub;
        pc2 = pc1 + (long long)nch * max_sub;
        pn = pc2 + (long long)nch * max_sub;
        out = pn + nch;
        tn = out;
        px = out + 1;
        pg = px + 3LL * nch;
        total = pg + (long long)nch * (4 * max_sub + 2) + 8;
    }
};

void ensure_davidson(sp_handle* h, int max_sub) {
    if (h->dav_sub >= max_sub && h->ld > 0) return;
    SP_REQUIRE(max_sub + 1 <= spk::kDavMaxVec, "max_sub too large");
    h->ld = (h->max_site + 63) / 64 * 64;
    const size_t vec = size_t(max_sub + 1) * h->ld;
    h->dV.alloc(vec);
    h->dHV.alloc(vec);
    h->dNV.alloc(vec);
    h->dRot.alloc(size_t(max_sub + 1) * h->ld);
    h->dx.alloc(h->ld);
    h->dt.alloc(h->ld);
    h->ddh.alloc(h->ld);
    h->ddn.alloc(h->ld);
    const int nch = spk::dav_chunks(int(h->ld));
    const DavLayout lay(max_sub, nch);
    h->dsmall.alloc(lay.total);
    h->dHt.alloc(size_t(max_sub + 1) * (max_sub + 1));
    h->dNt.alloc(size_t(max_sub + 1) * (max_sub + 1));
    h->dav_sub = max_sub;
    ensure_pinned(h, lay.total - lay.out + 8, lay.pc1 + 8);
}

// tot[i] = the sum over chunks q < nch of part[q * stride + i], i < stride,
// each in ascending q, read from the chunk-major partials in one contiguous
// pass (the same sums as chunk by chunk per i, without the strided reads)
void chunk_totals(const double* part, int nch, int stride, double* tot) {
    for (int i = 0; i < stride; ++i) tot[i] = 0.0;
    for (int q = 0; q < nch; ++q) {
        const double* row = part + (size_t)q * stride;
        for (int i = 0; i < stride; ++i) tot[i] += row[i];
    }
}

struct DavOut {
    double theta = 0, rnorm = 0, pnorm = 0;
    int iters = 0, matvecs = 0;
    bool converged = false;
};

// lowest eigenpair of the pencil restricted to range(Nt) (canonical
// orthogonalisation); returns false if the projected metric vanishes.  gp
// (may be null) keeps the reduction of the pencil between the calls of one
// solve, which grows it by one row and column per call until a restart
bool small_solve(int m, const std::vector<double>& Ht, const std::vector<double>& Nt, int stride, double drop,
                 bool need_all, double& theta, std::vector<double>& a, std::vector<double>& Xc, int& rk,
                 sph::GrowingPencil* gp) {
    std::vector<double> Hs(size_t(m) * m), Ns(size_t(m) * m);
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) {
            Hs[size_t(i) * m + j] = 0.5 * (Ht[size_t(i) * stride + j] + Ht[size_t(j) * stride + i]);
            Ns[size_t(i) * m + j] = 0.5 * (Nt[size_t(i) * stride + j] + Nt[size_t(j) * stride + i]);
        }
    a.assign(m, 0.0);
    if (gp && need_all) gp->reset();
    if (gp && !need_all) {
        const int r = gp->lowest(m, Hs.data(), Ns.data(), drop, &theta, a.data());
        if (r == -1) throw SpError(SP_ENAN, "subspace eigensolver failed");
        if (r == m) {
            if (!std::isfinite(theta)) throw SpError(SP_ENAN, "non-finite Ritz value");
            rk = m;
            return true;
        }
        a.assign(m, 0.0);
    }
    if (need_all) Xc.assign(size_t(m) * m, 0.0);
    const int r = sph::gen_lowest(m, Hs.data(), Ns.data(), drop, &theta, a.data(), need_all ? Xc.data() : nullptr, &rk);
    if (r < 0) throw SpError(SP_ENAN, "subspace eigensolver failed");
    if (r == 0) return false;
    if (!std::isfinite(theta)) throw SpError(SP_ENAN, "non-finite Ritz value");
    if (need_all) Xc.resize(size_t(m) * rk);
    return true;
}

// FP64 Rayleigh quotient at site k for the device vector x (any norm):
// theta = x.H_eff x / x.N_eff x, pnorm = x.N_eff x / x.x; uses dHV[0], dNV[0]
void rayleigh64(sp_handle* h, int k, const double* x, double& theta, double& pnorm, double& xx_out) {
    const int n = int(h->sites[k - 1].size);
    heff_apply(h, k, x, h->dHV.p, h->dNV.p, false, true);
    double* sm = h->dsmall.p;
    spk::multidot(h->stream, h->dHV.p, 0, 1, x, n, sm);
    spk::multidot(h->stream, h->dNV.p, 0, 1, x, n, sm + 1);
    spk::multidot(h->stream, x, 0, 1, x, n, sm + 2);
    HIPCK(hipMemcpyAsync(h->pin, sm, 3 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPCK(hipStreamSynchronize(h->stream));
    const double xy = h->pin[0], xny = h->pin[1], xx = h->pin[2];
    xx_out = xx;
    theta = xy / xny;
    pnorm = xx > 0.0 ? xny / xx : 0.0;
}

DavOut davidson(sp_handle* h, int k, const sp_sweep_opts& o) {
    const int n = int(h->sites[k - 1].size);
    const int max_sub = std::max(2, o.max_sub);
    const int keep = std::max(1, std::min(o.keep, max_sub - 1));
    const int max_iter = std::max(1, o.max_iter);
    ensure_davidson(h, max_sub);
    hipStream_t s = h->stream;
    const long long ld = h->ld;
    double* V = h->dV.p;
    double* HV = h->dHV.p;
    double* NV = h->dNV.p;
    const int nch = spk::dav_chunks(n);
    const DavLayout lay(h->dav_sub, spk::dav_chunks(int(ld)));
    double* sm = h->dsmall.p;
    double* up = h->pin_up;
    double* dn = h->pin;
    double* dn_dev = h->pin_dev;  // device view of dn: partial sums land here
    // new vector mm: on the tiled path H_eff is applied to the unnormalised
    // correction t (or V_0 for mm = 0) and the Gram pass normalises V_mm,
    // HV_mm and NV_mm; the plain path normalises first
    auto extend = [&](int mm, bool from_t) {
        double* vm = V + size_t(mm) * ld;
        double* tn = dn_dev + (lay.tn - lay.out);
        if (h->path == SP_PATH_PLAIN) {
            if (from_t) spk::dav_normalize(s, sm + lay.pn, nch, h->dt.p, vm, n, tn);
            heff_apply(h, k, vm, HV + size_t(mm) * ld, NV + size_t(mm) * ld);
            spk::dav_gram(s, V, HV, NV, ld, mm, n, nullptr, nullptr, 0, nullptr, nullptr, nullptr, n, h->G,
                          dn_dev + (lay.pg - lay.out));
        } else {
            heff_apply(h, k, from_t ? h->dt.p : vm, nullptr, nullptr, true);
            spk::dav_gram(s, V, HV, NV, ld, mm, n, from_t ? h->dt.p : nullptr, sm + lay.pn, nch, tn, h->ypart.p,
                          h->nypart.p, n, heff_parts(h, k), dn_dev + (lay.pg - lay.out));
        }
        // constrained pencil (Q H Q, Q N Q): the Gram rows above are the same
        // for the projected products, since every V_j is orthogonal to C
        project_out(h, HV + size_t(mm) * ld, n);
        project_out(h, NV + size_t(mm) * ld, n);
    };
    // canonical orthogonalisation threshold: with FP32 products the null
    // space of the projected metric is only resolved to about 1e-7 of its
    // largest eigenvalue, so directions below 1e-5 are dropped there
    const double drop = metric_drop(h), floor_ = 1e-8;
    DavOut out;
    // fixed-order sums of per-chunk partials (host side)
    auto chunk_total = [&](const double* part, int stride, int idx) {
        double acc = 0.0;
        for (int q = 0; q < nch; ++q) acc += part[(size_t)q * stride + idx];
        return acc;
    };

    // learned preconditioner: corrections from the model while the residual
    // keeps reaching new minima and halves at least every four iterations
    // (abandoned for the rest of the solve otherwise); training pairs
    // recorded for every iteration of a converged solve
    sp_mlp* use = h->mlp_use;
    sp_mlp* rec = h->mlp_rec;
    bool use_model = use != nullptr;
    double best_r = INFINITY;
    std::vector<double> rhist;
    int stall = 0, nrec = 0, rec_last_it = 0;
    const long long rec_base = rec ? rec->rows : 0;
    if (rec && h->xrec.n < size_t(max_iter) * ld) h->xrec.alloc(size_t(max_iter) * ld);
    if ((use || rec) && h->mlp_scal.n < 4) h->mlp_scal.alloc(4);
    SP_REQUIRE(!use || !rec || use->scope == rec->scope, "the model in use and the recording one differ in scope");
    const NBlocks* nbk = ((use && use->scope == SP_MLP_NBLOCK) || (rec && rec->scope == SP_MLP_NBLOCK))
                             ? &site_nblocks(h, k)
                             : nullptr;
    if (nbk && h->mlp_grms.n < size_t(2 * nbk->ng)) h->mlp_grms.alloc(2 * nbk->ng);
    if (nbk && rec && h->mlp_tscal.n < size_t(2 * max_iter)) h->mlp_tscal.alloc(2 * max_iter);
    diag(h, k, h->ddh.p, h->ddn.p);
    spk::normalize(s, site_ptr(h, k), V, n, nullptr);
    if (h->con_active) {  // start in the complement of the constraints
        project_out(h, V, n);
        spk::normalize(s, V, V, n, nullptr);
    }
    extend(0, false);
    out.matvecs = 1;
    HIPCK(hipStreamSynchronize(s));
    const int S = max_sub + 1;
    std::vector<double> Ht(size_t(S) * S, 0.0), Nt(size_t(S) * S, 0.0);
    Ht[0] = chunk_total(dn + (lay.pg - lay.out), 2, 0);
    Nt[0] = chunk_total(dn + (lay.pg - lay.out), 2, 1);
    int m = 1;
    std::vector<double> a, Xc, gt;
    sph::GrowingPencil gp;
    for (int it = 1; it <= max_iter; ++it) {
        out.iters = it;
        double theta;
        int rk = 0;
        const bool last = (it == max_iter);
        const bool restart = !last && m >= max_sub;
        if (!small_solve(m, Ht, Nt, S, drop, restart, theta, a, Xc, rk, &gp))
            throw SpError(SP_ENORM, "projected norm vanishes in the search space");
        out.theta = theta;
        int nk = 0;
        std::vector<double> Qk;
        if (restart) {
            // the lowest Ritz vectors, Euclidean-orthonormalised (modified
            // Gram-Schmidt on their coefficient vectors)
            nk = std::min(keep, rk);
            Qk.assign(size_t(m) * nk, 0.0);
            for (int c = 0; c < nk; ++c) {
                std::vector<double> v(m);
                for (int i = 0; i < m; ++i) v[i] = Xc[i * rk + c];
                for (int p = 0; p < c; ++p) {
                    double d = 0.0;
                    for (int i = 0; i < m; ++i) d += Qk[i * nk + p] * v[i];
                    for (int i = 0; i < m; ++i) v[i] -= d * Qk[i * nk + p];
                }
                double nr = 0.0;
                for (int i = 0; i < m; ++i) nr += v[i] * v[i];
                nr = std::sqrt(nr);
                for (int i = 0; i < m; ++i) Qk[i * nk + c] = v[i] / nr;
            }
        }
        // a and theta are read by the Ritz kernel straight from mapped host
        // memory; the restart rotation is copied to the device
        for (int i = 0; i < m; ++i) up[lay.a + i] = a[i];
        up[lay.a + m] = theta;
        if (restart) {
            std::copy(Qk.begin(), Qk.end(), up + lay.q);
            HIPCK(hipMemcpyAsync(sm + lay.q, up + lay.q, Qk.size() * sizeof(double), hipMemcpyHostToDevice, s));
        }
        spk::dav_ritz(s, V, HV, NV, ld, m, h->pin_up_dev + lay.a, h->ddh.p, h->ddn.p, n, floor_, h->dx.p, h->dt.p,
                      dn_dev + (lay.px - lay.out), sm + lay.pc1);
        if (!last) {
            const bool record_now = rec && rec_base + (long long)(nrec + 1) * n <= rec->cap;
            if (use_model || record_now) {
                if (nbk) {
                    spk::mlp_group_rms(s, h->dt.p, h->ddh.p, h->ddn.p, h->pin_up_dev + lay.a + m, floor_,
                                       nbk->groups(), h->mlp_grms.p);
                } else {
                    spk::sum_partials(s, dn_dev + (lay.px - lay.out), nch, 3, 1, h->mlp_scal.p);
                    spk::sumsq(s, h->dt.p, n, h->mlp_scal.p + 1);
                }
                spk::mlp_apply_grouped(
                    s, use_model ? use->w.p : nullptr, use ? use->hidden : 0, h->dt.p, h->ddh.p, h->ddn.p,
                    h->pin_up_dev + lay.a + m, h->mlp_scal.p, h->mlp_scal.p + 1, n, floor_,
                    record_now ? rec->F.p + (rec_base + (long long)nrec * n) * spk::kMlpIn : nullptr,
                    record_now ? rec->Y.p + rec_base + (long long)nrec * n : nullptr, nbk ? nbk->gid.p : nullptr,
                    nbk ? h->mlp_grms.p : nullptr);
                if (record_now) {
                    HIPCK(hipMemcpyAsync(h->xrec.p + size_t(nrec) * ld, h->dx.p, size_t(n) * sizeof(double),
                                         hipMemcpyDeviceToDevice, s));
                    ++nrec;
                    rec_last_it = it;
                }
                // the dots of the new correction with the search space
                if (use_model) spk::dav_cgs(s, V, ld, 0, m, sm + lay.pc1, nch, h->dt.p, n, sm + lay.pc1, 0);
            }
            // the correction stays in the complement of the constraints (its
            // dots with V are unchanged, V being orthogonal to them)
            project_out(h, h->dt.p, n);
            if (restart) {
                for (double* B : {V, HV, NV}) {
                    spk::basis_rotate(s, B, ld, m, sm + lay.q, nk, h->dRot.p, n);
                    HIPCK(hipMemcpyAsync(B, h->dRot.p, size_t(nk) * ld * sizeof(double), hipMemcpyDeviceToDevice, s));
                }
                auto rot = [&](std::vector<double>& M) {
                    std::vector<double> tmp(size_t(m) * nk, 0.0), res(size_t(S) * S, 0.0);
                    for (int i = 0; i < m; ++i)
                        for (int c = 0; c < nk; ++c) {
                            double v = 0.0;
                            for (int j = 0; j < m; ++j) v += M[i * S + j] * Qk[j * nk + c];
                            tmp[i * nk + c] = v;
                        }
                    for (int r = 0; r < nk; ++r)
                        for (int c = 0; c < nk; ++c) {
                            double v = 0.0;
                            for (int i = 0; i < m; ++i) v += Qk[i * nk + r] * tmp[i * nk + c];
                            res[r * S + c] = v;
                        }
                    M.swap(res);
                };
                rot(Ht);
                rot(Nt);
                m = nk;
                // the first projections must be taken against the new basis
                spk::dav_cgs(s, V, ld, 0, m, sm + lay.pc2, nch, h->dt.p, n, sm + lay.pc1, 0);
            }
            // CGS2 of the correction against the search space, then normalise
            spk::dav_cgs(s, V, ld, m, m, sm + lay.pc1, nch, h->dt.p, n, sm + lay.pc2, 0);
            spk::dav_cgs(s, V, ld, m, 0, sm + lay.pc2, nch, h->dt.p, n, sm + lay.pn, 1);
            extend(m, true);
            out.matvecs++;
        }
        HIPCK(hipStreamSynchronize(s));
        double xt[3];
        chunk_totals(dn + (lay.px - lay.out), nch, 3, xt);
        const double xx = xt[0], uu = xt[1], xn = xt[2];
        if (!std::isfinite(xx) || !std::isfinite(uu) || !(xx > 0.0)) throw SpError(SP_ENAN, "non-finite Ritz vector");
        out.rnorm = std::sqrt(uu / xx);
        out.pnorm = xn / xx;
        if (out.rnorm <= o.tol) {
            out.converged = true;
            break;
        }
        if (use_model) {
            if (out.rnorm < best_r) {
                best_r = out.rnorm;
                stall = 0;
            } else {
                ++stall;
            }
            rhist.push_back(out.rnorm);
            const size_t nh = rhist.size();
            const bool slow = nh >= 5 && out.rnorm > 0.5 * rhist[nh - 5];
            if (stall >= 3 || slow) use_model = false;
        }
        if (last) break;
        const double tn = dn[lay.tn - lay.out];
        if (!(tn >= 1e-14)) break;
        // extend the projected matrices with the new vector m
        const int nd = 4 * m + 2;
        gt.resize(nd);
        chunk_totals(dn + (lay.pg - lay.out), nch, nd, gt.data());
        for (int j = 0; j <= m; ++j) {
            const double hv_new = gt[j];          // V_j . HV_m
            const double nv_new = gt[m + 1 + j];  // V_j . NV_m
            const double hv_old = (j < m) ? gt[2 * m + 2 + j] : hv_new;  // V_m . HV_j
            const double nv_old = (j < m) ? gt[3 * m + 2 + j] : nv_new;
            Ht[j * S + m] = hv_new;
            Ht[m * S + j] = hv_old;
            Nt[j * S + m] = nv_new;
            Nt[m * S + j] = nv_old;
        }
        ++m;
    }
    // normalise x and write it into the site
    spk::normalize(s, h->dx.p, site_ptr(h, k), n, nullptr);
    if (rec && out.converged && nrec > 0) {
        // iterations before the converged one: targets against the final x
        const int keep = nrec - (rec_last_it == out.iters ? 1 : 0);
        if (nbk)
            spk::mlp_targets_grouped(s, h->xrec.p, ld, keep, site_ptr(h, k), n, nbk->groups(), h->mlp_tscal.p,
                                     rec->Y.p + rec_base);
        else
            spk::mlp_targets(s, h->xrec.p, ld, keep, site_ptr(h, k), n, rec->Y.p + rec_base);
        rec->rows = rec_base + (long long)keep * n;
    }
    if (reduced(h)) {
        // the reported energy and norm: one FP64 product with the FP64
        // environments (the vector itself comes from the FP32 solve)
        double th, pn, xx;
        rayleigh64(h, k, site_ptr(h, k), th, pn, xx);
        if (!std::isfinite(th)) throw SpError(SP_ENAN, "non-finite Rayleigh quotient");
        out.theta = th;
        out.pnorm = pn;
    }
    return out;
}

// ---------------------------------------------------------------------------
// Batched sweeps: many SP-MPS states advanced together, one site step of
// each per round.  Within a round the Davidson iterations of all states run
// in lockstep: their subspace solves on a host thread pool, then one Ritz,
// two CGS and one Gram launch for all of them and one fused H_eff launch
// per row count (every state's quadrature points in the same launch).

class Pool {
  public:
    explicit Pool(int n) {
        for (int i = 0; i < n; ++i) th_.emplace_back([this] { loop(); });
    }
    ~Pool() {
        {
            std::lock_guard<std::mutex> l(mu_);
            stop_ = true;
        }
        cv_.notify_all();
        for (auto& t : th_) t.join();
    }
    // fn(i) for i < n on the pool and the calling thread
    void run(int n, const std::function<void(int)>& fn) {
        if (th_.empty() || n <= 1) {
            for (int i = 0; i < n; ++i) fn(i);
            return;
        }
        {
            std::lock_guard<std::mutex> l(mu_);
            job_ = &fn;
            njobs_ = n;
            next_ = 0;
            ++gen_;
        }
        cv_.notify_all();
        for (int i = next_.fetch_add(1); i < n; i = next_.fetch_add(1)) fn(i);
        std::unique_lock<std::mutex> l(mu_);
        done_.wait(l, [&] { return busy_ == 0; });
        job_ = nullptr;
    }

  private:
    void loop() {
        long seen = 0;
        for (;;) {
            const std::function<void(int)>* fn;
            int nj;
            {
                std::unique_lock<std::mutex> l(mu_);
                cv_.wait(l, [&] { return stop_ || gen_ != seen; });
                if (stop_) return;
                seen = gen_;
                fn = job_;
                nj = njobs_;
                if (!fn) continue;
                ++busy_;
            }
            for (int i = next_.fetch_add(1); i < nj; i = next_.fetch_add(1)) (*fn)(i);
            {
                std::lock_guard<std::mutex> l(mu_);
                if (--busy_ == 0) done_.notify_all();
            }
        }
    }
    std::vector<std::thread> th_;
    std::mutex mu_;
    std::condition_variable cv_, done_;
    const std::function<void(int)>* job_ = nullptr;
    int njobs_ = 0, busy_ = 0;
    std::atomic<int> next_{0};
    long gen_ = 0;
    bool stop_ = false;
};

struct BatchState {
    sph::GrowingPencil gp;  // reduction of the growing subspace pencil
    sp_handle* h = nullptr;
    std::vector<std::pair<int, int>> order;  // (site, dir) of every step
    size_t step = 0;
    int sweep_len = 1;
    // Davidson state of the current step
    int k = 0, n = 0, nch = 0, m = 0, it = 0, rk = 0, nk = 0;
    bool last = false, restart = false;
    double theta = 0;
    std::vector<double> Ht, Nt, a, Xc, Qk;
    DavOut out;
    std::chrono::steady_clock::time_point t0;
    std::string err;
    int err_code = 0;
};

struct BatchBufs {
    DArr<spk::H3Task> tasks;
    DArr<spk::H3Inst> insts;
    DArr<spk::DavInst> dav;
    double* pin = nullptr;  // staging of the per-round uploads
    size_t pin_n = 0;
    ~BatchBufs() {
        if (pin) (void)hipHostFree(pin);
    }
    double* staging(size_t bytes) {
        const size_t n = (bytes + 7) / 8;
        if (pin_n < n) {
            if (pin) HIPCK(hipHostFree(pin));
            pin = nullptr;
            HIPCK(hipHostMalloc(&pin, n * 8, hipHostMallocDefault));
            pin_n = n;
        }
        return pin;
    }
};

// one fused H_eff application for every state in `idx` (tiled path), with
// x = V_0 where from_v0[i] else t; outputs stay as per-g partials in each
// handle.  The staging buffer is rewritten by the next call only after the
// caller has synchronised the stream (once per round).
void batch_heff_mixed(std::vector<BatchState>& B, const std::vector<int>& idx, const std::vector<int>& from_v0,
                      BatchBufs& bb, hipStream_t s) {
    if (idx.empty()) return;
    std::vector<spk::H3Inst> insts(idx.size());
    std::map<int, std::vector<spk::H3Task>> by_rc;
    std::map<int, int> lds_by_rc;
    const bool f32 = reduced(B[idx[0]].h);
    for (size_t q = 0; q < idx.size(); ++q) {
        BatchState& st = B[idx[q]];
        sp_handle* h = st.h;
        const double* x = from_v0[idx[q]] ? h->dV.p : h->dt.p;
        insts[q] = heff_inst(h, st.k, x, f32);
        const SitePlan& P = h->plan[st.k - 1];
        if (P.h_rows == 0) {  // no fused plan: this state's tiled lists, same partials
            heff_tiled(h, st.k, x, h->precision == SP_BF16X3);
            continue;
        }
        auto& v = by_rc[P.h_rows];
        for (spk::H3Task t : P.h_tasks) {
            if (t.blk < 0) continue;
            t.inst = int(q);
            v.push_back(t);
        }
        lds_by_rc[P.h_rows] = std::max(lds_by_rc[P.h_rows], P.h_lds);
    }
    size_t ntask = 0;
    for (auto& kv : by_rc) ntask += kv.second.size();
    const size_t bytes = insts.size() * sizeof(spk::H3Inst) + ntask * sizeof(spk::H3Task);
    char* stage = reinterpret_cast<char*>(bb.staging(bytes));
    std::memcpy(stage, insts.data(), insts.size() * sizeof(spk::H3Inst));
    size_t off = insts.size() * sizeof(spk::H3Inst);
    for (auto& kv : by_rc) {
        std::memcpy(stage + off, kv.second.data(), kv.second.size() * sizeof(spk::H3Task));
        off += kv.second.size() * sizeof(spk::H3Task);
    }
    if (bb.insts.n < insts.size()) bb.insts.alloc(insts.size());
    if (bb.tasks.n < ntask) bb.tasks.alloc(ntask);
    HIPCK(hipMemcpyAsync(bb.insts.p, stage, insts.size() * sizeof(spk::H3Inst), hipMemcpyHostToDevice, s));
    HIPCK(hipMemcpyAsync(bb.tasks.p, stage + insts.size() * sizeof(spk::H3Inst), ntask * sizeof(spk::H3Task),
                         hipMemcpyHostToDevice, s));
    size_t t0 = 0;
    for (auto& kv : by_rc) {
        const int nt = int(kv.second.size());
        if (f32) spk::heff3_f32(s, kv.first, lds_by_rc[kv.first], bb.tasks.p + t0, nt, insts[0], bb.insts.p);
        else spk::heff3(s, kv.first, lds_by_rc[kv.first], bb.tasks.p + t0, nt, insts[0], bb.insts.p);
        t0 += nt;
    }
}

void batch_dav_upload(std::vector<spk::DavInst>& D, BatchBufs& bb, hipStream_t s) {
    if (bb.dav.n < D.size()) bb.dav.alloc(D.size());
    HIPCK(hipMemcpyAsync(bb.dav.p, D.data(), D.size() * sizeof(spk::DavInst), hipMemcpyHostToDevice, s));
}

spk::DavInst dav_inst(BatchState& st) {
    sp_handle* h = st.h;
    const long long ld = h->ld;
    const DavLayout lay(h->dav_sub, spk::dav_chunks(int(ld)));
    double* sm = h->dsmall.p;
    double* dn_dev = h->pin_dev;
    spk::DavInst I{};
    I.V = h->dV.p;
    I.HV = h->dHV.p;
    I.NV = h->dNV.p;
    I.ld = ld;
    I.aq = h->pin_up_dev + lay.a;
    I.dh = h->ddh.p;
    I.dn = h->ddn.p;
    I.floor_ = 1e-8;
    I.x = h->dx.p;
    I.t = h->dt.p;
    I.part_x = dn_dev + (lay.px - lay.out);
    I.pc1 = sm + lay.pc1;
    I.pc2 = sm + lay.pc2;
    I.pn = sm + lay.pn;
    I.pg = dn_dev + (lay.pg - lay.out);
    I.tnorm = dn_dev + (lay.tn - lay.out);
    I.ypart = h->ypart.p;
    I.nypart = h->nypart.p;
    I.gstride = st.n;
    I.G = heff_parts(h, st.k);
    I.m = st.m;
    I.mr = st.m;
    I.n = st.n;
    I.active = 1;
    I.ext = 1;
    I.from_t = 1;
    return I;
}

// A finished site step: into the caller's report (while it has room) and,
// when asked, one line on stderr.
void record_step(sp_sweep_report* r, int verbose, int state, const sp_step_report& st) {
    if (r && r->steps && r->n_steps < r->capacity) r->steps[r->n_steps++] = st;
    if (verbose)
        std::fprintf(stderr, "[sp_sweep] state %d sweep %d site %d dir %+d: theta %.12f, %d matvecs%s, %.1f ms\n",
                     state, st.sweep, st.site, st.dir, st.theta, st.matvecs, st.converged ? "" : " (not converged)",
                     st.usec * 1e-3);
}

// One Davidson iteration of every running state per round (states are not
// aligned on site steps: a state that finishes its local solve moves its
// gauge, updates its environments and starts its next step at once).
int sweep_batch(std::vector<BatchState>& B, const sp_sweep_opts& o, std::vector<sp_sweep_report*>& reps) {
    hipStream_t s = B[0].h->stream;
    const int max_sub = std::max(2, o.max_sub);
    const int keep = std::max(1, std::min(o.keep, max_sub - 1));
    const int max_iter = std::max(1, o.max_iter);
    const int S = max_sub + 1;
    BatchBufs bb;
    const int nthreads =
        std::max(0, std::min<int>(int(B.size()), std::min(16u, std::thread::hardware_concurrency())) - 1);
    Pool pool(nthreads);
    int status = SP_OK;
    for (auto& st : B) ensure_davidson(st.h, max_sub);
    auto chunk_total = [](const double* part, int nch, int stride, int idx) {
        double acc = 0.0;
        for (int q = 0; q < nch; ++q) acc += part[(size_t)q * stride + idx];
        return acc;
    };
    // phase: 0 = start a step, 1 = Davidson iterations, 2 = done
    std::vector<int> phase(B.size());
    for (size_t i = 0; i < B.size(); ++i) phase[i] = B[i].order.empty() ? 2 : 0;
    std::vector<spk::H3Inst> hinst;
    for (;;) {
        std::vector<int> starting, iterating;
        for (size_t i = 0; i < B.size(); ++i) {
            if (phase[i] == 0) starting.push_back(int(i));
            else if (phase[i] == 1) iterating.push_back(int(i));
        }
        if (starting.empty() && iterating.empty()) break;
        // step start: diagonal and V_0
        for (int i : starting) {
            BatchState& st = B[i];
            sp_handle* h = st.h;
            st.k = st.order[st.step].first;
            st.n = int(h->sites[st.k - 1].size);
            st.nch = spk::dav_chunks(st.n);
            st.m = 0;
            st.it = 0;
            st.out = DavOut{};
            st.t0 = std::chrono::steady_clock::now();
            st.Ht.assign(size_t(S) * S, 0.0);
            st.Nt.assign(size_t(S) * S, 0.0);
            diag(h, st.k, h->ddh.p, h->ddn.p);
            spk::normalize(s, site_ptr(h, st.k), h->dV.p, st.n, nullptr);
        }
        // subspace solves of the iterating states
        pool.run(int(iterating.size()), [&](int q) {
            BatchState& st = B[iterating[q]];
            try {
                st.it += 1;
                st.out.iters = st.it;
                st.last = (st.it == max_iter);
                st.restart = !st.last && st.m >= max_sub;
                const double drop = metric_drop(st.h);
                if (!small_solve(st.m, st.Ht, st.Nt, S, drop, st.restart, st.theta, st.a, st.Xc, st.rk, &st.gp))
                    throw SpError(SP_ENORM, "projected norm vanishes in the search space");
                st.out.theta = st.theta;
                st.nk = 0;
                if (st.restart) {
                    const int m = st.m;
                    st.nk = std::min(keep, st.rk);
                    st.Qk.assign(size_t(m) * st.nk, 0.0);
                    for (int c = 0; c < st.nk; ++c) {
                        std::vector<double> v(m);
                        for (int r = 0; r < m; ++r) v[r] = st.Xc[r * st.rk + c];
                        for (int p = 0; p < c; ++p) {
                            double d = 0.0;
                            for (int r = 0; r < m; ++r) d += st.Qk[r * st.nk + p] * v[r];
                            for (int r = 0; r < m; ++r) v[r] -= d * st.Qk[r * st.nk + p];
                        }
                        double nr = 0.0;
                        for (int r = 0; r < m; ++r) nr += v[r] * v[r];
                        nr = std::sqrt(nr);
                        for (int r = 0; r < m; ++r) st.Qk[r * st.nk + c] = v[r] / nr;
                    }
                }
                sp_handle* h = st.h;
                const DavLayout lay(h->dav_sub, spk::dav_chunks(int(h->ld)));
                for (int r = 0; r < st.m; ++r) h->pin_up[lay.a + r] = st.a[r];
                h->pin_up[lay.a + st.m] = st.theta;
                if (st.restart) std::copy(st.Qk.begin(), st.Qk.end(), h->pin_up + lay.q);
            } catch (const SpError& e) {
                st.err = e.what();
                st.err_code = e.code;
            }
        });
        for (int i : iterating)
            if (B[i].err_code) throw SpError(B[i].err_code, B[i].err);
        std::vector<spk::DavInst> D;
        int max_n = 0, max_m = 0;
        if (!iterating.empty()) {
            for (int i : iterating) {
                D.push_back(dav_inst(B[i]));
                max_n = std::max(max_n, B[i].n);
            }
            batch_dav_upload(D, bb, s);
            spk::bdav_ritz(s, bb.dav.p, int(D.size()), max_n);
        }
        std::vector<int> ext;
        for (int i : iterating) {
            BatchState& st = B[i];
            if (st.last) continue;
            ext.push_back(i);
            st.out.matvecs++;
            if (!st.restart) continue;
            sp_handle* h = st.h;
            const long long ld = h->ld;
            const DavLayout lay(h->dav_sub, spk::dav_chunks(int(ld)));
            double* sm = h->dsmall.p;
            HIPCK(hipMemcpyAsync(sm + lay.q, h->pin_up + lay.q, st.Qk.size() * sizeof(double), hipMemcpyHostToDevice,
                                 s));
            for (double* Bv : {h->dV.p, h->dHV.p, h->dNV.p}) {
                spk::basis_rotate(s, Bv, ld, st.m, sm + lay.q, st.nk, h->dRot.p, st.n);
                HIPCK(hipMemcpyAsync(Bv, h->dRot.p, size_t(st.nk) * ld * sizeof(double), hipMemcpyDeviceToDevice, s));
            }
            const int m = st.m, nk = st.nk;
            auto rot = [&](std::vector<double>& M) {
                std::vector<double> tmp(size_t(m) * nk, 0.0), res(size_t(S) * S, 0.0);
                for (int r = 0; r < m; ++r)
                    for (int c = 0; c < nk; ++c) {
                        double v = 0.0;
                        for (int j = 0; j < m; ++j) v += M[r * S + j] * st.Qk[j * nk + c];
                        tmp[r * nk + c] = v;
                    }
                for (int r = 0; r < nk; ++r)
                    for (int c = 0; c < nk; ++c) {
                        double v = 0.0;
                        for (int j = 0; j < m; ++j) v += st.Qk[j * nk + r] * tmp[j * nk + c];
                        res[r * S + c] = v;
                    }
                M.swap(res);
            };
            rot(st.Ht);
            rot(st.Nt);
            st.m = nk;
            spk::dav_cgs(s, h->dV.p, ld, 0, st.m, sm + lay.pc2, st.nch, h->dt.p, st.n, sm + lay.pc1, 0);
        }
        // CGS2 of the extending states
        D.clear();
        max_n = 0;
        for (int i : ext) {
            D.push_back(dav_inst(B[i]));
            max_n = std::max(max_n, B[i].n);
        }
        if (!D.empty()) {
            batch_dav_upload(D, bb, s);
            spk::bdav_cgs(s, bb.dav.p, int(D.size()), max_n, 0);
            spk::bdav_cgs(s, bb.dav.p, int(D.size()), max_n, 1);
        }
        // one fused product for the new vectors (x = t) and the starting
        // vectors (x = V_0), then their Gram rows
        std::vector<int> prod = ext;
        prod.insert(prod.end(), starting.begin(), starting.end());
        if (!prod.empty()) {
            std::vector<int> from_v0(B.size(), 0);
            for (int i : starting) from_v0[i] = 1;
            batch_heff_mixed(B, prod, from_v0, bb, s);
            D.clear();
            max_n = 0;
            max_m = 0;
            for (int i : prod) {
                spk::DavInst I = dav_inst(B[i]);
                I.from_t = from_v0[i] ? 0 : 1;
                D.push_back(I);
                max_n = std::max(max_n, B[i].n);
                max_m = std::max(max_m, B[i].m);
            }
            batch_dav_upload(D, bb, s);
            spk::bdav_gram(s, bb.dav.p, int(D.size()), max_n, max_m);
        }
        HIPCK(hipStreamSynchronize(s));
        // results
        for (int i : starting) {
            BatchState& st = B[i];
            sp_handle* h = st.h;
            const DavLayout lay(h->dav_sub, spk::dav_chunks(int(h->ld)));
            const double* pg = h->pin + (lay.pg - lay.out);
            st.Ht[0] = chunk_total(pg, st.nch, 2, 0);
            st.Nt[0] = chunk_total(pg, st.nch, 2, 1);
            st.m = 1;
            st.out.matvecs = 1;
            phase[i] = 1;
        }
        std::vector<int> finished;
        for (int i : iterating) {
            BatchState& st = B[i];
            sp_handle* h = st.h;
            const DavLayout lay(h->dav_sub, spk::dav_chunks(int(h->ld)));
            const double* dn = h->pin;
            double xt[3];
            chunk_totals(dn + (lay.px - lay.out), st.nch, 3, xt);
            const double xx = xt[0], uu = xt[1], xn = xt[2];
            if (!std::isfinite(xx) || !std::isfinite(uu) || !(xx > 0.0)) throw SpError(SP_ENAN, "non-finite Ritz vector");
            st.out.rnorm = std::sqrt(uu / xx);
            st.out.pnorm = xn / xx;
            if (st.out.rnorm <= o.tol) {
                st.out.converged = true;
                finished.push_back(i);
                continue;
            }
            if (st.last) {
                finished.push_back(i);
                continue;
            }
            const double tn = dn[lay.tn - lay.out];
            if (!(tn >= 1e-14)) {
                finished.push_back(i);
                continue;
            }
            const int m = st.m, nd = 4 * m + 2;
            std::vector<double> gt(nd);
            chunk_totals(dn + (lay.pg - lay.out), st.nch, nd, gt.data());
            for (int j = 0; j <= m; ++j) {
                const double hv_new = gt[j];
                const double nv_new = gt[m + 1 + j];
                const double hv_old = (j < m) ? gt[2 * m + 2 + j] : hv_new;
                const double nv_old = (j < m) ? gt[3 * m + 2 + j] : nv_new;
                st.Ht[j * S + m] = hv_new;
                st.Nt[j * S + m] = nv_new;
                st.Ht[m * S + j] = hv_old;
                st.Nt[m * S + j] = nv_old;
            }
            ++st.m;
        }
        // step end of the states whose local solve is over
        for (int i : finished) {
            BatchState& st = B[i];
            sp_handle* h = st.h;
            const int k = st.k, d = st.order[st.step].second, L = h->L;
            spk::normalize(s, h->dx.p, site_ptr(h, k), st.n, nullptr);
            if (reduced(h)) {
                double th, pn, xx;
                rayleigh64(h, k, site_ptr(h, k), th, pn, xx);
                st.out.theta = th;
                st.out.pnorm = pn;
            }
            if (L > 1) {
                if (d > 0) {
                    move_right(h, k);
                    env_left(h, k);
                    h->center = k + 1;
                } else {
                    move_left(h, k);
                    env_right(h, k);
                    h->center = k - 1;
                }
            }
        }
        if (!finished.empty()) {
            HIPCK(hipStreamSynchronize(s));
            HIPCK(hipGetLastError());
        }
        const auto t1 = std::chrono::steady_clock::now();
        for (int i : finished) {
            BatchState& st = B[i];
            if (!st.out.converged) status = SP_ENOCONV;
            record_step(reps[i], o.verbose, i,
                        {int(st.step / st.sweep_len), st.k, st.order[st.step].second, st.out.iters,
                         st.out.converged ? 1 : 0, st.out.matvecs, st.out.theta, st.out.pnorm, st.out.rnorm,
                         std::chrono::duration<double, std::micro>(t1 - st.t0).count()});
            ++st.step;
            phase[i] = st.step < st.order.size() ? 0 : 2;
        }
    }
    return status;
}

}  // namespace

namespace {

// ---------------------------------------------------------------------------
// Sweeps with the device-resident Davidson iteration.  Every state (one or
// many) advances in rounds: in a round each unfinished state solves the
// local problem at its next site.  The first product (V_0) runs eagerly; then
// one iteration of every state - subspace solve, Ritz pass, restart
// rotation, CGS2, H_eff of the correction (one fused launch for all states
// and quadrature points), Gram pass, residual and convergence bookkeeping -
// is captured once in a HIP graph and replayed until no state iterates (the
// host polls a mapped status record every few replays).  A state whose solve
// has ended is idle in the remaining replays of its round: its passes and
// its fused H_eff tasks return at once.  Then the gauge moves and
// environment updates of all states run eagerly, and the next round starts.

// whether these settings run the device-resident iteration for a sweep of
// nstates states
bool device_solver_ok(const sp_handle* h, const sp_sweep_opts& o, int nstates) {
    const int max_sub = std::max(2, o.max_sub);
    const int keep = std::max(1, std::min(o.keep, max_sub - 1));
    const bool want = o.solver == SP_SOLVER_DEVICE || (o.solver == SP_SOLVER_AUTO && nstates >= 2);
    return want && h->path == SP_PATH_TILED && h->cons.empty() && !h->mlp_use && !h->mlp_rec &&
           max_sub + 1 <= spk::kDevSubMax && keep <= spk::kDevKeepMax;
}

spk::DavInst dev_inst(BatchState& st, const sp_sweep_opts& o, int max_sub, int keep, int max_iter, double* status) {
    sp_handle* h = st.h;
    const long long ld = h->ld;
    const DavLayout lay(h->dav_sub, spk::dav_chunks(int(ld)));
    double* sm = h->dsmall.p;
    spk::DavInst I{};
    I.V = h->dV.p;
    I.HV = h->dHV.p;
    I.NV = h->dNV.p;
    I.ld = ld;
    I.aqd = sm + lay.a;
    I.aq = I.aqd;
    I.dh = h->ddh.p;
    I.dn = h->ddn.p;
    I.floor_ = 1e-8;
    I.x = h->dx.p;
    I.t = h->dt.p;
    I.part_x = sm + lay.px;
    I.pc1 = sm + lay.pc1;
    I.pc2 = sm + lay.pc2;
    I.pn = sm + lay.pn;
    I.pg = sm + lay.pg;
    I.tnorm = sm + lay.tn;
    I.ypart = h->ypart.p;
    I.nypart = h->nypart.p;
    I.gstride = st.n;
    I.G = heff_parts(h, st.k);
    I.m = 0;  // the first Gram pass (V_0, products read from the partials)
    I.mr = 0;
    I.n = st.n;
    I.active = 1;
    I.from_t = 0;
    I.ext = 1;
    I.max_iter = max_iter;
    I.max_sub = max_sub;
    I.keep = keep;
    I.S = max_sub + 1;
    I.nch = st.nch;
    I.tol = o.tol;
    I.drop = metric_drop(h);
    I.Ht = h->dHt.p;
    I.Nt = h->dNt.p;
    I.Qk = sm + lay.q;
    I.status = status;
    return I;
}

int sweep_rounds(std::vector<BatchState>& B, const sp_sweep_opts& o, std::vector<sp_sweep_report*>& reps) {
    hipStream_t s = B[0].h->stream;
    const int max_sub = std::max(2, o.max_sub);
    const int keep = std::max(1, std::min(o.keep, max_sub - 1));
    const int max_iter = std::max(1, o.max_iter);
    const int nb = int(B.size());
    for (auto& st : B) ensure_davidson(st.h, max_sub);
    BatchBufs bb;
    // mapped status (8 doubles per state) and pinned staging of the records
    double *stat = nullptr, *stat_dev = nullptr, *stage = nullptr;
    HIPCK(hipHostMalloc(&stat, size_t(8) * nb * sizeof(double), hipHostMallocMapped | hipHostMallocCoherent));
    HIPCK(hipHostGetDevicePointer((void**)&stat_dev, stat, 0));
    HIPCK(hipHostMalloc(&stage, size_t(nb) * sizeof(spk::DavInst), hipHostMallocDefault));
    hipStream_t gs = nullptr;
    HIPCK(hipStreamCreateWithFlags(&gs, hipStreamNonBlocking));
    struct Cleanup {
        double *a, *b;
        hipStream_t g;
        ~Cleanup() {
            if (a) (void)hipHostFree(a);
            if (b) (void)hipHostFree(b);
            if (g) (void)hipStreamDestroy(g);
        }
    } cleanup{stat, stage, gs};
    DArr<spk::DavInst> dinst;
    dinst.alloc(nb);
    DArr<spk::H3Inst> ginst;
    DArr<spk::H3Task> gtask;
    int status = SP_OK;
    const int poll = 4;  // replays between two looks at the status
    for (;;) {
        std::vector<int> idx;
        for (int i = 0; i < nb; ++i)
            if (B[i].step < B[i].order.size()) idx.push_back(i);
        if (idx.empty()) break;
        const int na = int(idx.size());
        int max_n = 0;
        // step start: diagonal, V_0 and its products (eager)
        for (int i : idx) {
            BatchState& st = B[i];
            sp_handle* h = st.h;
            st.k = st.order[st.step].first;
            st.n = int(h->sites[st.k - 1].size);
            st.nch = spk::dav_chunks(st.n);
            st.t0 = std::chrono::steady_clock::now();
            max_n = std::max(max_n, st.n);
            diag(h, st.k, h->ddh.p, h->ddn.p);
            spk::normalize(s, site_ptr(h, st.k), h->dV.p, st.n, nullptr);
        }
        {
            std::vector<int> from_v0(B.size(), 1);
            batch_heff_mixed(B, idx, from_v0, bb, s);
        }
        spk::DavInst* D = reinterpret_cast<spk::DavInst*>(stage);
        for (int q = 0; q < na; ++q) {
            for (int c = 0; c < 8; ++c) stat[8 * q + c] = 0.0;
            D[q] = dev_inst(B[idx[q]], o, max_sub, keep, max_iter, stat_dev + 8 * q);
        }
        HIPCK(hipMemcpyAsync(dinst.p, D, size_t(na) * sizeof(spk::DavInst), hipMemcpyHostToDevice, s));
        spk::bdav_gram(s, dinst.p, na, max_n, 0);
        spk::bdav_start(s, dinst.p, na);
        // the fused H_eff of the corrections: instance records and tasks on
        // the device for the whole round, each instance gated by its record
        std::vector<spk::H3Inst> hi(na);
        std::map<int, std::vector<spk::H3Task>> by_rc;
        std::map<int, int> lds_by_rc;
        std::vector<int> tiled;
        const bool f32 = reduced(B[idx[0]].h);
        for (int q = 0; q < na; ++q) {
            BatchState& st = B[idx[q]];
            sp_handle* h = st.h;
            hi[q] = heff_inst(h, st.k, h->dt.p, f32);
            hi[q].gate = reinterpret_cast<const int*>(reinterpret_cast<const char*>(dinst.p + q) +
                                                     offsetof(spk::DavInst, ext));
            const SitePlan& P = h->plan[st.k - 1];
            if (P.h_rows == 0) {
                tiled.push_back(q);
                continue;
            }
            for (spk::H3Task t : P.h_tasks) {
                if (t.blk < 0) continue;
                t.inst = q;
                by_rc[P.h_rows].push_back(t);
            }
            lds_by_rc[P.h_rows] = std::max(lds_by_rc[P.h_rows], P.h_lds);
        }
        std::vector<spk::H3Task> all;
        std::vector<std::pair<int, std::pair<size_t, int>>> groups;
        for (auto& kv : by_rc) {
            groups.push_back({kv.first, {all.size(), int(kv.second.size())}});
            all.insert(all.end(), kv.second.begin(), kv.second.end());
        }
        if (ginst.n < size_t(na)) ginst.alloc(na);
        if (gtask.n < all.size()) gtask.alloc(all.size());
        HIPCK(hipMemcpy(ginst.p, hi.data(), size_t(na) * sizeof(spk::H3Inst), hipMemcpyHostToDevice));
        if (!all.empty())
            HIPCK(hipMemcpy(gtask.p, all.data(), all.size() * sizeof(spk::H3Task), hipMemcpyHostToDevice));
        HIPCK(hipStreamSynchronize(s));
        // one iteration of every state, captured on the private stream
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        std::vector<hipStream_t> saved;
        for (int q : tiled) saved.push_back(B[idx[q]].h->stream);
        for (int q : tiled) B[idx[q]].h->stream = gs;  // their block products launch on the capture stream
        hipError_t ce = hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal);
        if (ce == hipSuccess) {
            spk::bdav_solve(gs, dinst.p, na, max_sub);
            spk::bdav_ritz(gs, dinst.p, na, max_n);
            spk::bdav_rotate(gs, dinst.p, na, max_n);
            spk::bdav_cgs(gs, dinst.p, na, max_n, 2);
            spk::bdav_cgs(gs, dinst.p, na, max_n, 0);
            spk::bdav_cgs(gs, dinst.p, na, max_n, 1);
            for (auto& gr : groups) {
                const spk::H3Task* tp = gtask.p + gr.second.first;
                if (f32) spk::heff3_f32(gs, gr.first, lds_by_rc[gr.first], tp, gr.second.second, hi[0], ginst.p);
                else spk::heff3(gs, gr.first, lds_by_rc[gr.first], tp, gr.second.second, hi[0], ginst.p);
            }
            for (int q : tiled) {
                BatchState& st = B[idx[q]];
                heff_tiled(st.h, st.k, st.h->dt.p, st.h->precision == SP_BF16X3);
            }
            spk::bdav_gram(gs, dinst.p, na, max_n, max_sub);
            spk::bdav_update(gs, dinst.p, na);
            ce = hipStreamEndCapture(gs, &graph);
        }
        for (size_t j = 0; j < tiled.size(); ++j) B[idx[tiled[j]]].h->stream = saved[j];
        hip_check(ce, "capture of the Davidson iteration");
        HIPCK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
        int replays = 0;
        bool running = true;
        while (running && replays < max_iter + 1) {
            for (int r = 0; r < poll && replays < max_iter + 1; ++r, ++replays) HIPCK(hipGraphLaunch(exec, gs));
            HIPCK(hipStreamSynchronize(gs));
            running = false;
            for (int q = 0; q < na; ++q) running = running || stat[8 * q] != 0.0;
        }
        (void)hipGraphExecDestroy(exec);
        (void)hipGraphDestroy(graph);
        HIPCK(hipGetLastError());
        if (running) throw SpError(SP_EHIP, "internal: a device-resident local solve did not end");
        // step end
        for (int q = 0; q < na; ++q) {
            const double* sq = stat + 8 * q;
            const int err = int(sq[7]);
            if (err == SP_ENORM) throw SpError(SP_ENORM, "projected norm vanishes in the search space");
            if (err != 0) throw SpError(SP_ENAN, "non-finite value in a local solve");
            BatchState& st = B[idx[q]];
            st.out = DavOut{};
            st.out.converged = sq[1] != 0.0;
            st.out.iters = int(sq[2]);
            st.out.matvecs = int(sq[3]);
            st.out.theta = sq[4];
            st.out.rnorm = sq[5];
            st.out.pnorm = sq[6];
            sp_handle* h = st.h;
            const int k = st.k, d = st.order[st.step].second, L = h->L;
            spk::normalize(s, h->dx.p, site_ptr(h, k), st.n, nullptr);
            if (reduced(h)) {
                double th, pn, xx;
                rayleigh64(h, k, site_ptr(h, k), th, pn, xx);
                if (!std::isfinite(th)) throw SpError(SP_ENAN, "non-finite Rayleigh quotient");
                st.out.theta = th;
                st.out.pnorm = pn;
            }
            if (L > 1) {
                if (d > 0) {
                    move_right(h, k);
                    env_left(h, k);
                    h->center = k + 1;
                } else {
                    move_left(h, k);
                    env_right(h, k);
                    h->center = k - 1;
                }
            }
        }
        HIPCK(hipStreamSynchronize(s));
        HIPCK(hipGetLastError());
        const auto t1 = std::chrono::steady_clock::now();
        for (int q = 0; q < na; ++q) {
            const int i = idx[q];
            BatchState& st = B[i];
            if (!st.out.converged) status = SP_ENOCONV;
            record_step(reps[i], o.verbose, i,
                        {int(st.step / st.sweep_len), st.k, st.order[st.step].second, st.out.iters,
                         st.out.converged ? 1 : 0, st.out.matvecs, st.out.theta, st.out.pnorm, st.out.rnorm,
                         std::chrono::duration<double, std::micro>(t1 - st.t0).count()});
            ++st.step;
        }
    }
    return status;
}

}  // namespace

// ---------------------------------------------------------------------------
// Allocation-free H_eff x (sp_heff_apply_noalloc): its per-g partial slots
// live in a fixed device array instead of the handle's buffers.  Every GPU
// that runs the library holds its own copy until the process ends.  Host code
// never passes the array's name to a kernel: its device address on each
// device comes from hipGetSymbolAddress, taken once per device at
// sp_init_mps with that device current.

constexpr long long kNoAllocSlots = 1LL << 21;  // doubles per output (y, ny): 16 MiB each
static __device__ __align__(256) double scratch[2 * kNoAllocSlots];

namespace {
std::mutex g_scratch_mu;
std::map<int, double*> g_scratch_ptr;  // device -> device address of its scratch

// address of the scratch array on `device`; resolved on the first call for
// the device (with that device current), cached afterwards
double* noalloc_scratch(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(device);
    if (it != g_scratch_ptr.end()) return it->second;
    int cur = 0;
    HIPCK(hipGetDevice(&cur));
    if (cur != device) HIPCK(hipSetDevice(device));
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != device) HIPCK(hipSetDevice(cur));
    hip_check(e, "hipGetSymbolAddress(scratch)");
    if (!ptr) throw SpError(SP_EHIP, "hipGetSymbolAddress(scratch) returned a null address");
    g_scratch_ptr[device] = static_cast<double*>(ptr);
    return static_cast<double*>(ptr);
}
}  // namespace

// ---------------------------------------------------------------------------
// C ABI

namespace {
int guarded(const std::function<int()>& f) {
    try {
        return f();
    } catch (const SpError& e) {
        g_last_error = e.what();
        return e.code;
    } catch (const std::bad_alloc&) {
        g_last_error = "host allocation failed";
        return SP_ENOMEM;
    } catch (const std::exception& e) {
        g_last_error = e.what();
        return SP_EINVAL;
    }
}
}  // namespace

extern "C" {

const char* sp_last_error(void) { return g_last_error.c_str(); }

int sp_init_mps(const sp_problem* p, const sp_mpo* W, const sp_block_table* bonds, const double* init_blocks,
                void* hip_stream, sp_handle** out) {
    return guarded([&]() -> int {
        SP_REQUIRE(p && W && bonds && init_blocks && out, "null argument");
        *out = nullptr;
        SP_REQUIRE(p->L >= 1 && p->d == 4, "need L >= 1 and d == 4");
        SP_REQUIRE(p->precision == SP_FP64 || p->precision == SP_FP32 || p->precision == SP_BF16X3,
                   "precision must be SP_FP64, SP_FP32 or SP_BF16X3");
        SP_REQUIRE(p->precision == SP_FP64 || p->path == SP_PATH_TILED, "reduced precision needs the tiled path");
        SP_REQUIRE(p->path == SP_PATH_TILED || p->path == SP_PATH_PLAIN, "unknown kernel path");
        SP_REQUIRE(p->N >= 0 && p->N <= 2 * p->L, "N out of range");
        SP_REQUIRE((p->N + p->twoS) % 2 == 0, "N and 2S must have the same parity");
        SP_REQUIRE((p->N + p->twoM) % 2 == 0, "N and 2M must have the same parity");
        SP_REQUIRE(p->twoS >= 0 && std::abs(p->twoM) <= p->twoS, "need |M| <= S");
        SP_REQUIRE(p->twoS <= sph::max_seniority(p->N, p->twoM, p->L), "S exceeds the largest seniority");
        SP_REQUIRE(p->G >= 1 && p->G <= 1024, "G out of range");
        std::unique_ptr<sp_handle> h(new sp_handle());
        h->stream = reinterpret_cast<hipStream_t>(hip_stream);
        h->path = p->path;
        h->precision = p->precision;
        h->L = p->L;
        h->N = p->N;
        h->twoS = p->twoS;
        h->twoM = p->twoM;
        h->G = p->G;
        h->inexact = p->G < sph::exact_points(p->N, p->L, p->twoS, p->twoM);
        h->qx.resize(h->G);
        h->qw.resize(h->G);
        h->qc.resize(h->G);
        h->qs.resize(h->G);
        h->qcoef.resize(h->G);
        sph::projector_quadrature(h->G, h->twoS, h->twoM, h->qx.data(), h->qw.data(), h->qc.data(), h->qs.data(),
                                  h->qcoef.data());
        build_mpo(h.get(), W);
        build_bonds(h.get(), bonds);
        {
            int tot = 0;
            for (int k = 0; k <= h->L; ++k) tot += bonds->nsec[k];
            h->tab_nsec.assign(bonds->nsec, bonds->nsec + h->L + 1);
            h->tab_n.assign(bonds->sec_n, bonds->sec_n + tot);
            h->tab_2m.assign(bonds->sec_2m, bonds->sec_2m + tot);
            h->tab_dim.assign(bonds->sec_dim, bonds->sec_dim + tot);
        }
        build_env_layouts(h.get());
        h->plan.resize(h->L);
        long long Tmax = 0, Vmax = 0, qrs = 0, qrr = 0, LTmax = 0;
        for (int k = 1; k <= h->L; ++k) {
            build_plan(h.get(), k);
            if (h->path == SP_PATH_TILED && !build_fused(h.get(), k)) build_fused(h.get(), k, kHeffLdsMax);
            if (h->path == SP_PATH_TILED && h->plan[k - 1].h_rows == 1) {
                // one row per task re-reads the right environment once per
                // row (wide MPOs): the tiled block products are faster there
                // (3.6 ms against about 1 ms at the K = 12 ab-initio sites)
                SitePlan& P1 = h->plan[k - 1];
                P1.h_rows = 0;
                P1.h_lds = 0;
                P1.h_tasks.clear();
            }
            const SitePlan& P = h->plan[k - 1];
            Tmax = std::max({Tmax, P.Tsize, P.Zsize});
            Vmax = std::max({Vmax, P.Vsize, P.Ztsize});
            LTmax = std::max(LTmax, P.LTsize);
            qrs = std::max({qrs, P.qr_scratch, P.lq_scratch});
            qrr = std::max({qrr, P.qr_rsize, P.lq_rsize});
        }
        h->T_cap = h->G * std::max(1LL, Tmax);
        h->V_cap = h->G * std::max(1LL, Vmax);
        h->LT_cap = h->path == SP_PATH_TILED ? h->G * std::max(1LL, LTmax) : 1;
        h->qr_scratch_cap = std::max(1LL, qrs);
        h->qr_r_cap = std::max(1LL, qrr);
        for (int k = 1; k <= h->L; ++k) {
            h->Xd_cap = std::max(h->Xd_cap, h->plan[k - 1].Xd_size);
            h->tr_split_max = std::max(h->tr_split_max, h->plan[k - 1].tr_split);
        }
        h->Xd_cap = std::max(1LL, h->Xd_cap);
        validate_plans(h.get());
        // every host-side check is done; device work starts here
        HIPCK(hipGetDevice(&h->device));
        alloc_envs(h.get());
        for (int k = 1; k <= h->L; ++k) upload_plan(h.get(), k);
        h->T.alloc(h->T_cap);
        h->V.alloc(h->V_cap);
        h->LT.alloc(h->LT_cap);
        h->diag_part.alloc(size_t(spk::kDiagSplitMax) * std::max(1LL, h->max_site));
        h->qr_scratch.alloc(h->qr_scratch_cap);
        h->qr_r.alloc(h->qr_r_cap);
        h->tmp_site.alloc(h->max_site);
        h->mps.alloc(h->mps_size);
        if (h->path == SP_PATH_TILED) {
            h->Xd.alloc(h->Xd_cap);
            h->ypart.alloc(size_t(h->G) * h->tr_split_max * h->max_site);
            h->nypart.alloc(size_t(h->G) * h->tr_split_max * h->max_site);
        }
        HIPCK(hipMemcpyAsync(h->mps.p, init_blocks, h->mps_size * sizeof(double), hipMemcpyHostToDevice, h->stream));
        // right-canonical form of sites L..2 and the right environments
        for (int k = h->L; k >= 2; --k) {
            move_left(h.get(), k);
            env_right(h.get(), k);
        }
        h->center = 1;
        HIPCK(hipStreamSynchronize(h->stream));
        HIPCK(hipGetLastError());
        if (h->path == SP_PATH_TILED) (void)noalloc_scratch(h->device);
        *out = h.release();
        return (*out)->inexact ? SP_WINEXACT : SP_OK;
    });
}

int sp_destroy(sp_handle* h) {
    return guarded([&]() -> int {
        if (!h) return SP_OK;
        (void)hipStreamSynchronize(h->stream);
        delete h;
        return SP_OK;
    });
}

int sp_env_update(sp_handle* h, int site, int dir) {
    return guarded([&]() -> int {
        SP_REQUIRE(h, "null handle");
        check_site(h, site);
        SP_REQUIRE(dir == 1 || dir == -1, "dir must be +1 or -1");
        if (dir > 0) env_left(h, site);
        else env_right(h, site);
        HIPCK(hipGetLastError());
        return SP_OK;
    });
}

int sp_heff_apply(sp_handle* h, int site, const double* x, double* y, double* ny) {
    return guarded([&]() -> int {
        SP_REQUIRE(h && x && y && ny, "null argument");
        check_site(h, site);
        SP_REQUIRE(x != y && x != ny && y != ny, "x, y and ny must not alias");
        heff_apply(h, site, x, y, ny);
        HIPCK(hipGetLastError());
        return SP_OK;
    });
}

int sp_heff_apply_noalloc(sp_handle* h, int site, const double* x, double* y, double* ny) {
    return guarded([&]() -> int {
        SP_REQUIRE(h && x && y && ny, "null argument");
        check_site(h, site);
        SP_REQUIRE(x != y && x != ny && y != ny, "x, y and ny must not alias");
        SP_REQUIRE(h->path == SP_PATH_TILED, "sp_heff_apply_noalloc: tiled path only");
        const long long need = (long long)heff_parts(h, site) * h->sites[site - 1].size;
        if (need > kNoAllocSlots)
            throw SpError(SP_EINVAL, "sp_heff_apply_noalloc: the site needs " + std::to_string(need) +
                                         " partial slots per output, more than the fixed " +
                                         std::to_string(kNoAllocSlots));
        std::unique_lock<std::mutex> lk(g_scratch_mu);
        auto it = g_scratch_ptr.find(h->device);
        SP_REQUIRE(it != g_scratch_ptr.end(), "internal: scratch address of the device not resolved");
        double* base = it->second;
        lk.unlock();
        heff_apply(h, site, x, y, ny, false, false, base, base + kNoAllocSlots);
        HIPCK(hipGetLastError());
        return SP_OK;
    });
}

int sp_heff_diag(sp_handle* h, int site, double* dh, double* dn) {
    return guarded([&]() -> int {
        SP_REQUIRE(h && dh && dn, "null argument");
        check_site(h, site);
        diag(h, site, dh, dn);
        HIPCK(hipGetLastError());
        return SP_OK;
    });
}

int sp_sweep(sp_handle* h, const sp_sweep_opts* o, sp_sweep_report* r) {
    return guarded([&]() -> int {
        SP_REQUIRE(h && o, "null argument");
        SP_REQUIRE(o->n_sweeps >= 0 && o->max_iter >= 1 && o->max_sub >= 2 && o->keep >= 1 && o->tol >= 0,
                   "bad sweep options");
        SP_REQUIRE(h->center == 1, "sweeps start with the canonical centre at site 1");
        if (r) r->n_steps = 0;
        SP_REQUIRE(o->solver >= SP_SOLVER_AUTO && o->solver <= SP_SOLVER_DEVICE, "unknown solver");
        if (device_solver_ok(h, *o, 1)) {
            std::vector<BatchState> B(1);
            std::vector<sp_sweep_report*> reps(1, r);
            B[0].h = h;
            const int L = h->L;
            std::vector<std::pair<int, int>> one;
            for (int k = 1; k < L; ++k) one.push_back({k, +1});
            for (int k = L; k >= 2; --k) one.push_back({k, -1});
            if (L == 1) one.push_back({1, +1});
            B[0].sweep_len = int(one.size());
            for (int sw = 0; sw < o->n_sweeps; ++sw) B[0].order.insert(B[0].order.end(), one.begin(), one.end());
            return sweep_rounds(B, *o, reps);
        }
        int status = SP_OK;
        const int L = h->L;
        for (int sw = 0; sw < o->n_sweeps; ++sw) {
            std::vector<std::pair<int, int>> order;
            for (int k = 1; k < L; ++k) order.push_back({k, +1});
            for (int k = L; k >= 2; --k) order.push_back({k, -1});
            if (L == 1) order.push_back({1, +1});
            for (auto [k, d] : order) {
                const auto t0 = std::chrono::steady_clock::now();
                prepare_constraints(h, k);
                DavOut dv = davidson(h, k, *o);
                if (L > 1) {
                    if (d > 0) {
                        move_right(h, k);
                        env_left(h, k);
                        for (auto& a : h->cons) env_left_mixed(a.get(), k, site_ptr(h, k));
                        h->center = k + 1;
                    } else {
                        move_left(h, k);
                        env_right(h, k);
                        for (auto& a : h->cons) env_right_mixed(a.get(), k, site_ptr(h, k));
                        h->center = k - 1;
                    }
                }
                HIPCK(hipStreamSynchronize(h->stream));
                HIPCK(hipGetLastError());
                const auto t1 = std::chrono::steady_clock::now();
                if (!dv.converged) status = SP_ENOCONV;
                record_step(r, o->verbose, 0,
                            {sw, k, d, dv.iters, dv.converged ? 1 : 0, dv.matvecs, dv.theta, dv.pnorm, dv.rnorm,
                             std::chrono::duration<double, std::micro>(t1 - t0).count()});
            }
        }
        return status;
    });
}

int sp_sweep_batch(sp_handle** hs, int n, const sp_sweep_opts* o, sp_sweep_report* r) {
    return guarded([&]() -> int {
        SP_REQUIRE(hs && o && n >= 1, "bad arguments");
        SP_REQUIRE(o->n_sweeps >= 0 && o->max_iter >= 1 && o->max_sub >= 2 && o->keep >= 1 && o->tol >= 0,
                   "bad sweep options");
        std::vector<BatchState> B(n);
        std::vector<sp_sweep_report*> reps(n, nullptr);
        for (int i = 0; i < n; ++i) {
            sp_handle* h = hs[i];
            SP_REQUIRE(h, "null handle");
            SP_REQUIRE(h->path == SP_PATH_TILED, "batched sweeps need the tiled path");
            SP_REQUIRE(h->cons.empty(), "states with orthogonality constraints sweep with sp_sweep");
            SP_REQUIRE(!h->mlp_use && !h->mlp_rec, "states with a learned preconditioner sweep with sp_sweep");
            SP_REQUIRE(h->stream == hs[0]->stream && h->device == hs[0]->device,
                       "batched handles must share one device and one stream");
            SP_REQUIRE(h->precision == hs[0]->precision, "batched handles must share the precision");
            SP_REQUIRE(h->center == 1, "sweeps start with the canonical centre at site 1");
            for (int j = 0; j < i; ++j) SP_REQUIRE(hs[j] != h, "a handle appears twice in the batch");
            B[i].h = h;
            const int L = h->L;
            std::vector<std::pair<int, int>> one;
            for (int k = 1; k < L; ++k) one.push_back({k, +1});
            for (int k = L; k >= 2; --k) one.push_back({k, -1});
            if (L == 1) one.push_back({1, +1});
            B[i].sweep_len = int(one.size());
            for (int sw = 0; sw < o->n_sweeps; ++sw) B[i].order.insert(B[i].order.end(), one.begin(), one.end());
            if (r) {
                reps[i] = &r[i];
                r[i].n_steps = 0;
            }
        }
        SP_REQUIRE(o->solver >= SP_SOLVER_AUTO && o->solver <= SP_SOLVER_DEVICE, "unknown solver");
        bool dev = true;
        for (int i = 0; i < n; ++i) dev = dev && device_solver_ok(hs[i], *o, n);
        return dev ? sweep_rounds(B, *o, reps) : sweep_batch(B, *o, reps);
    });
}

int sp_autotune(sp_handle* h, int reps, int* budget_out, int* rows_out, double* usec_out) {
    return guarded([&]() -> int {
        SP_REQUIRE(h && reps >= 1, "bad arguments");
        SP_REQUIRE(h->path == SP_PATH_TILED, "the autotuner tunes the fused kernel of the tiled path");
        const int candidates[] = {4608, 9216, 13824, kHeffLdsMax};
        hipStream_t s = h->stream;
        hipEvent_t e0, e1;
        HIPCK(hipEventCreate(&e0));
        HIPCK(hipEventCreate(&e1));
        for (int k = 1; k <= h->L; ++k) {
            SitePlan& P = h->plan[k - 1];
            const double* x = site_ptr(h, k);
            int best_b = 0, best_rc = 0, last_rc = -1;
            float best = 1e30f;
            for (int b : candidates) {
                if (!build_fused(h, k, b)) continue;  // a block too wide for this budget
                if (P.h_rows == last_rc) continue;  // same plan as the previous budget
                last_rc = P.h_rows;
                validate_fused(h, k);
                upload_fused(h, k);
                HIPCK(hipStreamSynchronize(s));
                const bool f32 = reduced(h);
                const spk::H3Inst I = heff_inst(h, k, x, f32);
                auto launch = [&]() {
                    if (f32) spk::heff3_f32(s, P.h_rows, P.h_lds, P.dh_tasks.p, int(P.h_tasks.size()), I);
                    else spk::heff3(s, P.h_rows, P.h_lds, P.dh_tasks.p, int(P.h_tasks.size()), I);
                };
                (void)hipGetLastError();
                launch();  // warm-up
                if (hipGetLastError() != hipSuccess) {  // this LDS size does not launch here
                    HIPCK(hipStreamSynchronize(s));
                    continue;
                }
                HIPCK(hipEventRecord(e0, s));
                for (int r = 0; r < reps; ++r) launch();
                HIPCK(hipEventRecord(e1, s));
                HIPCK(hipEventSynchronize(e1));
                float ms = 0.f;
                HIPCK(hipEventElapsedTime(&ms, e0, e1));
                HIPCK(hipGetLastError());
                if (ms < best) {
                    best = ms;
                    best_b = b;
                    best_rc = P.h_rows;
                }
            }
            {
                // the LDS-tiled block products are a candidate too: for wide
                // MPOs a fused plan of one or two rows per task re-reads the
                // right environment once per row and can lose to them
                P.h_rows = 0;
                P.h_lds = 0;
                P.h_tasks.clear();
                validate_fused(h, k);
                upload_fused(h, k);
                HIPCK(hipStreamSynchronize(s));
                const bool bf3 = h->precision == SP_BF16X3;
                heff_tiled(h, k, x, bf3);  // warm-up (also forms the pre-mixed environment)
                HIPCK(hipEventRecord(e0, s));
                for (int r = 0; r < reps; ++r) heff_tiled(h, k, x, bf3);
                HIPCK(hipEventRecord(e1, s));
                HIPCK(hipEventSynchronize(e1));
                float ms = 0.f;
                HIPCK(hipEventElapsedTime(&ms, e0, e1));
                HIPCK(hipGetLastError());
                if (ms < best) {
                    best = ms;
                    best_b = 0;
                    best_rc = 0;
                }
            }
            if (best_b > 0) {
                build_fused(h, k, best_b);
            } else {  // the tiled block products were fastest, or no budget fits
                P.h_rows = 0;
                P.h_lds = 0;
                P.h_tasks.clear();
            }
            validate_fused(h, k);
            upload_fused(h, k);
            HIPCK(hipStreamSynchronize(s));
            if (budget_out) budget_out[k - 1] = best_b;
            if (rows_out) rows_out[k - 1] = best_rc;
            if (usec_out) usec_out[k - 1] = 1e3 * double(best) / reps;
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        return SP_OK;
    });
}

int sp_heff_plan(const sp_handle* h, int site, int* rows, int* lds_doubles) {
    return guarded([&]() -> int {
        SP_REQUIRE(h && rows, "bad arguments");
        check_site(h, site);
        *rows = h->plan[site - 1].h_rows;
        if (lds_doubles) *lds_doubles = h->plan[site - 1].h_lds;
        return SP_OK;
    });
}

int sp_set_heff_plan(sp_handle* h, int site, int lds_budget, int* rows) {
    return guarded([&]() -> int {
        SP_REQUIRE(h, "bad arguments");
        check_site(h, site);
        SP_REQUIRE(h->path == SP_PATH_TILED, "H_eff plans belong to the tiled path");
        SP_REQUIRE(lds_budget == 0 || (lds_budget >= 1 && lds_budget <= kHeffLdsMax),
                   "LDS budget outside 0..18432 doubles");
        SitePlan& P = h->plan[site - 1];
        HIPCK(hipStreamSynchronize(h->stream));  // the old plan may still be in use
        if (lds_budget == 0 || !build_fused(h, site, lds_budget)) {
            P.h_rows = 0;
            P.h_lds = 0;
            P.h_tasks.clear();
        }
        validate_fused(h, site);
        upload_fused(h, site);
        HIPCK(hipStreamSynchronize(h->stream));
        if (rows) *rows = P.h_rows;
        return SP_OK;
    });
}

int sp_expect(sp_handle* h, const sp_mpo* O, double* value, double* normP) {
    return guarded([&]() -> int {
        SP_REQUIRE(h && O && value, "null argument");
        // a second state with the operator's environments: the same site
        // tensors (its set-up moves the canonical centre to site 1 without
        // changing the state), then <O P>/<P> at its centre
        std::vector<double> blocks(h->mps_size);
        HIPCK(hipMemcpyAsync(blocks.data(), h->mps.p, h->mps_size * sizeof(double), hipMemcpyDeviceToHost, h->stream));
        HIPCK(hipStreamSynchronize(h->stream));
        sp_problem p{h->L, 4, h->N, h->twoS, h->twoM, h->G, SP_FP64, h->path};
        sp_block_table bt{h->tab_nsec.data(), h->tab_n.data(), h->tab_2m.data(), h->tab_dim.data()};
        sp_handle* t = nullptr;
        const int rc = sp_init_mps(&p, O, &bt, blocks.data(), h->stream, &t);
        if (rc < 0) throw SpError(rc, std::string("operator state: ") + g_last_error);
        std::unique_ptr<sp_handle, int (*)(sp_handle*)> guard(t, sp_destroy);
        double np = 0.0;
        const int rc2 = sp_energy(t, value, &np);
        if (rc2 < 0) throw SpError(rc2, g_last_error);
        if (normP) *normP = np;
        return SP_OK;
    });
}

int sp_add_orthogonality(sp_handle* h, sp_handle* lower) {
    return guarded([&]() -> int {
        SP_REQUIRE(h && lower && h != lower, "bad arguments");
        SP_REQUIRE(int(h->cons.size()) < kMaxConstraints, "at most 8 orthogonality constraints");
        SP_REQUIRE(h->center == 1, "constraints are added with the canonical centre at site 1");
        SP_REQUIRE(lower->L == h->L && lower->N == h->N && lower->twoS == h->twoS && lower->twoM == h->twoM &&
                       lower->G == h->G,
                   "the lower state must have the same L, N, S, M and quadrature");
        SP_REQUIRE(lower->tab_nsec == h->tab_nsec && lower->tab_n == h->tab_n && lower->tab_2m == h->tab_2m &&
                       lower->tab_dim == h->tab_dim,
                   "the lower state must have the same block table");
        SP_REQUIRE(lower->device == h->device, "the lower state must live on the same device");
        const int L = h->L;
        // the lower state's tensors as they are now
        std::vector<double> blocks(lower->mps_size);
        HIPCK(hipStreamSynchronize(h->stream));
        HIPCK(hipMemcpyAsync(blocks.data(), lower->mps.p, lower->mps_size * sizeof(double), hipMemcpyDeviceToHost,
                             lower->stream));
        HIPCK(hipStreamSynchronize(lower->stream));
        std::vector<int> w(L + 1);
        long long nw = 0;
        sph::mpo_identity(L, w.data(), nullptr, &nw);
        std::vector<double> wd(nw);
        sph::mpo_identity(L, w.data(), wd.data(), &nw);
        sp_problem p{L, 4, h->N, h->twoS, h->twoM, h->G, SP_FP64, SP_PATH_PLAIN};
        sp_mpo W{w.data(), wd.data()};
        sp_block_table bt{h->tab_nsec.data(), h->tab_n.data(), h->tab_2m.data(), h->tab_dim.data()};
        sp_handle* a = nullptr;
        const int rc = sp_init_mps(&p, &W, &bt, blocks.data(), h->stream, &a);
        if (rc < 0) throw SpError(rc, std::string("constraint state: ") + g_last_error);
        std::unique_ptr<sp_handle> ap(a);
        // mixed right environments against this state's right-canonical sites
        for (int k = L; k >= 2; --k) env_right_mixed(a, k, site_ptr(h, k));
        if (h->conB.n == 0) {
            h->cld = (h->max_site + 63) / 64 * 64;
            h->conB.alloc(size_t(kMaxConstraints) * h->cld);
            const int nch = spk::dav_chunks(int(h->max_site));
            h->conPart.alloc(size_t(2) * nch * kMaxConstraints);
            void* hp = nullptr;
            HIPCK(hipHostMalloc(&hp, (size_t(2) * nch + 8) * sizeof(double), hipHostMallocMapped | hipHostMallocCoherent));
            h->con_pin = static_cast<double*>(hp);
            void* dp = nullptr;
            HIPCK(hipHostGetDevicePointer(&dp, hp, 0));
            h->con_pin_dev = static_cast<double*>(dp);
        }
        HIPCK(hipStreamSynchronize(h->stream));
        HIPCK(hipGetLastError());
        h->cons.push_back(std::move(ap));
        return SP_OK;
    });
}

int sp_clear_orthogonality(sp_handle* h) {
    return guarded([&]() -> int {
        SP_REQUIRE(h, "null argument");
        HIPCK(hipStreamSynchronize(h->stream));
        h->cons.clear();
        h->con_active = 0;
        return SP_OK;
    });
}

int sp_orthogonality_overlaps(sp_handle* h, double* out) {
    return guarded([&]() -> int {
        SP_REQUIRE(h && (out || h->cons.empty()), "null argument");
        const int c = h->center;
        const int n = int(h->sites[c - 1].size);
        const size_t nc = h->cons.size();
        if (nc == 0) return SP_OK;
        // per constraint: B.x, then |lower| (its site 1 carries the norm: the
        // constraint state stays right-canonical) and |x| (x = the centre)
        DArr<double> d;
        d.alloc(2 * h->max_site + 2 * nc + 1);
        double* res = d.p + 2 * h->max_site;
        for (size_t j = 0; j < nc; ++j) {
            sp_handle* a = h->cons[j].get();
            SP_REQUIRE(a->Lvalid[c - 1] && a->Rvalid[c], "constraint environments do not reach the centre");
            constraint_vector(a, c, d.p, d.p + h->max_site);
            spk::multidot(h->stream, d.p, 0, 1, site_ptr(h, c), n, res + j);
            spk::normalize(h->stream, site_ptr(a, 1), d.p, int(a->sites[0].size), res + nc + j);
        }
        spk::normalize(h->stream, site_ptr(h, c), d.p, n, res + 2 * nc);
        std::vector<double> hres(2 * nc + 1);
        HIPCK(hipMemcpyAsync(hres.data(), res, hres.size() * sizeof(double), hipMemcpyDeviceToHost, h->stream));
        HIPCK(hipStreamSynchronize(h->stream));
        HIPCK(hipGetLastError());
        for (size_t j = 0; j < nc; ++j) {
            const double den = hres[nc + j] * hres[2 * nc];
            out[j] = den > 0.0 ? hres[j] / den : 0.0;
        }
        return SP_OK;
    });
}

int sp_mlp_create(int hidden, const float* w_init, long long capacity, sp_mlp** out) {
    return guarded([&]() -> int {
        SP_REQUIRE(out && w_init && hidden >= 1 && hidden <= spk::kMlpMaxHidden && capacity >= 0, "bad arguments");
        auto m = std::make_unique<sp_mlp>();
        m->hidden = hidden;
        HIPCK(hipGetDevice(&m->device));
        const long long P = spk::mlp_size(hidden);
        m->w.alloc(P);
        HIPCK(hipMemcpy(m->w.p, w_init, P * sizeof(float), hipMemcpyHostToDevice));
        m->m.alloc(P);
        m->v.alloc(P);
        HIPCK(hipMemset(m->m.p, 0, P * sizeof(double)));
        HIPCK(hipMemset(m->v.p, 0, P * sizeof(double)));
        m->cap = capacity;
        if (capacity > 0) {
            m->F.alloc(size_t(capacity) * spk::kMlpIn);
            m->Y.alloc(capacity);
        }
        m->nparts = 256;
        m->gpart.alloc(size_t(m->nparts) * (P + 1));
        m->scal.alloc(4096);
        *out = m.release();
        return SP_OK;
    });
}

int sp_mlp_set_scope(sp_mlp* m, int scope) {
    return guarded([&]() -> int {
        SP_REQUIRE(m, "null argument");
        SP_REQUIRE(scope == SP_MLP_VECTOR || scope == SP_MLP_NBLOCK, "unknown model scope");
        SP_REQUIRE(m->rows == 0 || scope == m->scope, "the model holds training pairs of the other scope");
        m->scope = scope;
        return SP_OK;
    });
}

int sp_mlp_destroy(sp_mlp* m) {
    return guarded([&]() -> int {
        if (m) {
            (void)hipDeviceSynchronize();
            delete m;
        }
        return SP_OK;
    });
}

int sp_mlp_get(sp_mlp* m, float* w_out, long long* rows) {
    return guarded([&]() -> int {
        SP_REQUIRE(m, "null argument");
        HIPCK(hipDeviceSynchronize());
        if (w_out) HIPCK(hipMemcpy(w_out, m->w.p, spk::mlp_size(m->hidden) * sizeof(float), hipMemcpyDeviceToHost));
        if (rows) *rows = m->rows;
        return SP_OK;
    });
}

int sp_mlp_dataset(sp_mlp* m, long long first, long long count, float* F_out, float* Y_out) {
    return guarded([&]() -> int {
        SP_REQUIRE(m && F_out && Y_out && first >= 0 && count >= 0 && first + count <= m->rows, "bad arguments");
        HIPCK(hipDeviceSynchronize());
        if (count == 0) return SP_OK;
        HIPCK(hipMemcpy(F_out, m->F.p + first * spk::kMlpIn, count * spk::kMlpIn * sizeof(float),
                        hipMemcpyDeviceToHost));
        HIPCK(hipMemcpy(Y_out, m->Y.p + first, count * sizeof(float), hipMemcpyDeviceToHost));
        return SP_OK;
    });
}

int sp_mlp_forward(sp_mlp* m, const float* F, long long n, float* y, void* stream) {
    return guarded([&]() -> int {
        SP_REQUIRE(m && (n == 0 || (F && y)) && n >= 0, "bad arguments");
        hipStream_t s = static_cast<hipStream_t>(stream);
        spk::mlp_forward(s, m->w.p, m->hidden, F, n, y);
        HIPCK(hipGetLastError());
        return SP_OK;
    });
}

int sp_mlp_train_step(sp_mlp* m, const float* F, const float* Y, long long n, double lr, double* loss, void* stream) {
    return guarded([&]() -> int {
        SP_REQUIRE(m && F && Y && n >= 1 && lr > 0.0, "bad arguments");
        hipStream_t s = static_cast<hipStream_t>(stream);
        const int parts = int(std::min<long long>(m->nparts, std::max<long long>(1, n / 1024)));
        spk::mlp_grad(s, m->w.p, m->hidden, F, Y, 0, 1, n, m->gpart.p, parts);
        m->step++;
        spk::mlp_adam(s, m->w.p, m->m.p, m->v.p, m->hidden, m->gpart.p, parts, 1.0 / double(n), lr, m->step,
                      m->scal.p);
        double l = 0.0;
        HIPCK(hipMemcpyAsync(&l, m->scal.p, sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCK(hipStreamSynchronize(s));
        if (loss) *loss = l;
        return SP_OK;
    });
}

int sp_mlp_train(sp_mlp* m, int epochs, long long batch, double lr, double* loss_out, void* stream) {
    return guarded([&]() -> int {
        SP_REQUIRE(m && epochs >= 0 && batch >= 1 && lr > 0.0, "bad arguments");
        SP_REQUIRE(m->rows > 0, "no recorded training pairs");
        hipStream_t s = static_cast<hipStream_t>(stream);
        const long long rows = m->rows;
        const long long nb = std::min<long long>((rows + batch - 1) / batch, 4096);
        for (int e = 0; e < epochs; ++e) {
            // batch b: rows b, b + nb, b + 2 nb, ... (interleaves the solves)
            for (long long b = 0; b < nb; ++b) {
                const long long count = (rows - b + nb - 1) / nb;
                const int parts = int(std::min<long long>(m->nparts, std::max<long long>(1, count / 1024)));
                spk::mlp_grad(s, m->w.p, m->hidden, m->F.p, m->Y.p, b, nb, count, m->gpart.p, parts);
                m->step++;
                spk::mlp_adam(s, m->w.p, m->m.p, m->v.p, m->hidden, m->gpart.p, parts, 1.0 / double(count), lr,
                              m->step, m->scal.p + b);
            }
            std::vector<double> l(nb);
            HIPCK(hipMemcpyAsync(l.data(), m->scal.p, nb * sizeof(double), hipMemcpyDeviceToHost, s));
            HIPCK(hipStreamSynchronize(s));
            double tot = 0.0;
            for (double x : l) tot += x;
            if (loss_out) loss_out[e] = tot / double(nb);
        }
        HIPCK(hipGetLastError());
        return SP_OK;
    });
}

int sp_set_precond(sp_handle* h, sp_mlp* use, sp_mlp* record) {
    return guarded([&]() -> int {
        SP_REQUIRE(h, "null argument");
        for (sp_mlp* m : {use, record})
            if (m) SP_REQUIRE(m->device == h->device, "the model must live on the state's device");
        if (record) SP_REQUIRE(record->cap > 0, "the recording model has no room for training pairs");
        if (use && record)
            SP_REQUIRE(use->scope == record->scope, "the model in use and the recording one differ in scope");
        HIPCK(hipStreamSynchronize(h->stream));
        h->mlp_use = use;
        h->mlp_rec = record;
        return SP_OK;
    });
}

int sp_energy(sp_handle* h, double* E, double* normP) {
    return guarded([&]() -> int {
        SP_REQUIRE(h && E && normP, "null argument");
        const int k = h->center;
        const int n = int(h->sites[k - 1].size);
        ensure_davidson(h, std::max(h->dav_sub, 2));
        // always FP64 (also with SP_FP32)
        heff_apply(h, k, site_ptr(h, k), h->dHV.p, h->dNV.p, false, true);
        double* sm = h->dsmall.p;
        spk::multidot(h->stream, h->dHV.p, 0, 1, site_ptr(h, k), n, sm);
        spk::multidot(h->stream, h->dNV.p, 0, 1, site_ptr(h, k), n, sm + 1);
        spk::multidot(h->stream, site_ptr(h, k), 0, 1, site_ptr(h, k), n, sm + 2);
        HIPCK(hipMemcpyAsync(h->pin, sm, 3 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
        HIPCK(hipStreamSynchronize(h->stream));
        const double xy = h->pin[0], xny = h->pin[1], xx = h->pin[2];
        if (!(xx > 0.0) || !(std::fabs(xny) / xx >= 1e-12)) {
            *E = NAN;
            *normP = xx > 0.0 ? xny / xx : 0.0;
            throw SpError(SP_ENORM, "projected norm vanishes");
        }
        *E = xy / xny;
        *normP = xny / xx;
        return SP_OK;
    });
}

int sp_site_size(const sp_handle* h, int site, long long* n) {
    return guarded([&]() -> int {
        SP_REQUIRE(h && n, "null argument");
        check_site(h, site);
        *n = h->sites[site - 1].size;
        return SP_OK;
    });
}

int sp_get_site(sp_handle* h, int site, double* host) {
    return guarded([&]() -> int {
        SP_REQUIRE(h && host, "null argument");
        check_site(h, site);
        HIPCK(hipMemcpyAsync(host, site_ptr(h, site), h->sites[site - 1].size * sizeof(double),
                             hipMemcpyDeviceToHost, h->stream));
        HIPCK(hipStreamSynchronize(h->stream));
        return SP_OK;
    });
}

int sp_set_site(sp_handle* h, int site, const double* host) {
    return guarded([&]() -> int {
        SP_REQUIRE(h && host, "null argument");
        check_site(h, site);
        HIPCK(hipMemcpyAsync(site_ptr(h, site), host, h->sites[site - 1].size * sizeof(double),
                             hipMemcpyHostToDevice, h->stream));
        HIPCK(hipStreamSynchronize(h->stream));
        invalidate_for_site(h, site);
        return SP_OK;
    });
}

int sp_center(const sp_handle* h, int* site) {
    return guarded([&]() -> int {
        SP_REQUIRE(h && site, "null argument");
        *site = h->center;
        return SP_OK;
    });
}

int sp_heff_flops(const sp_handle* h, int site, double* flops) {
    return guarded([&]() -> int {
        SP_REQUIRE(h && flops, "null argument");
        check_site(h, site);
        *flops = h->plan[site - 1].heff_flops;
        return SP_OK;
    });
}

int sp_heff_batch_profile(sp_handle** hs, int n, const int* sites, int reps, double* out) {
    return guarded([&]() -> int {
        SP_REQUIRE(hs && sites && out && n >= 1 && reps >= 1, "bad arguments");
        hipStream_t s = hs[0]->stream;
        std::vector<spk::H3Inst> insts(n);
        std::map<int, std::vector<spk::H3Task>> by_rc;
        std::map<int, int> lds_by_rc;
        double flops = 0.0, bytes = 0.0;
        for (int i = 0; i < n; ++i) {
            sp_handle* h = hs[i];
            SP_REQUIRE(h, "null handle");
            check_site(h, sites[i]);
            const int k = sites[i];
            SP_REQUIRE(h->path == SP_PATH_TILED && h->plan[k - 1].h_rows > 0, "every site must have a fused plan");
            SP_REQUIRE(h->stream == s && h->device == hs[0]->device && h->precision == hs[0]->precision,
                       "one device, stream and precision");
            SP_REQUIRE(h->Lvalid[k - 1] && h->Rvalid[k], "environments are not built");
            for (int j = 0; j < i; ++j) SP_REQUIRE(hs[j] != h, "a handle appears twice");
            insts[i] = heff_inst(h, k, site_ptr(h, k), reduced(h));
            const SitePlan& P = h->plan[k - 1];
            for (spk::H3Task t : P.h_tasks) {
                if (t.blk < 0) continue;
                t.inst = i;
                by_rc[P.h_rows].push_back(t);
            }
            lds_by_rc[P.h_rows] = std::max(lds_by_rc[P.h_rows], P.h_lds);
            flops += P.heff_flops;
            const double G = h->G, xs = double(h->sites[k - 1].size);
            bytes += 8.0 * (G * h->env[k - 1].size + G * h->env[k].size + xs + 2.0 * G * xs);
        }
        std::vector<spk::H3Task> all;
        std::vector<std::pair<int, std::pair<size_t, int>>> groups;  // rc -> (first, count)
        for (auto& kv : by_rc) {
            groups.push_back({kv.first, {all.size(), int(kv.second.size())}});
            all.insert(all.end(), kv.second.begin(), kv.second.end());
        }
        DArr<spk::H3Inst> dinst;
        DArr<spk::H3Task> dtask;
        dinst.upload(insts, s);
        dtask.upload(all, s);
        HIPCK(hipStreamSynchronize(s));
        const bool f32 = reduced(hs[0]);
        auto launch_on = [&](hipStream_t st) {
            for (auto& gr : groups) {
                const int rc = gr.first;
                const spk::H3Task* tp = dtask.p + gr.second.first;
                if (f32) spk::heff3_f32(st, rc, lds_by_rc[rc], tp, gr.second.second, insts[0], dinst.p);
                else spk::heff3(st, rc, lds_by_rc[rc], tp, gr.second.second, insts[0], dinst.p);
            }
        };
        auto launch = [&]() { launch_on(s); };
        launch();  // warm-up
        hipEvent_t e0, e1;
        HIPCK(hipEventCreate(&e0));
        HIPCK(hipEventCreate(&e1));
        HIPCK(hipEventRecord(e0, s));
        for (int r = 0; r < reps; ++r) launch();
        HIPCK(hipEventRecord(e1, s));
        HIPCK(hipEventSynchronize(e1));
        float ms = 0.f;
        HIPCK(hipEventElapsedTime(&ms, e0, e1));
        HIPCK(hipGetLastError());
        out[0] = 1e3 * double(ms) / reps;
        out[1] = flops;
        out[2] = bytes;
        out[3] = double(all.size());

        // The same launches captured once in a HIP graph (on a private
        // stream: the handles' stream may be the null stream) and replayed.
        // Every checked replay follows eager work that clears the partials,
        // and its partials must equal the eager launch's bit for bit.
        std::vector<std::vector<double>> ref(n), got(n);
        auto partials = [&](std::vector<std::vector<double>>& dst) {
            for (int i = 0; i < n; ++i) {
                const size_t m = size_t(hs[i]->G) * hs[i]->sites[sites[i] - 1].size;
                dst[i].resize(2 * m);
                HIPCK(hipMemcpy(dst[i].data(), hs[i]->ypart.p, m * sizeof(double), hipMemcpyDeviceToHost));
                HIPCK(hipMemcpy(dst[i].data() + m, hs[i]->nypart.p, m * sizeof(double), hipMemcpyDeviceToHost));
            }
        };
        launch();
        HIPCK(hipStreamSynchronize(s));
        partials(ref);
        hipStream_t gs = nullptr;
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        HIPCK(hipStreamCreateWithFlags(&gs, hipStreamNonBlocking));
        HIPCK(hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal));
        launch_on(gs);
        HIPCK(hipStreamEndCapture(gs, &graph));
        HIPCK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
        double maxdiff = 0.0;
        for (int c = 0; c < 3; ++c) {
            for (int i = 0; i < n; ++i) {
                const long long m = (long long)hs[i]->G * hs[i]->sites[sites[i] - 1].size;
                spk::fill(s, hs[i]->ypart.p, m, 0.0);
                spk::fill(s, hs[i]->nypart.p, m, 0.0);
            }
            HIPCK(hipStreamSynchronize(s));
            HIPCK(hipGraphLaunch(exec, gs));
            HIPCK(hipStreamSynchronize(gs));
            partials(got);
            for (int i = 0; i < n; ++i)
                for (size_t e = 0; e < ref[i].size(); ++e)
                    maxdiff = std::max(maxdiff, std::fabs(got[i][e] - ref[i][e]));
        }
        HIPCK(hipEventRecord(e0, gs));
        for (int r = 0; r < reps; ++r) HIPCK(hipGraphLaunch(exec, gs));
        HIPCK(hipEventRecord(e1, gs));
        HIPCK(hipEventSynchronize(e1));
        float gms = 0.f;
        HIPCK(hipEventElapsedTime(&gms, e0, e1));
        (void)hipGraphExecDestroy(exec);
        (void)hipGraphDestroy(graph);
        (void)hipStreamDestroy(gs);
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        HIPCK(hipGetLastError());
        out[4] = 1e3 * double(gms) / reps;
        out[5] = maxdiff;
        return SP_OK;
    });
}

int sp_heff_profile(sp_handle* h, int site, int reps, const double* x, double* y, double* ny, double* out) {
    return guarded([&]() -> int {
        SP_REQUIRE(h && x && y && ny && out && reps >= 1, "bad arguments");
        check_site(h, site);
        if (!h->Lvalid[site - 1] || !h->Rvalid[site]) throw SpError(SP_ESTATE, "environments are not built");
        SitePlan& P = h->plan[site - 1];
        hipStream_t s = h->stream;
        const bool plain = h->path == SP_PATH_PLAIN;
        const spk::BufSet b = plain ? bufset(h, site, x, y, ny, nullptr)
                                    : bufset(h, site, h->Xd.p, h->ypart.p, h->nypart.p, nullptr);
        const int n = int(h->sites[site - 1].size);
        hipEvent_t ev[4];
        for (auto& e : ev) HIPCK(hipEventCreate(&e));
        double ms[3] = {0, 0, 0};
        double premix_ms = 0.0;
        if (!plain && P.h_rows == 0) {
            // the pre-mixed left environment of the block products is built
            // once per local problem and reused by every product of the
            // solve: timed on its own, outside the products
            HIPCK(hipEventRecord(ev[0], s));
            P.premix.launch(s, b, P.coef.p);
            HIPCK(hipEventRecord(ev[1], s));
            HIPCK(hipEventSynchronize(ev[1]));
            float t = 0.f;
            HIPCK(hipEventElapsedTime(&t, ev[0], ev[1]));
            premix_ms = t;
            h->lt_site = site;
            h->lt_gen = h->Lgen[site - 1];
        }
        for (int r = 0; r < reps; ++r) {
            HIPCK(hipEventRecord(ev[0], s));
            if (plain) {
                P.p1.launch(s, b, P.coef.p);
            } else {
                heff_apply(h, site, x, nullptr, nullptr, true);
            }
            HIPCK(hipEventRecord(ev[1], s));
            if (plain) P.mixl.launch(s, b, P.coef.p);
            HIPCK(hipEventRecord(ev[2], s));
            if (plain) {
                P.yout.launch(s, b, P.coef.p);
            } else {
                spk::gsum2(s, h->ypart.p, h->nypart.p, n, heff_parts(h, site), n, y, ny);
            }
            HIPCK(hipEventRecord(ev[3], s));
            HIPCK(hipEventSynchronize(ev[3]));
            for (int i = 0; i < 3; ++i) {
                float t = 0.f;
                HIPCK(hipEventElapsedTime(&t, ev[i], ev[i + 1]));
                ms[i] += t;
            }
        }
        for (auto& e : ev) (void)hipEventDestroy(e);
        const double G = h->G, xs = double(h->sites[site - 1].size);
        const double Lb = G * h->env[site - 1].size, Rb = G * h->env[site].size;
        for (int i = 0; i < 3; ++i) out[i] = ms[i] / reps;
        if (plain) {
            out[3] = P.p1.flops;
            out[4] = P.mixl.flops;
            out[5] = P.yout.flops;
            out[6] = 8.0 * (Lb + xs + G * P.Tsize);
            out[7] = 8.0 * (G * P.Tsize + G * P.Vsize);
            out[8] = 8.0 * (G * P.Vsize + G * P.Tsize + Rb + 2.0 * xs);
        } else {
            // the product into per-g partials (the fused launch, or the tiled
            // lists at a site without a fused plan): environments and x read
            // once, per-g partials written
            out[1] = premix_ms;
            out[3] = P.p1.flops + P.mixl.flops + P.yout.flops;
            out[4] = P.h_rows == 0 ? P.premix.flops : 0.0;
            out[5] = 2.0 * G * xs;
            out[6] = 8.0 * (Lb + Rb + xs + 2.0 * G * xs);
            out[7] = 0.0;
            out[8] = 8.0 * (2.0 * G * xs + 2.0 * xs);
        }
        HIPCK(hipGetLastError());
        return SP_OK;
    });
}

int sp_quadrature(int G, int twoS, int twoM, double* x, double* w, double* coef) {
    return guarded([&]() -> int {
        SP_REQUIRE(G >= 1 && G <= 1024 && x && w && coef, "bad arguments");
        SP_REQUIRE(twoS >= 0 && std::abs(twoM) <= twoS && (twoS - twoM) % 2 == 0, "need |M| <= S, S - M integer");
        std::vector<double> c(G), s(G);
        sph::projector_quadrature(G, twoS, twoM, x, w, c.data(), s.data(), coef);
        return SP_OK;
    });
}

int sp_exact_points(int N, int K, int twoS, int twoM) { return sph::exact_points(N, K, twoS, twoM); }

int sp_mpo_hubbard(int L, double t, double U, int* w, double* data, long long* n) {
    return guarded([&]() -> int {
        SP_REQUIRE(L >= 1 && w && n, "bad arguments");
        return sph::mpo_hubbard(L, t, U, w, data, n);
    });
}
int sp_mpo_s2(int L, int* w, double* data, long long* n) {
    return guarded([&]() -> int {
        SP_REQUIRE(L >= 1 && w && n, "bad arguments");
        return sph::mpo_s2(L, w, data, n);
    });
}
int sp_mpo_identity(int L, int* w, double* data, long long* n) {
    return guarded([&]() -> int {
        SP_REQUIRE(L >= 1 && w && n, "bad arguments");
        return sph::mpo_identity(L, w, data, n);
    });
}

int sp_mpo_site_op(int L, int p, const double* op, int* w, double* data, long long* n) {
    return guarded([&]() -> int {
        SP_REQUIRE(L >= 1 && p >= 1 && p <= L && op && w && n, "bad arguments");
        return sph::mpo_site_op(L, p, op, w, data, n);
    });
}
int sp_mpo_epq(int L, int p, int q, int* w, double* data, long long* n) {
    return guarded([&]() -> int {
        SP_REQUIRE(L >= 1 && p >= 1 && p <= L && q >= 1 && q <= L && w && n, "bad arguments");
        return sph::mpo_epq(L, p, q, w, data, n);
    });
}
int sp_mpo_spin_corr(int L, int X, int Y, int* w, double* data, long long* n) {
    return guarded([&]() -> int {
        SP_REQUIRE(L >= 1 && X >= 1 && X <= L && Y >= 1 && Y <= L && w && n, "bad arguments");
        return sph::mpo_spin_corr(L, X, Y, w, data, n);
    });
}

int sp_mpo_abinitio(int K, const double* h, const double* eri, int* w, double* data, long long* n) {
    return guarded([&]() -> int {
        SP_REQUIRE(K >= 2 && K <= 64 && h && eri && w && n, "bad arguments");
        const int r = sph::mpo_abinitio(K, h, eri, w, data, n);
        SP_REQUIRE(r != -2, "ab-initio MPO: a bond needs more than 4096 channels");
        SP_REQUIRE(r == 0, "ab-initio MPO: internal error");
        return 0;
    });
}

int sp_mpo_abinitio_component(int K, int p, const double* h, const double* eri, int* w, double* data, long long* n) {
    return guarded([&]() -> int {
        SP_REQUIRE(K >= 2 && K <= 64 && h && eri && w && n, "bad arguments");
        SP_REQUIRE(p >= 1 && p <= K, "orbital p out of range");
        const int r = sph::mpo_abinitio(K, h, eri, w, data, n, p - 1);
        SP_REQUIRE(r != -2, "ab-initio MPO: a bond needs more than 4096 channels");
        SP_REQUIRE(r == 0, "ab-initio MPO: internal error");
        return 0;
    });
}

int sp_mpo_hubbard_component(int L, int p, double t, double U, int* w, double* data, long long* n) {
    return guarded([&]() -> int {
        SP_REQUIRE(L >= 2 && L <= 64 && w && n, "bad arguments");
        SP_REQUIRE(p >= 1 && p <= L, "site p out of range");
        // the open chain as integrals: h = -t on nearest neighbours, (pp|pp) = U
        std::vector<double> hh(size_t(L) * L, 0.0), eri(size_t(L) * L * L * L, 0.0);
        for (int q = 0; q + 1 < L; ++q) hh[size_t(q) * L + q + 1] = hh[size_t(q + 1) * L + q] = -t;
        for (int q = 0; q < L; ++q) eri[((size_t(q) * L + q) * L + q) * L + q] = U;
        const int r = sph::mpo_abinitio(L, hh.data(), eri.data(), w, data, n, p - 1);
        SP_REQUIRE(r == 0, "Hubbard component MPO: internal error");
        return 0;
    });
}

int sp_small_gen_lowest(int m, const double* H, const double* N, double drop, double* theta, double* a,
                        int* rank) {
    return guarded([&]() -> int {
        SP_REQUIRE(m >= 1 && H && N && theta && a && rank, "bad arguments");
        const int r = sph::gen_lowest(m, H, N, drop, theta, a, nullptr, rank);
        if (r < 0) throw SpError(SP_ENAN, "subspace eigensolver failed");
        if (r == 0) throw SpError(SP_ENORM, "the metric vanishes");
        return SP_OK;
    });
}

int sp_small_gen_lowest_gpu(int m, double* H, double* N, double drop, int need_all, int keep, double* theta,
                            double* a, double* Qk, int* rank) {
    return guarded([&]() -> int {
        SP_REQUIRE(m >= 1 && m < spk::kDevSubMax && H && N && theta && a && rank, "bad arguments");
        SP_REQUIRE(!need_all || (Qk && keep >= 1 && keep <= spk::kDevKeepMax), "bad restart arguments");
        const int r = spk::dev_small_solve(m, H, N, drop, need_all, keep, theta, a, Qk);
        SP_REQUIRE(r >= 0, "device subspace solve failed");
        *rank = r;
        if (r == 0) throw SpError(SP_ENORM, "the projected metric vanishes");
        return SP_OK;
    });
}

int sp_small_eigh(int n, double* a, double* ev, double* vec) {
    return guarded([&]() -> int {
        SP_REQUIRE(n >= 0 && a && ev && vec, "bad arguments");
        if (sph::sym_eigh(n, a, ev, vec) != 0) throw SpError(SP_ENAN, "eigensolver did not converge");
        return SP_OK;
    });
}

}  // extern "C"
