// Host-side numerics of the SP-MPS library: projector quadrature, MPO
// construction and the small symmetric eigensolver of the Davidson subspace.
#include "host_linalg.h"

#include <algorithm>
#include <functional>
#include <map>
#include <tuple>
#include <cmath>
#include <numeric>
#include <vector>

namespace sph {

// ---------------------------------------------------------------------------
// Gauss-Legendre nodes by Newton's method on P_G (three-term recurrence for
// P_G and its derivative), weights 2 / ((1 - x^2) P_G'(x)^2).  Initial
// guesses cos(pi (i + 3/4) / (G + 1/2)).

static void legendre_pair(int G, double x, double& p, double& dp) {
    double p0 = 1.0, p1 = x;
    if (G == 0) {
        p = 1.0;
        dp = 0.0;
        return;
    }
    for (int j = 1; j < G; ++j) {
        const double p2 = ((2.0 * j + 1.0) * x * p1 - j * p0) / (j + 1.0);
        p0 = p1;
        p1 = p2;
    }
    p = p1;
    dp = G * (x * p1 - p0) / (x * x - 1.0);
}

void gauss_legendre(int G, double* x, double* w) {
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < G; ++i) {
        double z = std::cos(pi * (i + 0.75) / (G + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p, dp;
            legendre_pair(G, z, p, dp);
            const double dz = p / dp;
            z -= dz;
            if (std::fabs(dz) <= 1e-16 * std::max(1.0, std::fabs(z))) break;
        }
        double p, dp;
        legendre_pair(G, z, p, dp);
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
    // ascending order
    std::vector<int> idx(G);
    std::iota(idx.begin(), idx.end(), 0);
    std::sort(idx.begin(), idx.end(), [&](int a, int b) { return x[a] < x[b]; });
    std::vector<double> xs(G), ws(G);
    for (int i = 0; i < G; ++i) {
        xs[i] = x[idx[i]];
        ws[i] = w[idx[i]];
    }
    std::copy(xs.begin(), xs.end(), x);
    std::copy(ws.begin(), ws.end(), w);
}

// d^J_MM at cos(beta) = x through the Jacobi polynomial
// d^J_MM = cos(beta/2)^(2|M|) P^(0, 2|M|)_(J-|M|)(x), with cos(beta/2)^2 =
// (1 + x)/2 and d^J_MM = d^J_{-M,-M}.
double wigner_d_diag(int twoJ, int twoM, double x) {
    const int b = std::abs(twoM);
    const int n = (twoJ - b) / 2;
    double P0 = 1.0;
    double P1 = 1.0 + (b + 2.0) * (x - 1.0) / 2.0;
    double Pn = (n == 0) ? P0 : P1;
    for (int k = 2; k <= n; ++k) {
        const double A = 2.0 * k * (k + b) * (2.0 * k + b - 2.0);
        const double B = (2.0 * k + b - 1.0) * ((2.0 * k + b) * (2.0 * k + b - 2.0) * x - double(b) * b);
        const double C = 2.0 * (k - 1.0) * (k + b - 1.0) * (2.0 * k + b);
        Pn = (B * P1 - C * P0) / A;
        P0 = P1;
        P1 = Pn;
    }
    const double half = (1.0 + x) / 2.0;
    double pre = std::pow(half, b / 2);
    if (b % 2) pre *= std::sqrt(half);
    return pre * Pn;
}

int max_seniority(int N, int twoM, int K) {
    const int na = (N + twoM) / 2, nb = (N - twoM) / 2;
    return std::min(na, K - nb) + std::min(nb, K - na);
}

int exact_points(int N, int K, int twoS, int twoM) {
    const int om = max_seniority(N, twoM, K);
    return (om + twoS + 2 + 3) / 4;  // ceil((om + 2S + 2) / 4)
}

void projector_quadrature(int G, int twoS, int twoM, double* x, double* w, double* c, double* s,
                          double* coef) {
    gauss_legendre(G, x, w);
    for (int g = 0; g < G; ++g) {
        c[g] = std::sqrt((1.0 + x[g]) / 2.0);
        s[g] = std::sqrt((1.0 - x[g]) / 2.0);
        coef[g] = (twoS + 1) / 2.0 * w[g] * wigner_d_diag(twoS, twoM, x[g]);
    }
}

// ---------------------------------------------------------------------------
// local operators, basis (|0>, |b>, |a>, |ab>), |ab> = a+_alpha a+_beta |0>

using M4 = std::array<double, 16>;

static M4 zero4() { M4 m{}; m.fill(0.0); return m; }
static M4 eye4() { M4 m = zero4(); for (int i = 0; i < 4; ++i) m[i * 4 + i] = 1.0; return m; }
static M4 mul4(const M4& a, const M4& b) {
    M4 c = zero4();
    for (int i = 0; i < 4; ++i)
        for (int k = 0; k < 4; ++k)
            for (int j = 0; j < 4; ++j) c[i * 4 + j] += a[i * 4 + k] * b[k * 4 + j];
    return c;
}
static M4 tr4(const M4& a) {
    M4 c;
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) c[i * 4 + j] = a[j * 4 + i];
    return c;
}
static M4 scal4(double f, const M4& a) { M4 c; for (int i = 0; i < 16; ++i) c[i] = f * a[i]; return c; }

// annihilators: c_alpha |a> = |0>, c_alpha |ab> = |b>;
// c_beta |b> = |0>, c_beta |ab> = -|a> (the alpha occupation precedes beta)
static M4 c_alpha() { M4 m = zero4(); m[0 * 4 + 2] = 1.0; m[1 * 4 + 3] = 1.0; return m; }
static M4 c_beta() { M4 m = zero4(); m[0 * 4 + 1] = 1.0; m[2 * 4 + 3] = -1.0; return m; }
static M4 parity() { M4 m = eye4(); m[1 * 4 + 1] = -1.0; m[2 * 4 + 2] = -1.0; return m; }

struct MpoBuilder {
    int L, w;
    std::vector<M4> full;  // w*w operators of a bulk site
    M4& at(int a, int b) { return full[a * w + b]; }
};

static int emit(const MpoBuilder& mb, int* wout, double* data, long long* n) {
    const int L = mb.L, w = mb.w;
    long long total = 0;
    for (int k = 1; k <= L; ++k) {
        const int wl = (k == 1) ? 1 : w;
        const int wr = (k == L) ? 1 : w;
        total += (long long)wl * wr * 16;
    }
    if (wout) {
        for (int k = 0; k <= L; ++k) wout[k] = (k == 0 || k == L) ? 1 : w;
    }
    if (n) *n = total;
    if (!data) return 0;
    long long pos = 0;
    for (int k = 1; k <= L; ++k) {
        const int a0 = 0, a1 = (k == 1) ? 1 : w;           // first row at site 1
        const int b0 = (k == L) ? w - 1 : 0, b1 = w;        // last column at site L
        for (int a = a0; a < a1; ++a)
            for (int b = b0; b < b1; ++b)
                for (int e = 0; e < 16; ++e) data[pos++] = mb.full[a * w + b][e];
    }
    return 0;
}

int mpo_hubbard(int L, double t, double U, int* w, double* data, long long* n) {
    MpoBuilder mb{L, 6, std::vector<M4>(36, zero4())};
    const M4 ca = c_alpha(), cb = c_beta(), F = parity();
    const M4 cda = tr4(ca), cdb = tr4(cb);
    mb.at(0, 0) = eye4();
    mb.at(0, 1) = scal4(-t, mul4(cda, F));
    mb.at(0, 2) = scal4(-t, mul4(cdb, F));
    mb.at(0, 3) = scal4(-t, mul4(F, ca));
    mb.at(0, 4) = scal4(-t, mul4(F, cb));
    M4 nn = zero4();
    nn[15] = U;
    mb.at(0, 5) = nn;
    mb.at(1, 5) = ca;
    mb.at(2, 5) = cb;
    mb.at(3, 5) = cda;
    mb.at(4, 5) = cdb;
    mb.at(5, 5) = eye4();
    return emit(mb, w, data, n);
}

int mpo_s2(int L, int* w, double* data, long long* n) {
    MpoBuilder mb{L, 5, std::vector<M4>(25, zero4())};
    M4 sp = zero4(), sm = zero4(), sz = zero4(), s2 = zero4();
    sp[2 * 4 + 1] = 1.0;
    sm[1 * 4 + 2] = 1.0;
    sz[1 * 4 + 1] = -0.5;
    sz[2 * 4 + 2] = 0.5;
    s2[1 * 4 + 1] = 0.75;
    s2[2 * 4 + 2] = 0.75;
    mb.at(0, 0) = eye4();
    mb.at(0, 1) = sm;
    mb.at(0, 2) = sp;
    mb.at(0, 3) = scal4(2.0, sz);
    mb.at(0, 4) = s2;
    mb.at(1, 1) = eye4();
    mb.at(1, 4) = sp;
    mb.at(2, 2) = eye4();
    mb.at(2, 4) = sm;
    mb.at(3, 3) = eye4();
    mb.at(3, 4) = sz;
    mb.at(4, 4) = eye4();
    return emit(mb, w, data, n);
}

// site-dependent MPOs: full[k-1] holds the w x w operators of site k
static int emit_sites(int L, int w, const std::vector<std::vector<M4>>& full, int* wout, double* data,
                      long long* n) {
    long long total = 0;
    for (int k = 1; k <= L; ++k) total += (long long)((k == 1) ? 1 : w) * ((k == L) ? 1 : w) * 16;
    if (wout)
        for (int k = 0; k <= L; ++k) wout[k] = (k == 0 || k == L) ? 1 : w;
    if (n) *n = total;
    if (!data) return 0;
    long long pos = 0;
    for (int k = 1; k <= L; ++k) {
        const int a1 = (k == 1) ? 1 : w;
        const int b0 = (k == L) ? w - 1 : 0;
        for (int a = 0; a < a1; ++a)
            for (int b = b0; b < w; ++b)
                for (int e = 0; e < 16; ++e) data[pos++] = full[k - 1][a * w + b][e];
    }
    return 0;
}

// channel 0 = nothing applied yet, channel w-1 = complete (identity carried
// on both), in between: open two-site terms
static std::vector<std::vector<M4>> blank_sites(int L, int w) {
    std::vector<std::vector<M4>> full(L, std::vector<M4>(size_t(w) * w, zero4()));
    for (int k = 0; k < L; ++k) {
        full[k][0] = eye4();
        full[k][size_t(w - 1) * w + (w - 1)] = eye4();
    }
    return full;
}

int mpo_site_op(int L, int p, const double* op, int* w, double* data, long long* n) {
    if (p < 1 || p > L) return -1;
    auto full = blank_sites(L, 2);
    M4 m;
    for (int e = 0; e < 16; ++e) m[e] = op[e];
    full[p - 1][0 * 2 + 1] = m;
    return emit_sites(L, 2, full, w, data, n);
}

int mpo_epq(int L, int p, int q, int* w, double* data, long long* n) {
    if (p < 1 || p > L || q < 1 || q > L) return -1;
    if (p == q) {
        const M4 ca = c_alpha(), cb = c_beta();
        const M4 nsum = [&] {
            M4 a = mul4(tr4(ca), ca), b = mul4(tr4(cb), cb), r;
            for (int e = 0; e < 16; ++e) r[e] = a[e] + b[e];
            return r;
        }();
        return mpo_site_op(L, p, nsum.data(), w, data, n);
    }
    // sum over sigma of a+_{p sigma} a_{q sigma}: channels 1 (alpha) and 2
    // (beta) carry the open term with the site parity as Jordan-Wigner
    // string; the left end takes (a+ F) or (F a), the right end the bare
    // operator, as in the hopping terms of the Hubbard MPO
    const M4 ca = c_alpha(), cb = c_beta(), F = parity();
    const M4 cda = tr4(ca), cdb = tr4(cb);
    auto full = blank_sites(L, 4);
    const int lo = std::min(p, q), hi = std::max(p, q);
    const bool create_left = p < q;
    full[lo - 1][0 * 4 + 1] = create_left ? mul4(cda, F) : mul4(F, ca);
    full[lo - 1][0 * 4 + 2] = create_left ? mul4(cdb, F) : mul4(F, cb);
    for (int k = lo + 1; k < hi; ++k) {
        full[k - 1][1 * 4 + 1] = F;
        full[k - 1][2 * 4 + 2] = F;
    }
    full[hi - 1][1 * 4 + 3] = create_left ? ca : cda;
    full[hi - 1][2 * 4 + 3] = create_left ? cb : cdb;
    return emit_sites(L, 4, full, w, data, n);
}

int mpo_spin_corr(int L, int X, int Y, int* w, double* data, long long* n) {
    if (X < 1 || X > L || Y < 1 || Y > L) return -1;
    M4 sp = zero4(), sm = zero4(), sz = zero4(), s2 = zero4();
    sp[2 * 4 + 1] = 1.0;
    sm[1 * 4 + 2] = 1.0;
    sz[1 * 4 + 1] = -0.5;
    sz[2 * 4 + 2] = 0.5;
    s2[1 * 4 + 1] = 0.75;
    s2[2 * 4 + 2] = 0.75;
    if (X == Y) return mpo_site_op(L, X, s2.data(), w, data, n);
    // S_X.S_Y = Sz Sz + (S+ S- + S- S+)/2: spin operators are even, no string
    const int lo = std::min(X, Y), hi = std::max(X, Y);
    auto full = blank_sites(L, 5);
    full[lo - 1][0 * 5 + 1] = sz;
    full[lo - 1][0 * 5 + 2] = scal4(0.5, sp);
    full[lo - 1][0 * 5 + 3] = scal4(0.5, sm);
    for (int k = lo + 1; k < hi; ++k)
        for (int c = 1; c <= 3; ++c) full[k - 1][size_t(c) * 5 + c] = eye4();
    full[hi - 1][1 * 5 + 4] = sz;
    full[hi - 1][2 * 5 + 4] = sm;
    full[hi - 1][3 * 5 + 4] = sp;
    return emit_sites(L, 5, full, w, data, n);
}

int mpo_identity(int L, int* w, double* data, long long* n) {
    MpoBuilder mb{L, 1, std::vector<M4>(1, eye4())};
    return emit(mb, w, data, n);
}

// ---------------------------------------------------------------------------
// Ab-initio Hamiltonian (Eq. [sqH], real orbitals, chemists' integrals)
//   H = sum_pq h_pq sum_s a+_ps a_qs + 1/2 sum_pqrs (pq|rs) sum_st a+_ps a+_rt a_st a_qs
// as an MPO whose channels at a bond hold partial operator products.
//
// Every term is first brought to site order: a stable sort of its fermion
// operators by site (operators on different sites anticommute, so the sign is
// the parity of the sort; operators on one site keep their order).  Under the
// Jordan-Wigner mapping of Sec. 2.1 the site factor of a site-ordered even
// product at site j is (product of its operators at j) x F^(number of its
// operators on later sites), F the site parity.  Across a bond the product
// therefore splits into a left part fixed by the left operators and the
// parity of the right count, and a right part fixed by the right operators.
//
// A term waits at a bond either in a "left" channel, named by its left part
// (terms with the same left part share it; the coefficient is not applied
// yet), or in a "right" channel, named by its right part (coefficient already
// applied).  It uses the left form while fewer of its operators lie left of
// the bond than right of it, and on a tie when the left side of the chain is
// not longer than the right; once it switches it stays in right channels.
// The coefficient enters on the one edge where a term switches.  With at most
// two operators on the named side, a bond carries O(K^2) channels.
//
// With only_p >= 0 (0-based) only the terms whose first creator acts on
// orbital only_p are built: the energy component H_p of Sec. 2.4,
//   H_p = sum_q h_pq sum_s a+_ps a_qs + 1/2 sum_qrs (pq|rs) sum_st a+_ps a+_rt a_st a_qs,
// so that sum_p H_p = H and every H_p contains both spin orbitals of p.

namespace {
struct FOp {
    int site, spin, dag;  // site 1-based, spin 0 = alpha, dag 1 = creator
    bool operator<(const FOp& o) const {
        return std::tie(site, spin, dag) < std::tie(o.site, o.spin, o.dag);
    }
};
// channel label: kind (0 left, 1 right), right-count parity (left kind), ops
using Label = std::vector<int>;
}  // namespace

int mpo_abinitio(int K, const double* h, const double* eri, int* wout, double* data, long long* n, int only_p) {
    if (K < 2 || K > 64 || !h || !eri || only_p >= K) return -1;
    const M4 ca = c_alpha(), cb = c_beta(), F = parity(), I = eye4();
    const M4 cda = tr4(ca), cdb = tr4(cb);
    auto local = [&](const FOp& o) -> const M4& {
        return o.spin == 0 ? (o.dag ? cda : ca) : (o.dag ? cdb : cb);
    };
    // enumerate the terms: f(coef, ops in operator order)
    auto for_terms = [&](const std::function<void(double, std::vector<FOp>)>& f) {
        const int p0 = only_p < 0 ? 0 : only_p, p1 = only_p < 0 ? K : only_p + 1;
        for (int p = p0; p < p1; ++p)
            for (int q = 0; q < K; ++q) {
                const double v = h[p * K + q];
                if (v == 0.0) continue;
                for (int s = 0; s < 2; ++s) f(v, {{p + 1, s, 1}, {q + 1, s, 0}});
            }
        for (int p = p0; p < p1; ++p)
            for (int q = 0; q < K; ++q)
                for (int r = 0; r < K; ++r)
                    for (int t = 0; t < K; ++t) {
                        const double v = eri[((size_t(p) * K + q) * K + r) * K + t];
                        if (v == 0.0) continue;
                        for (int a = 0; a < 2; ++a)
                            for (int b = 0; b < 2; ++b)
                                f(0.5 * v, {{p + 1, a, 1}, {r + 1, b, 1}, {t + 1, b, 0}, {q + 1, a, 0}});
                    }
    };
    // site order, sign and site factors; false if the product vanishes
    struct Term {
        double coef;
        std::vector<FOp> ops;  // site-ordered
        std::vector<M4> f;     // factors of sites pmin..pmax
        int pmin, pmax;
    };
    auto prepare = [&](double coef, std::vector<FOp> ops, Term& T) -> bool {
        int inv = 0;
        for (size_t i = 0; i < ops.size(); ++i)
            for (size_t j = i + 1; j < ops.size(); ++j)
                if (ops[i].site > ops[j].site) ++inv;
        std::stable_sort(ops.begin(), ops.end(), [](const FOp& a, const FOp& b) { return a.site < b.site; });
        T.coef = (inv & 1) ? -coef : coef;
        T.pmin = ops.front().site;
        T.pmax = ops.back().site;
        T.f.clear();
        for (int j = T.pmin; j <= T.pmax; ++j) {
            M4 m = I;
            int later = 0;
            for (const FOp& o : ops) {
                if (o.site == j) m = mul4(m, local(o));
                if (o.site > j) ++later;
            }
            if (later & 1) m = mul4(m, F);
            bool nz = false;
            for (double x : m) nz = nz || x != 0.0;
            if (!nz) return false;
            T.f.push_back(m);
        }
        T.ops = std::move(ops);
        return true;
    };
    // channel of term T at inner bond b (pmin <= b < pmax)
    auto label_at = [&](const Term& T, int b) -> Label {
        int nl = 0;
        for (const FOp& o : T.ops) nl += o.site <= b;
        const int nr = int(T.ops.size()) - nl;
        const bool left = nl < nr || (nl == nr && b <= K - b);
        Label lab{left ? 0 : 1, left ? (nr & 1) : 0};
        for (const FOp& o : T.ops)
            if ((o.site <= b) == left) {
                lab.push_back(o.site);
                lab.push_back(o.spin);
                lab.push_back(o.dag);
            }
        return lab;
    };
    // pass 1: the channels of every bond
    std::vector<std::map<Label, int>> chan(K + 1);
    Term T;
    for_terms([&](double c, std::vector<FOp> ops) {
        if (!prepare(c, std::move(ops), T)) return;
        for (int b = T.pmin; b < T.pmax; ++b) chan[b].emplace(label_at(T, b), 0);
    });
    // numbering: 0 = nothing applied yet, then left channels, then right
    // channels (map order puts kind 0 first), last = complete
    std::vector<int> w(K + 1, 1);
    for (int b = 1; b < K; ++b) {
        int i = 1;
        for (auto& kv : chan[b]) kv.second = i++;
        w[b] = i + 1;
        if (w[b] > 4096) return -2;
    }
    long long total = 0;
    for (int k = 1; k <= K; ++k) total += (long long)w[k - 1] * w[k] * 16;
    if (wout)
        for (int k = 0; k <= K; ++k) wout[k] = w[k];
    if (n) *n = total;
    if (!data) return 0;
    // pass 2: the edges
    std::vector<std::map<std::pair<int, int>, M4>> edge(K + 1);
    for (int k = 1; k <= K; ++k) {
        if (k < K) edge[k][{0, 0}] = I;
        if (k > 1) edge[k][{w[k - 1] - 1, w[k] - 1}] = I;
    }
    for_terms([&](double c, std::vector<FOp> ops) {
        if (!prepare(c, std::move(ops), T)) return;
        int a = 0;
        bool a_left = true;  // "nothing applied yet" counts as a left channel
        for (int k = T.pmin; k <= T.pmax; ++k) {
            int b;
            bool b_left;
            if (k == T.pmax) {
                b = w[k] - 1;
                b_left = false;
            } else {
                const Label lab = label_at(T, k);
                b = chan[k].at(lab);
                b_left = lab[0] == 0;
            }
            const M4& fk = T.f[size_t(k - T.pmin)];
            auto it = edge[k].find({a, b});
            if (a_left && !b_left) {  // the switch: the coefficient enters here
                const M4 add = scal4(T.coef, fk);
                if (it == edge[k].end()) edge[k][{a, b}] = add;
                else
                    for (int e = 0; e < 16; ++e) it->second[e] += add[e];
            } else {
                edge[k][{a, b}] = fk;
            }
            a = b;
            a_left = b_left;
        }
    });
    std::fill(data, data + total, 0.0);
    long long pos = 0;
    for (int k = 1; k <= K; ++k) {
        const int wl = w[k - 1], wr = w[k];
        for (auto& kv : edge[k]) {
            const int a = kv.first.first, b = kv.first.second;
            if (a >= wl || b >= wr) return -3;
            std::copy(kv.second.begin(), kv.second.end(), data + pos + (size_t(a) * wr + b) * 16);
        }
        pos += (long long)wl * wr * 16;
    }
    return 0;
}

// ---------------------------------------------------------------------------
// Symmetric eigensolver: Householder reduction to tridiagonal form with the
// transformations accumulated, then implicit symmetric QR steps with
// Wilkinson shifts (Givens bulge chase), deflating at negligible
// off-diagonals.  Eigenvalues ascending; eigenvectors are columns of vec.

// Householder reduction of a symmetric matrix to tridiagonal form.  On
// return d, e hold the diagonal and the off-diagonal (e[i] couples i, i+1) and
// the Householder vectors are kept in hv (row k: the vector of step k, length
// n-k-1, scaled so that H_k = I - beta_k v v^T) with their betas.
struct Tridiag {
    int n;
    std::vector<double> d, e, hv, beta;
};

static void tridiagonalize(int n, double* a, Tridiag& T) {
    T.n = n;
    T.d.assign(n, 0.0);
    T.e.assign(n, 0.0);
    T.hv.assign(size_t(n) * n, 0.0);
    T.beta.assign(n, 0.0);
    std::vector<double> p(n), wv(n);
    auto A = [&](int i, int j) -> double& { return a[size_t(i) * n + j]; };
    for (int k = 0; k + 2 < n; ++k) {
        const int len = n - k - 1;
        double* v = &T.hv[size_t(k) * n];
        double ss = 0.0;
        for (int i = 0; i < len; ++i) {
            v[i] = A(k + 1 + i, k);
            ss += v[i] * v[i];
        }
        const double nrm = std::sqrt(ss);
        if (nrm == 0.0) continue;
        const double x0 = v[0];
        const double alpha = (x0 >= 0.0) ? -nrm : nrm;
        v[0] = x0 - alpha;
        const double vv = ss - x0 * x0 + v[0] * v[0];
        if (vv == 0.0) continue;
        const double beta = 2.0 / vv;
        T.beta[k] = beta;
        // trailing block S = A[k+1:, k+1:]:  S -= v w^T + w v^T
        // (dot products with four independent partial sums)
        double vp = 0.0;
        for (int i = 0; i < len; ++i) {
            const double* row = &A(k + 1 + i, k + 1);
            double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
            int j = 0;
            for (; j + 4 <= len; j += 4) {
                s0 += row[j] * v[j];
                s1 += row[j + 1] * v[j + 1];
                s2 += row[j + 2] * v[j + 2];
                s3 += row[j + 3] * v[j + 3];
            }
            for (; j < len; ++j) s0 += row[j] * v[j];
            p[i] = beta * ((s0 + s1) + (s2 + s3));
            vp += v[i] * p[i];
        }
        const double K = 0.5 * beta * vp;
        for (int i = 0; i < len; ++i) wv[i] = p[i] - K * v[i];
        for (int i = 0; i < len; ++i) {
            double* row = &A(k + 1 + i, k + 1);
            const double vi = v[i], wi = wv[i];
            for (int j = 0; j < len; ++j) row[j] -= vi * wv[j] + wi * v[j];
        }
        A(k + 1, k) = A(k, k + 1) = alpha;
        for (int i = 1; i < len; ++i) A(k + 1 + i, k) = A(k, k + 1 + i) = 0.0;
    }
    for (int i = 0; i < n; ++i) T.d[i] = A(i, i);
    for (int i = 0; i + 1 < n; ++i) T.e[i] = A(i + 1, i);
}

// apply Q = H_0 H_1 ... H_{n-3} to the columns of Z (n x nz, row-major):
// Z <- Q Z
static void apply_q(const Tridiag& T, double* Z, int nz) {
    const int n = T.n;
    std::vector<double> tmp(nz);
    for (int k = n - 3; k >= 0; --k) {
        if (T.beta[k] == 0.0) continue;
        const int len = n - k - 1;
        const double* v = &T.hv[size_t(k) * n];
        std::fill(tmp.begin(), tmp.end(), 0.0);
        for (int i = 0; i < len; ++i) {
            const double* row = Z + size_t(k + 1 + i) * nz;
            for (int c = 0; c < nz; ++c) tmp[c] += v[i] * row[c];
        }
        for (int i = 0; i < len; ++i) {
            double* row = Z + size_t(k + 1 + i) * nz;
            const double f = T.beta[k] * v[i];
            for (int c = 0; c < nz; ++c) row[c] -= f * tmp[c];
        }
    }
}

// implicit symmetric QR steps with Wilkinson shifts on the tridiagonal
// (d, e); rotations are applied to the rows of Zt (eigenvectors stored as
// rows, n x n) when Zt != nullptr.  Returns false if it does not converge.
static bool tridiag_qr(int n, double* d, double* e, double* Zt) {
    const double eps = 2.220446049250313e-16;
    int m = n - 1;
    int guard = 0;
    while (m > 0) {
        if (std::fabs(e[m - 1]) <= eps * (std::fabs(d[m - 1]) + std::fabs(d[m]))) {
            e[m - 1] = 0.0;
            --m;
            continue;
        }
        int l = m - 1;
        while (l > 0 && std::fabs(e[l - 1]) > eps * (std::fabs(d[l - 1]) + std::fabs(d[l]))) --l;
        if (l > 0) e[l - 1] = 0.0;
        if (++guard > 60 * n) return false;
        const double delta = 0.5 * (d[m - 1] - d[m]);
        const double b2 = e[m - 1] * e[m - 1];
        const double sg = (delta >= 0.0) ? 1.0 : -1.0;
        const double mu = d[m] - b2 / (delta + sg * std::sqrt(delta * delta + b2));
        double x = d[l] - mu;
        double z = e[l];
        for (int k = l; k < m; ++k) {
            const double r = std::sqrt(x * x + z * z);
            double c = 1.0, s = 0.0;
            if (r != 0.0) {
                c = x / r;
                s = z / r;
            }
            if (k > l) e[k - 1] = r;
            const double ak = d[k], bk = e[k], ck = d[k + 1];
            d[k] = c * c * ak + 2.0 * c * s * bk + s * s * ck;
            d[k + 1] = s * s * ak - 2.0 * c * s * bk + c * c * ck;
            e[k] = c * s * (ck - ak) + (c * c - s * s) * bk;
            if (k + 1 < m) {
                z = s * e[k + 1];  // bulge at (k, k+2)
                e[k + 1] = c * e[k + 1];
                x = e[k];
            }
            if (Zt) {
                double* rk = Zt + size_t(k) * n;
                double* rk1 = Zt + size_t(k + 1) * n;
                for (int j = 0; j < n; ++j) {
                    const double a0 = rk[j], a1 = rk1[j];
                    rk[j] = c * a0 + s * a1;
                    rk1[j] = -s * a0 + c * a1;
                }
            }
        }
    }
    return true;
}

int sym_eigh(int n, double* a, double* ev, double* vec) {
    if (n <= 0) return 0;
    Tridiag T;
    tridiagonalize(n, a, T);
    // eigenvectors of the tridiagonal as rows of Zt (rotations act on rows:
    // contiguous memory), then back-transformed by the Householder vectors
    std::vector<double> Zt(size_t(n) * n, 0.0);
    for (int i = 0; i < n; ++i) Zt[size_t(i) * n + i] = 1.0;
    std::vector<double> d = T.d, e = T.e;
    if (!tridiag_qr(n, d.data(), e.data(), Zt.data())) return -1;
    std::vector<int> idx(n);
    std::iota(idx.begin(), idx.end(), 0);
    std::sort(idx.begin(), idx.end(), [&](int i, int j) { return d[i] < d[j]; });
    // Z (n x n, column i = eigenvector i of the tridiagonal) = Zt^T, sorted
    std::vector<double> Z(size_t(n) * n);
    for (int i = 0; i < n; ++i) {
        ev[i] = d[idx[i]];
        const double* row = &Zt[size_t(idx[i]) * n];
        for (int r = 0; r < n; ++r) Z[size_t(r) * n + i] = row[r];
    }
    apply_q(T, Z.data(), n);
    std::copy(Z.begin(), Z.end(), vec);
    return 0;
}

// number of eigenvalues of the tridiagonal (d, e) below x (Sturm sequence
// of the LDL^T pivots of T - x I)
static int sturm_count(int n, const double* d, const double* e, double x) {
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

// solve (T - shift) z = z in place (Gaussian elimination with partial
// pivoting on the tridiagonal band) and normalise z
static void tridiag_inverse_step(int n, const double* d, const double* e, double shift, double* z) {
    std::vector<double> dd(n), du(n, 0.0), du2(n, 0.0), dl(n, 0.0);
    std::vector<char> swp(n, 0);
    for (int i = 0; i < n; ++i) dd[i] = d[i] - shift;
    for (int i = 0; i + 1 < n; ++i) du[i] = dl[i] = e[i];
    for (int i = 0; i + 1 < n; ++i) {
        if (std::fabs(dd[i]) >= std::fabs(dl[i])) {
            const double f = (dd[i] != 0.0) ? dl[i] / dd[i] : 0.0;
            dl[i] = f;
            dd[i + 1] -= f * du[i];
        } else {
            swp[i] = 1;
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
        if (!swp[i]) {
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
    nr = std::sqrt(nr);
    for (int i = 0; i < n; ++i) z[i] /= nr;
}

// Lowest eigenpair of a symmetric tridiagonal: bisection with Sturm counts
// narrows [lo, hi] around the lowest eigenvalue (lo stays strictly below
// it), inverse iteration shifted to lo gives the vector, and the Rayleigh
// quotient the value.
static void tridiag_lowest(int n, const double* d, const double* e, double* lam, double* z) {
    if (n == 1) {
        *lam = d[0];
        z[0] = 1.0;
        return;
    }
    double lo = d[0], hi = d[0];
    for (int i = 0; i < n; ++i) {
        const double r = (i > 0 ? std::fabs(e[i - 1]) : 0.0) + (i + 1 < n ? std::fabs(e[i]) : 0.0);
        lo = std::min(lo, d[i] - r);
        hi = std::max(hi, d[i] + r);
    }
    const double spread = std::max(hi - lo, 1e-300);
    lo -= 1e-3 * spread;
    hi += 1e-3 * spread;
    // count(lo) == 0 <= count(hi) - 1
    for (int it = 0; it < 200 && hi - lo > 1e-7 * spread; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (sturm_count(n, d, e, mid) >= 1) hi = mid;
        else lo = mid;
    }
    for (int i = 0; i < n; ++i) z[i] = 1.0 / std::sqrt(double(n)) * (1.0 + 0.01 * i);
    for (int it = 0; it < 3; ++it) tridiag_inverse_step(n, d, e, lo, z);
    double rq = 0.0;
    for (int i = 0; i < n; ++i) {
        double tz = d[i] * z[i];
        if (i > 0) tz += e[i - 1] * z[i - 1];
        if (i + 1 < n) tz += e[i] * z[i + 1];
        rq += z[i] * tz;
    }
    *lam = rq;
}

int sym_eig_lowest(int n, double* a, double* ev0, double* v0) {
    if (n <= 0) return 0;
    Tridiag T;
    tridiagonalize(n, a, T);
    std::vector<double> z(n);
    tridiag_lowest(n, T.d.data(), T.e.data(), ev0, z.data());
    if (!std::isfinite(*ev0)) return -1;
    apply_q(T, z.data(), 1);
    std::copy(z.begin(), z.end(), v0);
    return 0;
}

// Cholesky N = L L^T (row-major, lower); false if a pivot is not positive
static bool cholesky(int m, const double* N, double shift, std::vector<double>& L) {
    L.assign(size_t(m) * m, 0.0);
    for (int j = 0; j < m; ++j) {
        double dsum = N[size_t(j) * m + j] - shift;
        const double* lj = &L[size_t(j) * m];
        for (int k = 0; k < j; ++k) dsum -= lj[k] * lj[k];
        if (!(dsum > 0.0)) return false;
        const double ljj = std::sqrt(dsum);
        L[size_t(j) * m + j] = ljj;
        for (int i = j + 1; i < m; ++i) {
            const double* li = &L[size_t(i) * m];
            double s0 = N[size_t(i) * m + j], s1 = 0.0;
            int k = 0;
            for (; k + 2 <= j; k += 2) {
                s0 -= li[k] * lj[k];
                s1 -= li[k + 1] * lj[k + 1];
            }
            for (; k < j; ++k) s0 -= li[k] * lj[k];
            L[size_t(i) * m + j] = (s0 + s1) / ljj;
        }
    }
    return true;
}

int gen_lowest(int m, const double* H, const double* N, double drop, double* theta, double* a, double* Xc,
               int* rank) {
    if (m <= 0) return -1;
    // fast path (lowest pair only): if N - drop * U is positive definite,
    // where U >= lambda_max(N) is the Gershgorin bound, no eigenvalue of N is
    // dropped, and the restriction is the whole space: reduce with the
    // Cholesky factor of N instead of its eigenvectors
    if (!Xc) {
        double U = 0.0;
        for (int i = 0; i < m; ++i) {
            double r = 0.0;
            for (int j = 0; j < m; ++j) r += std::fabs(N[size_t(i) * m + j]);
            U = std::max(U, r);
        }
        std::vector<double> L;
        if (U > 1e-12 && cholesky(m, N, drop * U, L) && cholesky(m, N, 0.0, L)) {
            // W = L^-1 H (columns by forward substitution), B = L^-1 W^T
            std::vector<double> W(H, H + size_t(m) * m), B(size_t(m) * m);
            for (int i = 0; i < m; ++i) {
                double* wi = &W[size_t(i) * m];
                for (int k = 0; k < i; ++k) {
                    const double lik = L[size_t(i) * m + k];
                    const double* wk = &W[size_t(k) * m];
                    for (int c = 0; c < m; ++c) wi[c] -= lik * wk[c];
                }
                const double inv = 1.0 / L[size_t(i) * m + i];
                for (int c = 0; c < m; ++c) wi[c] *= inv;
            }
            for (int i = 0; i < m; ++i)
                for (int c = 0; c < m; ++c) B[size_t(i) * m + c] = W[size_t(c) * m + i];
            for (int i = 0; i < m; ++i) {
                double* bi = &B[size_t(i) * m];
                for (int k = 0; k < i; ++k) {
                    const double lik = L[size_t(i) * m + k];
                    const double* bk = &B[size_t(k) * m];
                    for (int c = 0; c < m; ++c) bi[c] -= lik * bk[c];
                }
                const double inv = 1.0 / L[size_t(i) * m + i];
                for (int c = 0; c < m; ++c) bi[c] *= inv;
            }
            for (int r = 0; r < m; ++r)
                for (int c = 0; c < r; ++c)
                    B[size_t(r) * m + c] = B[size_t(c) * m + r] = 0.5 * (B[size_t(r) * m + c] + B[size_t(c) * m + r]);
            std::vector<double> c0(m);
            if (sym_eig_lowest(m, B.data(), theta, c0.data()) != 0) return -1;
            // a = L^-T c0
            for (int i = m - 1; i >= 0; --i) {
                double v = c0[i];
                for (int k = i + 1; k < m; ++k) v -= L[size_t(k) * m + i] * a[k];
                a[i] = v / L[size_t(i) * m + i];
            }
            *rank = m;
            return m;
        }
    }
    // canonical orthogonalisation through the eigenvectors of N
    std::vector<double> A(N, N + size_t(m) * m), ev(m), U(size_t(m) * m);
    if (sym_eigh(m, A.data(), ev.data(), U.data()) != 0) return -1;
    const double lmax = ev[m - 1];
    if (!(lmax > 1e-12)) return 0;
    std::vector<int> keep;
    for (int i = 0; i < m; ++i)
        if (ev[i] > drop * lmax) keep.push_back(i);
    const int rk = int(keep.size());
    std::vector<double> X(size_t(m) * rk);
    for (int i = 0; i < m; ++i)
        for (int c = 0; c < rk; ++c) X[size_t(i) * rk + c] = U[size_t(i) * m + keep[c]] / std::sqrt(ev[keep[c]]);
    // B = X^T H X
    std::vector<double> HX(size_t(m) * rk, 0.0), B(size_t(rk) * rk, 0.0);
    for (int i = 0; i < m; ++i) {
        double* hx = &HX[size_t(i) * rk];
        for (int j = 0; j < m; ++j) {
            const double hij = H[size_t(i) * m + j];
            const double* xj = &X[size_t(j) * rk];
            for (int c = 0; c < rk; ++c) hx[c] += hij * xj[c];
        }
    }
    for (int i = 0; i < m; ++i) {
        const double* xi = &X[size_t(i) * rk];
        const double* hx = &HX[size_t(i) * rk];
        for (int r = 0; r < rk; ++r) {
            const double xir = xi[r];
            double* br = &B[size_t(r) * rk];
            for (int c = 0; c < rk; ++c) br[c] += xir * hx[c];
        }
    }
    for (int r = 0; r < rk; ++r)
        for (int c = 0; c < r; ++c)
            B[size_t(r) * rk + c] = B[size_t(c) * rk + r] = 0.5 * (B[size_t(r) * rk + c] + B[size_t(c) * rk + r]);
    *rank = rk;
    if (!Xc) {
        std::vector<double> c0(rk);
        if (sym_eig_lowest(rk, B.data(), theta, c0.data()) != 0) return -1;
        for (int i = 0; i < m; ++i) {
            double v = 0.0;
            for (int c = 0; c < rk; ++c) v += X[size_t(i) * rk + c] * c0[c];
            a[i] = v;
        }
        return rk;
    }
    std::vector<double> mu(rk), C(size_t(rk) * rk);
    if (sym_eigh(rk, B.data(), mu.data(), C.data()) != 0) return -1;
    *theta = mu[0];
    for (int i = 0; i < m * rk; ++i) Xc[i] = 0.0;
    for (int i = 0; i < m; ++i) {
        double* xc = Xc + size_t(i) * rk;
        for (int j = 0; j < rk; ++j) {
            const double xij = X[size_t(i) * rk + j];
            const double* cj = &C[size_t(j) * rk];
            for (int c = 0; c < rk; ++c) xc[c] += xij * cj[c];
        }
    }
    for (int i = 0; i < m; ++i) a[i] = Xc[size_t(i) * rk];
    return rk;
}

// ---------------------------------------------------------------------------
// GrowingPencil: every entry below is formed by the expression and in the
// order that cholesky() and the reduction in gen_lowest use for it.

void GrowingPencil::reserve(int m) {
    if (m <= cap_) return;
    const int nc = std::max(m, 2 * cap_);
    for (std::vector<double>* v : {&H_, &N_, &L_, &Ls_, &W_, &B_}) {
        std::vector<double> t(size_t(nc) * nc, 0.0);
        for (int i = 0; i < m_; ++i)
            for (int j = 0; j < m_; ++j) t[size_t(i) * nc + j] = (*v)[size_t(i) * cap_ + j];
        v->swap(t);
    }
    cap_ = nc;
}

// row i of the Cholesky factor of N - shift I (rows < i present)
static bool chol_row(std::vector<double>& L, int ld, const double* N, int nld, int i, double shift) {
    double* li = &L[size_t(i) * ld];
    for (int j = 0; j < i; ++j) {
        const double* lj = &L[size_t(j) * ld];
        double s0 = N[size_t(i) * nld + j], s1 = 0.0;
        int k = 0;
        for (; k + 2 <= j; k += 2) {
            s0 -= li[k] * lj[k];
            s1 -= li[k + 1] * lj[k + 1];
        }
        for (; k < j; ++k) s0 -= li[k] * lj[k];
        li[j] = (s0 + s1) / lj[j];
    }
    double dsum = N[size_t(i) * nld + i] - shift;
    for (int k = 0; k < i; ++k) dsum -= li[k] * li[k];
    if (!(dsum > 0.0)) return false;
    li[i] = std::sqrt(dsum);
    return true;
}

int GrowingPencil::build(int m, const double* H, const double* N, double drop) {
    m_ = 0;
    double U = 0.0;
    for (int i = 0; i < m; ++i) {
        double r = 0.0;
        for (int j = 0; j < m; ++j) r += std::fabs(N[size_t(i) * m + j]);
        U = std::max(U, r);
    }
    if (!(U > 1e-12)) return -2;
    reserve(m);
    shift_ = 2.0 * drop * U;
    for (int i = 0; i < m; ++i)
        if (!chol_row(Ls_, cap_, N, m, i, shift_) || !chol_row(L_, cap_, N, m, i, 0.0)) return -2;
    const int ld = cap_;
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) {
            H_[size_t(i) * ld + j] = H[size_t(i) * m + j];
            N_[size_t(i) * ld + j] = N[size_t(i) * m + j];
        }
    // W = L^-1 H, B = L^-1 W^T (rows by forward substitution)
    for (int i = 0; i < m; ++i) {
        double* wi = &W_[size_t(i) * ld];
        for (int c = 0; c < m; ++c) wi[c] = H[size_t(i) * m + c];
        for (int k = 0; k < i; ++k) {
            const double lik = L_[size_t(i) * ld + k];
            const double* wk = &W_[size_t(k) * ld];
            for (int c = 0; c < m; ++c) wi[c] -= lik * wk[c];
        }
        const double inv = 1.0 / L_[size_t(i) * ld + i];
        for (int c = 0; c < m; ++c) wi[c] *= inv;
    }
    for (int i = 0; i < m; ++i) {
        double* bi = &B_[size_t(i) * ld];
        for (int c = 0; c < m; ++c) bi[c] = W_[size_t(c) * ld + i];
        for (int k = 0; k < i; ++k) {
            const double lik = L_[size_t(i) * ld + k];
            const double* bk = &B_[size_t(k) * ld];
            for (int c = 0; c < m; ++c) bi[c] -= lik * bk[c];
        }
        const double inv = 1.0 / L_[size_t(i) * ld + i];
        for (int c = 0; c < m; ++c) bi[c] *= inv;
    }
    m_ = m;
    return m;
}

// extend the cached factors of the leading (m-1) x (m-1) pencil to m
bool GrowingPencil::grow(int m, const double* H, const double* N, double drop) {
    const int p = m - 1;  // the new row and column
    for (int i = 0; i < p; ++i)
        for (int j = 0; j < p; ++j)
            if (H_[size_t(i) * cap_ + j] != H[size_t(i) * m + j] || N_[size_t(i) * cap_ + j] != N[size_t(i) * m + j])
                return false;
    double U = 0.0;
    for (int i = 0; i < m; ++i) {
        double r = 0.0;
        for (int j = 0; j < m; ++j) r += std::fabs(N[size_t(i) * m + j]);
        U = std::max(U, r);
    }
    if (!(drop * U <= shift_)) return false;
    reserve(m);
    const int ld = cap_;
    if (!chol_row(Ls_, ld, N, m, p, shift_) || !chol_row(L_, ld, N, m, p, 0.0)) return false;
    for (int j = 0; j < m; ++j) {
        H_[size_t(p) * ld + j] = H[size_t(p) * m + j];
        H_[size_t(j) * ld + p] = H[size_t(j) * m + p];
        N_[size_t(p) * ld + j] = N[size_t(p) * m + j];
        N_[size_t(j) * ld + p] = N[size_t(j) * m + p];
    }
    // W: the new column of rows 0..p-1, then the new row
    for (int i = 0; i < p; ++i) {
        double w = H[size_t(i) * m + p];
        for (int k = 0; k < i; ++k) w -= L_[size_t(i) * ld + k] * W_[size_t(k) * ld + p];
        W_[size_t(i) * ld + p] = w * (1.0 / L_[size_t(i) * ld + i]);
    }
    {
        double* wp = &W_[size_t(p) * ld];
        for (int c = 0; c < m; ++c) wp[c] = H[size_t(p) * m + c];
        for (int k = 0; k < p; ++k) {
            const double lpk = L_[size_t(p) * ld + k];
            const double* wk = &W_[size_t(k) * ld];
            for (int c = 0; c < m; ++c) wp[c] -= lpk * wk[c];
        }
        const double inv = 1.0 / L_[size_t(p) * ld + p];
        for (int c = 0; c < m; ++c) wp[c] *= inv;
    }
    // B: the new column of rows 0..p-1 (B[i][p] from W[p][i]), then the new row
    for (int i = 0; i < p; ++i) {
        double b = W_[size_t(p) * ld + i];
        for (int k = 0; k < i; ++k) b -= L_[size_t(i) * ld + k] * B_[size_t(k) * ld + p];
        B_[size_t(i) * ld + p] = b * (1.0 / L_[size_t(i) * ld + i]);
    }
    {
        double* bp = &B_[size_t(p) * ld];
        for (int c = 0; c < m; ++c) bp[c] = W_[size_t(c) * ld + p];
        for (int k = 0; k < p; ++k) {
            const double lpk = L_[size_t(p) * ld + k];
            const double* bk = &B_[size_t(k) * ld];
            for (int c = 0; c < m; ++c) bp[c] -= lpk * bk[c];
        }
        const double inv = 1.0 / L_[size_t(p) * ld + p];
        for (int c = 0; c < m; ++c) bp[c] *= inv;
    }
    m_ = m;
    return true;
}

int GrowingPencil::lowest(int m, const double* H, const double* N, double drop, double* theta, double* a) {
    if (m <= 0) return -2;
    const bool grown = (m_ > 0 && m == m_ + 1 && grow(m, H, N, drop));
    if (!grown && build(m, H, N, drop) != m) {
        m_ = 0;
        return -2;
    }
    const int ld = cap_;
    std::vector<double> Bs(size_t(m) * m);
    for (int r = 0; r < m; ++r)
        for (int c = 0; c < m; ++c) Bs[size_t(r) * m + c] = B_[size_t(r) * ld + c];
    for (int r = 0; r < m; ++r)
        for (int c = 0; c < r; ++c)
            Bs[size_t(r) * m + c] = Bs[size_t(c) * m + r] = 0.5 * (Bs[size_t(r) * m + c] + Bs[size_t(c) * m + r]);
    std::vector<double> c0(m);
    if (sym_eig_lowest(m, Bs.data(), theta, c0.data()) != 0) {
        m_ = 0;
        return -1;
    }
    for (int i = m - 1; i >= 0; --i) {
        double v = c0[i];
        for (int k = i + 1; k < m; ++k) v -= L_[size_t(k) * ld + i] * a[k];
        a[i] = v / L_[size_t(i) * ld + i];
    }
    return m;
}

}  // namespace sph
