// Host-side numerics of the SP-MPS library: projector quadrature, MPO
// construction and the small symmetric eigensolver of the Davidson subspace.
#include "host_linalg.h"

#include <algorithm>
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

int mpo_identity(int L, int* w, double* data, long long* n) {
    MpoBuilder mb{L, 1, std::vector<M4>(1, eye4())};
    return emit(mb, w, data, n);
}

// ---------------------------------------------------------------------------
// Symmetric eigensolver: Householder reduction to tridiagonal form with the
// transformations accumulated, then implicit symmetric QR steps with
// Wilkinson shifts (Givens bulge chase), deflating at negligible
// off-diagonals.  Eigenvalues ascending; eigenvectors are columns of vec.

int sym_eigh(int n, double* a, double* ev, double* vec) {
    if (n <= 0) return 0;
    std::vector<double> Q(size_t(n) * n, 0.0);
    for (int i = 0; i < n; ++i) Q[size_t(i) * n + i] = 1.0;
    std::vector<double> v(n), p(n), wv(n);
    auto A = [&](int i, int j) -> double& { return a[size_t(i) * n + j]; };
    for (int k = 0; k + 2 < n; ++k) {
        const int len = n - k - 1;
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
        // trailing block S = A[k+1:, k+1:]:  S -= v w^T + w v^T
        double vp = 0.0;
        for (int i = 0; i < len; ++i) {
            double s = 0.0;
            for (int j = 0; j < len; ++j) s += A(k + 1 + i, k + 1 + j) * v[j];
            p[i] = beta * s;
            vp += v[i] * p[i];
        }
        const double K = 0.5 * beta * vp;
        for (int i = 0; i < len; ++i) wv[i] = p[i] - K * v[i];
        for (int i = 0; i < len; ++i)
            for (int j = 0; j < len; ++j) A(k + 1 + i, k + 1 + j) -= v[i] * wv[j] + wv[i] * v[j];
        A(k + 1, k) = A(k, k + 1) = alpha;
        for (int i = 1; i < len; ++i) A(k + 1 + i, k) = A(k, k + 1 + i) = 0.0;
        // Q <- Q H
        for (int r = 0; r < n; ++r) {
            double s = 0.0;
            for (int j = 0; j < len; ++j) s += Q[size_t(r) * n + k + 1 + j] * v[j];
            s *= beta;
            for (int j = 0; j < len; ++j) Q[size_t(r) * n + k + 1 + j] -= s * v[j];
        }
    }
    std::vector<double> d(n), e(n, 0.0);
    for (int i = 0; i < n; ++i) d[i] = A(i, i);
    for (int i = 0; i + 1 < n; ++i) e[i] = A(i + 1, i);

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
        if (++guard > 60 * n) return -1;
        // Wilkinson shift from the trailing 2x2 of the block [l, m]
        const double delta = 0.5 * (d[m - 1] - d[m]);
        const double b2 = e[m - 1] * e[m - 1];
        const double sg = (delta >= 0.0) ? 1.0 : -1.0;
        const double mu = d[m] - b2 / (delta + sg * std::sqrt(delta * delta + b2));
        double x = d[l] - mu;
        double z = e[l];
        for (int k = l; k < m; ++k) {
            double r = std::hypot(x, z);
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
                z = s * e[k + 1];      // bulge at (k, k+2)
                e[k + 1] = c * e[k + 1];
                x = e[k];
            }
            for (int r0 = 0; r0 < n; ++r0) {
                double* row = &Q[size_t(r0) * n];
                const double qk = row[k], qk1 = row[k + 1];
                row[k] = c * qk + s * qk1;
                row[k + 1] = -s * qk + c * qk1;
            }
        }
    }
    std::vector<int> idx(n);
    std::iota(idx.begin(), idx.end(), 0);
    std::sort(idx.begin(), idx.end(), [&](int i, int j) { return d[i] < d[j]; });
    for (int i = 0; i < n; ++i) {
        ev[i] = d[idx[i]];
        for (int r = 0; r < n; ++r) vec[size_t(r) * n + i] = Q[size_t(r) * n + idx[i]];
    }
    return 0;
}

}  // namespace sph
