// Checks sph::GrowingPencil against sph::gen_lowest: on pencils that grow by
// one row and column per call the two give the same bits (theta and a); a
// pencil with a metric direction below the drop threshold, one that is not
// the cached one grown by one, and the restart of a solve are all handed back
// (-2) or rebuilt, never answered from a stale reduction.  Prints "ok" or the
// first mismatch.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

#include "host_linalg.h"

namespace {

std::mt19937_64 rng(20240611);
std::normal_distribution<double> nd;

// H symmetric, N = Y Y^T / M + eps I, one row of Y scaled by weak (if > 0)
void pencil(int M, std::vector<double>& H, std::vector<double>& N, double weak, double eps) {
    std::vector<double> A(size_t(M) * M), Y(size_t(M) * M);
    for (auto& v : A) v = nd(rng);
    for (auto& v : Y) v = nd(rng);
    if (weak > 0.0)
        for (int j = 0; j < M; ++j) Y[size_t(M / 2) * M + j] *= weak;
    H.assign(size_t(M) * M, 0.0);
    N.assign(size_t(M) * M, 0.0);
    for (int i = 0; i < M; ++i)
        for (int j = 0; j < M; ++j) {
            H[size_t(i) * M + j] = A[size_t(i) * M + j] + A[size_t(j) * M + i];
            double s = 0.0;
            for (int k = 0; k < M; ++k) s += Y[size_t(i) * M + k] * Y[size_t(j) * M + k];
            N[size_t(i) * M + j] = s / M + (i == j ? eps : 0.0);
        }
}

void lead(const std::vector<double>& X, int M, int m, std::vector<double>& out) {
    out.resize(size_t(m) * m);
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) out[size_t(i) * m + j] = X[size_t(i) * M + j];
}

int fails = 0;

void compare(const char* what, int m, const std::vector<double>& h, const std::vector<double>& n,
             sph::GrowingPencil& gp, int& fast) {
    double t0 = 0.0, t1 = 0.0;
    std::vector<double> a0(m), a1(m);
    int rk = 0;
    const int r0 = sph::gen_lowest(m, h.data(), n.data(), 1e-10, &t0, a0.data(), nullptr, &rk);
    const int r1 = gp.lowest(m, h.data(), n.data(), 1e-10, &t1, a1.data());
    if (r1 == -2) return;  // handed back: the caller takes gen_lowest
    ++fast;
    if (r1 != m || r0 != m || std::memcmp(&t0, &t1, sizeof t0) != 0 ||
        std::memcmp(a0.data(), a1.data(), sizeof(double) * m) != 0) {
        if (fails++ < 5) std::printf("%s m=%d: r %d/%d theta %.17g vs %.17g\n", what, m, r0, r1, t0, t1);
    }
}

}  // namespace

int main() {
    const int M = 40;
    std::vector<double> H, N, h, n;
    int fast = 0, handed = 0;
    for (int trial = 0; trial < 6; ++trial) {
        pencil(M, H, N, 0.0, 0.05);
        sph::GrowingPencil gp;
        for (int m = 1; m <= M; ++m) {  // one solve, growing one by one
            lead(H, M, m, h);
            lead(N, M, m, n);
            compare("grow", m, h, n, gp, fast);
        }
        // a restart: the next pencil is not the cached one grown by one
        for (int m = 8; m <= 20; ++m) {
            lead(H, M, m, h);
            lead(N, M, m, n);
            for (auto& v : h) v *= 0.5;
            compare("restart", m, h, n, gp, fast);
        }
        // same size again after a changed leading block
        lead(H, M, 12, h);
        lead(N, M, 12, n);
        h[1] += 1e-3;
        h[12] += 1e-3;
        compare("changed", 12, h, n, gp, fast);
    }
    // a weak metric direction: the certificate must not hold where
    // canonical orthogonalisation would drop it
    pencil(M, H, N, 1e-7, 0.0);
    sph::GrowingPencil gp;
    for (int m = 1; m <= M; ++m) {
        lead(H, M, m, h);
        lead(N, M, m, n);
        double t1 = 0.0;
        std::vector<double> a1(m);
        const int r1 = gp.lowest(m, h.data(), n.data(), 1e-10, &t1, a1.data());
        if (r1 == -2) {
            ++handed;
            continue;
        }
        double t0 = 0.0;
        std::vector<double> a0(m);
        int rk = 0;
        sph::gen_lowest(m, h.data(), n.data(), 1e-10, &t0, a0.data(), nullptr, &rk);
        if (rk != m || std::memcmp(&t0, &t1, sizeof t0) != 0) {
            if (fails++ < 5) std::printf("weak m=%d: rank %d theta %.17g vs %.17g\n", m, rk, t0, t1);
        }
    }
    if (fails == 0 && fast > 200 && handed > 0) {
        std::printf("ok %d fast, %d handed back\n", fast, handed);
        return 0;
    }
    std::printf("FAILED: %d mismatches, %d fast, %d handed back\n", fails, fast, handed);
    return 1;
}
