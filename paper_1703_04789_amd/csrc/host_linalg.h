// Host-side numerics of the SP-MPS library.
#pragma once
#include <array>
#include <vector>

namespace sph {

void gauss_legendre(int G, double* x, double* w);
double wigner_d_diag(int twoJ, int twoM, double x);
int max_seniority(int N, int twoM, int K);
int exact_points(int N, int K, int twoS, int twoM);
// x, w: nodes/weights; c = cos(beta/2), s = sin(beta/2); coef_g
void projector_quadrature(int G, int twoS, int twoM, double* x, double* w, double* c, double* s,
                          double* coef);
int mpo_hubbard(int L, double t, double U, int* w, double* data, long long* n);
int mpo_s2(int L, int* w, double* data, long long* n);
int mpo_identity(int L, int* w, double* data, long long* n);
// single-site operator op (4x4 row-major) at site p
int mpo_site_op(int L, int p, const double* op, int* w, double* data, long long* n);
// E_pq = sum_sigma a+_{p sigma} a_{q sigma} (p == q: the occupation n_p)
int mpo_epq(int L, int p, int q, int* w, double* data, long long* n);
// S_X . S_Y (X == Y: S_X^2)
int mpo_spin_corr(int L, int X, int Y, int* w, double* data, long long* n);
// ab-initio Hamiltonian of K orbitals from h (K x K) and (pq|rs) (K^4,
// index ((p*K + q)*K + r)*K + s); data == nullptr: sizes only.  only_p >= 0
// (0-based orbital): only the energy component H_p (the terms whose first
// creator acts on orbital p)
int mpo_abinitio(int K, const double* h, const double* eri, int* w, double* data, long long* n, int only_p = -1);
int sym_eigh(int n, double* a, double* ev, double* vec);
// lowest eigenvalue and its unit eigenvector (tridiagonal QR for the value,
// inverse iteration for the vector); a is destroyed
int sym_eig_lowest(int n, double* a, double* ev0, double* v0);
// Lowest eigenpair of the symmetric pencil (H, N), m x m row-major, within
// the span of the eigenvectors of N whose eigenvalues exceed drop * max
// (canonical orthogonalisation).  a: m coefficients with a^T N a = 1.  If
// Xc != nullptr it receives all Ritz coefficient vectors (m x rank,
// ascending Ritz values).  Returns the rank (> 0), 0 if N vanishes, -1 on
// failure.
int gen_lowest(int m, const double* H, const double* N, double drop, double* theta, double* a, double* Xc,
               int* rank);

// The fast path of gen_lowest (nothing dropped, Cholesky reduction) for a
// pencil that grows by one row and column per call, as the projected
// matrices of a Davidson solve do between restarts.  It keeps the Cholesky
// factor L of N, W = L^-1 H and B = L^-1 W^T and extends them by one row and
// column per call, each new entry formed by the same operations as in a
// full factorisation, so the result is the one gen_lowest gives.  The
// certificate that nothing would be dropped is a Cholesky factor of
// N - s I, s = 2 drop U (U the Gershgorin bound when the factors were
// built), extended alike and valid while drop U stays below s.  lowest()
// returns m, or -2 if the fast path does not apply (no certificate, or a
// pencil that is not the cached one grown by one): the caller then takes
// gen_lowest.
class GrowingPencil {
public:
    void reset() { m_ = 0; }
    int lowest(int m, const double* H, const double* N, double drop, double* theta, double* a);

private:
    int m_ = 0, cap_ = 0;
    double shift_ = 0.0;
    std::vector<double> H_, N_, L_, Ls_, W_, B_;  // cap_ x cap_, row-major
    void reserve(int m);
    int build(int m, const double* H, const double* N, double drop);
    bool grow(int m, const double* H, const double* N, double drop);
};

}  // namespace sph
