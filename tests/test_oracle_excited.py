"""Pins of the oracle's excited-state machinery (Sec. 2.3, Eq. [orthoB]):
the constraint vector B[k] against its brute-force definition, the
constrained Davidson against dense linear algebra, and state-specific
excited-state sweeps at full bond dimension against exact diagonalisation."""
import numpy as np
import pytest

import workloads as W
from oracle import ed, mpo, mps, quadrature as q


def _packed(o):
    return np.concatenate([o.mps.site_packed(k) for k in range(1, o.L + 1)])


def _spin_levels(L, N, twoM, twoS, U, t=1.0, n=3):
    """Lowest n eigenvalues of H within total spin S (exact diagonalisation)."""
    st = ed.sector_states(L, N, twoM)
    H = ed.hubbard_hamiltonian(L, t, U, st).toarray()
    ev, vec = np.linalg.eigh(ed.s2_operator(L, st).toarray())
    s = twoS / 2
    Z = vec[:, np.abs(ev - s * (s + 1)) < 1e-8]
    return np.linalg.eigvalsh(Z.T @ H @ Z)[:n]


@pytest.mark.parametrize("twoS", [0, 2])
def test_constraint_vector_equals_brute_force(twoS):
    # B[k] = d<Psi_0|P|Psi>/dA[k] = Phi_k^T P psi_0 with Phi_k the dense map
    # from site tensor k to the state
    L, N, twoM, D = 4, 4, 0, 8
    tab = W.make_block_table(L, N, twoM, D)
    G = q.exact_point_count(N, L, twoS, twoM)
    o = mps.SPMPSOracle(tab, W.random_blocks(tab, 21), mpo.hubbard_mpo(L, 1.0, 4.0), twoS, G)
    c = mps.OrthogonalityConstraint(o, tab, W.random_blocks(tab, 22))
    st = ed.sector_states(L, N, twoM)
    P = ed.spin_projector_dense(ed.s2_operator(L, st), twoS)
    psi0 = ed.mps_to_dense(c.psi0.A)[st]
    for k in range(1, L + 1):
        if k > 1:
            c.update_left(k - 1)
        n = o.mps.site_packed(k).size
        B = o.mps.site_packed(k, c.vector(k))
        saved = o.mps.A[k - 1]
        Phi = np.zeros((len(st), n))
        for i in range(n):
            e = np.zeros(n)
            e[i] = 1.0
            o.mps.A[k - 1] = o.mps.dense_site(k, e)
            Phi[:, i] = ed.mps_to_dense(o.mps.A)[st]
        o.mps.A[k - 1] = saved
        ref = Phi.T @ (P @ psi0)
        assert np.abs(B - ref).max() < 1e-12 * max(1.0, np.abs(ref).max()), k
        # the overlap through site k is the full one
        psi = ed.mps_to_dense(o.mps.A)[st]
        assert abs(c.overlap(k) - psi0 @ P @ psi) < 1e-12


def test_constrained_davidson_matches_dense_pencil():
    rng = np.random.default_rng(3)
    n, nc = 40, 3
    A = rng.standard_normal((n, n))
    H = A + A.T
    Bm = rng.standard_normal((n, n))
    Nm = Bm @ Bm.T / n + np.eye(n)
    C = mps.orthonormal_constraints(list(rng.standard_normal((nc, n))))
    res = mps.davidson(lambda v: (H @ v, Nm @ v), np.diag(H), np.diag(Nm), rng.standard_normal(n),
                       tol=1e-11, max_iter=200, max_sub=60, C=C)
    # dense reference: the pencil on an orthonormal basis of the complement
    U, _, _ = np.linalg.svd(np.eye(n) - C @ C.T)
    Z = U[:, : n - nc]
    Lc = np.linalg.cholesky(Z.T @ Nm @ Z)
    Li = np.linalg.inv(Lc)
    ref = np.linalg.eigvalsh(Li @ (Z.T @ H @ Z) @ Li.T)[0]
    assert res.converged
    assert abs(res.theta - ref) < 1e-10
    assert np.abs(C.T @ res.x).max() < 1e-12


def test_orthonormal_constraints_drops_dependent_vectors():
    rng = np.random.default_rng(0)
    a, b = rng.standard_normal(10), rng.standard_normal(10)
    C = mps.orthonormal_constraints([a, b, 2 * a - 3 * b])
    assert C.shape == (10, 2)
    assert np.abs(C.T @ C - np.eye(2)).max() < 1e-14


def _ground(L, U, twoS, seed=1):
    N = L
    tab = W.make_block_table(L, N, 0, 4 ** (L // 2))
    G = q.exact_point_count(N, L, twoS, 0)
    o = mps.SPMPSOracle(tab, W.random_blocks(tab, seed), mpo.hubbard_mpo(L, 1.0, U), twoS, G)
    mps.sweep(o, 3, max_sub=128, max_iter=200)
    return tab, G, o


@pytest.mark.parametrize("twoS", [0, 2])
def test_first_excited_state_at_full_bond_dimension(twoS):
    L, U = 4, 4.0
    ref = _spin_levels(L, L, 0, twoS, U)
    tab, G, o0 = _ground(L, U, twoS)
    assert abs(mps.sweep(o0, 1, max_sub=128, max_iter=200)[-1]["theta"] - ref[0]) < 1e-9
    o1 = mps.SPMPSOracle(tab, W.random_blocks(tab, 5), mpo.hubbard_mpo(L, 1.0, U), twoS, G)
    c = mps.OrthogonalityConstraint(o1, tab, _packed(o0))
    steps = mps.sweep(o1, 4, max_sub=128, max_iter=200, constraints=[c])
    assert abs(steps[-1]["theta"] - ref[1]) < 1e-9, (steps[-1]["theta"], ref)
    assert abs(c.overlap(1)) < 1e-10


def test_second_excited_state_with_two_constraints():
    L, U, twoS = 4, 4.0, 0
    ref = _spin_levels(L, L, 0, twoS, U)
    tab, G, o0 = _ground(L, U, twoS)
    o1 = mps.SPMPSOracle(tab, W.random_blocks(tab, 5), mpo.hubbard_mpo(L, 1.0, U), twoS, G)
    mps.sweep(o1, 4, max_sub=128, max_iter=200, constraints=[mps.OrthogonalityConstraint(o1, tab, _packed(o0))])
    o2 = mps.SPMPSOracle(tab, W.random_blocks(tab, 6), mpo.hubbard_mpo(L, 1.0, U), twoS, G)
    cs = [mps.OrthogonalityConstraint(o2, tab, _packed(o0)), mps.OrthogonalityConstraint(o2, tab, _packed(o1))]
    steps = mps.sweep(o2, 4, max_sub=128, max_iter=200, constraints=cs)
    assert abs(steps[-1]["theta"] - ref[2]) < 1e-9, (steps[-1]["theta"], ref)
    assert all(abs(c.overlap(1)) < 1e-10 for c in cs)
