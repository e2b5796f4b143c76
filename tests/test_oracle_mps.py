"""Pins of the oracle's SP-MPS machinery (Secs. 2.2, 2.3) against the plain
dense definition (exact diagonalisation with the exact projector), invariants
and closed forms."""
import json
import os

import numpy as np
import pytest
import scipy.linalg as sla

import workloads as W
from oracle import ed, mpo, mps, quadrature as q

ED = {(c["L"], c["N"], c["twoM"], c["U"], c["twoS"]): c["E"]
      for c in json.load(open(os.path.join(os.path.dirname(__file__), "golden", "ed_energies.json")))["cases"]}


def _state(L, N, twoM, D, twoS, seed, U=3.0, G=None, W_=None):
    tab = W.make_block_table(L, N, twoM, D)
    G = G or q.exact_point_count(N, L, twoS, twoM)
    Wm = W_ if W_ is not None else mpo.hubbard_mpo(L, 1.0, U)
    return tab, mps.SPMPSOracle(tab, W.random_blocks(tab, seed), Wm, twoS, G)


@pytest.mark.parametrize("L,N,twoM,twoS", [(4, 4, 0, 0), (4, 4, 0, 2), (5, 5, 1, 1), (5, 5, 1, 3),
                                          (5, 4, 0, 2), (6, 6, 0, 0)])
def test_energy_functional_equals_dense_definition(L, N, twoM, twoS):
    tab, o = _state(L, N, twoM, 12, twoS, seed=11)
    st = ed.sector_states(L, N, twoM)
    He = ed.hubbard_hamiltonian(L, 1.0, 3.0, st)
    Pd = ed.spin_projector_dense(ed.s2_operator(L, st), twoS)
    psi = ed.mps_to_dense(o.mps.A)[st]
    Eref, pref = ed.projected_energy(psi, He, Pd)
    E1, p1 = o.full_contraction()
    E2, p2 = o.energy(1)
    assert abs(E1 - Eref) < 1e-12 and abs(E2 - Eref) < 1e-12
    assert abs(p1 - pref) < 1e-12 * max(1, abs(pref))
    # more quadrature points than needed change nothing
    o2 = mps.SPMPSOracle(tab, W.random_blocks(tab, 11), mpo.hubbard_mpo(L, 1.0, 3.0), twoS, o.G + 2)
    assert abs(o2.full_contraction()[0] - Eref) < 1e-12


@pytest.mark.parametrize("twoS", [0, 2, 4])
def test_s2_mpo_through_projected_functional(twoS):
    L = 5
    tab, o = _state(L, 4, 0, 10, twoS, seed=5, W_=mpo.s2_mpo(L))
    E, p = o.full_contraction()
    s = twoS / 2
    assert p > 1e-8
    assert abs(E - s * (s + 1)) < 1e-12


def test_mps_is_right_canonical_and_state_unchanged():
    L = 5
    tab = W.make_block_table(L, 5, 1, 10)
    blocks = W.random_blocks(tab, 3)
    raw = mps.OracleMPS(tab, blocks)
    psi0 = ed.mps_to_dense(raw.A)
    tab, o = _state(L, 5, 1, 10, 1, seed=3)
    for k in range(2, L + 1):
        A = o.mps.A[k - 1]
        np.testing.assert_allclose(np.einsum("sab,scb->ac", A, A), np.eye(A.shape[1]), atol=1e-13)
    np.testing.assert_allclose(ed.mps_to_dense(o.mps.A), psi0, atol=1e-12)
    # moving the centre right with QR keeps the state
    for k in range(1, L):
        o.mps.left_orthonormalize(k)
        A = o.mps.A[k - 1]
        np.testing.assert_allclose(np.einsum("sab,sac->bc", A, A), np.eye(A.shape[2]), atol=1e-13)
    np.testing.assert_allclose(ed.mps_to_dense(o.mps.A), psi0, atol=1e-12)


def test_qr_positive_diagonal_is_unique():
    rng = np.random.default_rng(0)
    M = rng.standard_normal((9, 4))
    Q1, R1 = mps.OracleMPS._qr_pos(M)
    perm = rng.permutation(9)
    Q2, R2 = mps.OracleMPS._qr_pos(M[perm])
    np.testing.assert_allclose(R1, R2, atol=1e-14)
    np.testing.assert_allclose(Q1[perm], Q2, atol=1e-14)
    assert np.all(np.diag(R1) > 0)
    # Gram-Schmidt by hand gives the same factor
    Q = np.zeros_like(M)
    for j in range(4):
        v = M[:, j] - Q[:, :j] @ (Q[:, :j].T @ M[:, j])
        Q[:, j] = v / np.linalg.norm(v)
    np.testing.assert_allclose(Q, Q1, atol=1e-13)


def _dense_heff(o, k):
    m = o.mps.mask[k - 1]
    idx = np.flatnonzero(m.ravel())
    n = len(idx)
    H = np.zeros((n, n))
    N = np.zeros((n, n))
    for i in range(n):
        e = np.zeros(m.size)
        e[idx[i]] = 1.0
        y, ny = o.heff(k, e.reshape(m.shape))
        H[:, i] = y.ravel()[idx]
        N[:, i] = ny.ravel()[idx]
    return H, N, idx


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_heff_equals_brute_force_projection(k):
    L, N, twoM, twoS = 4, 4, 0, 2
    tab, o = _state(L, N, twoM, 16, twoS, seed=9)
    for j in range(1, k):            # bring the centre to site k
        o.mps.left_orthonormalize(j)
        o.update_left(j)
    H, Nm, idx = _dense_heff(o, k)
    # brute force: Phi maps the site tensor to the sector vector
    st = ed.sector_states(L, N, twoM)
    Hs = ed.hubbard_hamiltonian(L, 1.0, 3.0, st).toarray()
    P = ed.spin_projector_dense(ed.s2_operator(L, st), twoS)
    shape = o.mps.A[k - 1].shape
    Phi = np.zeros((len(st), len(idx)))
    saved = o.mps.A[k - 1].copy()
    for i in range(len(idx)):
        e = np.zeros(saved.size)
        e[idx[i]] = 1.0
        o.mps.A[k - 1] = e.reshape(shape)
        Phi[:, i] = ed.mps_to_dense(o.mps.A)[st]
    o.mps.A[k - 1] = saved
    np.testing.assert_allclose(H, Phi.T @ Hs @ P @ Phi, atol=1e-12)
    np.testing.assert_allclose(Nm, Phi.T @ P @ Phi, atol=1e-12)
    assert np.abs(H - H.T).max() < 1e-12
    assert np.linalg.eigvalsh(Nm).min() > -1e-12
    dh, dn = o.heff_diag(k)
    np.testing.assert_allclose(dh.ravel()[idx], np.diag(H), atol=1e-13)
    np.testing.assert_allclose(dn.ravel()[idx], np.diag(Nm), atol=1e-13)


def test_heff_symmetric_for_inexact_quadrature():
    # P_M R(beta) P_M is symmetric for any beta, so H_eff, N_eff are symmetric
    # even below the exact point count
    tab, o = _state(5, 5, 1, 10, 1, seed=2, G=2)
    H, Nm, _ = _dense_heff(o, 1)
    assert np.abs(H - H.T).max() < 1e-12 and np.abs(Nm - Nm.T).max() < 1e-12


def test_davidson_matches_dense_pencil():
    rng = np.random.default_rng(4)
    n = 40
    B = rng.standard_normal((n, 25))
    Nm = B @ B.T / 25            # PSD, rank 25
    A = rng.standard_normal((25, 25))
    Hm = B @ (A + A.T) @ B.T / 50  # vanishes on null(N)
    lam, U = np.linalg.eigh(Nm)
    sel = lam > 1e-10 * lam.max()
    X = U[:, sel] / np.sqrt(lam[sel])
    ref = np.linalg.eigvalsh(X.T @ Hm @ X)[0]
    res = mps.davidson(lambda v: (Hm @ v, Nm @ v), np.diag(Hm), np.diag(Nm), rng.standard_normal(n),
                       max_sub=48, max_iter=100)
    assert res.converged and abs(res.theta - ref) < 1e-10
    # restarts (subspace 16, keep 8) reach the same eigenvalue
    res = mps.davidson(lambda v: (Hm @ v, Nm @ v), np.diag(Hm), np.diag(Nm), rng.standard_normal(n),
                       max_sub=16, keep=8, max_iter=400)
    assert abs(res.theta - ref) < 1e-9


def test_sweep_two_sites_closed_form():
    for twoS, ref in ((0, (4.0 - np.sqrt(32.0)) / 2), (2, 0.0)):
        tab, o = _state(2, 2, 0, 4, twoS, seed=1, U=4.0)
        st = mps.sweep(o, 2)
        assert abs(st[-1]["theta"] - ref) < 1e-11


@pytest.mark.parametrize("L,twoS", [(4, 0), (4, 2), (6, 0), (6, 2)])
def test_sweep_full_bond_dimension_reaches_ed(L, twoS):
    tab, o = _state(L, L, 0, 4 ** (L // 2), twoS, seed=1, U=4.0)
    st = mps.sweep(o, 3, max_sub=128, max_iter=200)
    assert abs(st[-1]["theta"] - ED[(L, L, 0, 4.0, twoS)]) < 1e-10


def test_sweep_free_chain_full_bond_dimension():
    L = 6
    eps = np.sort(-2.0 * np.cos(np.pi * np.arange(1, L + 1) / (L + 1)))
    tab, o = _state(L, L, 0, 64, 0, seed=2, U=0.0)
    st = mps.sweep(o, 3, max_sub=128, max_iter=200)
    assert abs(st[-1]["theta"] - 2 * eps[:3].sum()) < 1e-10


@pytest.mark.slow
def test_sweep_small_workload_variational():
    wl = W.hubbard_small()
    tab = wl.table()
    o = mps.SPMPSOracle(tab, wl.blocks(), mpo.hubbard_mpo(wl.L, wl.t, wl.U), wl.twoS, wl.G)
    st = mps.sweep(o, wl.sweeps, max_sub=128, max_iter=200)
    e_ed = ED[(8, 8, 0, 4.0, 0)]
    E = np.array([s["theta"] for s in st])
    assert np.all(E > e_ed - 1e-10)
    assert E[-1] - e_ed < 2e-3
    # one-site sweeps with exact local solves never raise the energy
    assert np.all(np.diff(E) < 1e-10)
