"""Pins of the ab-initio Hamiltonian (Eq. [sqH]) in the oracle: the MPO
against exact diagonalisation built from bit strings, closed forms of small
sectors, spin symmetry, and the sweep at full bond dimension against the
projected exact ground state."""
import numpy as np
import pytest

import workloads as W
from oracle import ed, mpo, mps, quadrature as q


def _sectors(K):
    for N in range(1, 2 * K):
        for twoM in range(-N, N + 1, 2):
            st = ed.sector_states(K, N, twoM)
            if len(st):
                yield N, twoM, st


@pytest.mark.parametrize("K", [2, 3, 4])
def test_mpo_equals_bitstring_hamiltonian(K):
    h, eri = W.abinitio_integrals(K, seed=4)
    Hd = mpo.mpo_to_dense(mpo.abinitio_mpo(h, eri))
    for N, twoM, st in _sectors(K):
        A = ed.abinitio_hamiltonian(h, eri, st).toarray()
        np.testing.assert_allclose(Hd[np.ix_(st, st)], A, atol=1e-12, err_msg=f"N={N} 2M={twoM}")
    # nothing couples different (N, M) sectors
    full = np.zeros(4 ** K, dtype=int)
    for i, (N, twoM, st) in enumerate(_sectors(K)):
        full[st] = i + 1
    nz = np.abs(Hd) > 1e-14
    r, c = np.nonzero(nz)
    assert np.all(full[r] == full[c])


def test_integral_symmetries():
    h, eri = W.abinitio_integrals(6, seed=4)
    assert np.array_equal(h, h.T)
    for perm in [(1, 0, 2, 3), (0, 1, 3, 2), (2, 3, 0, 1)]:
        np.testing.assert_allclose(eri, eri.transpose(perm), atol=1e-15)
    ev = np.linalg.eigvalsh(eri.reshape(36, 36))
    assert ev.min() > -1e-12  # positive semidefinite as a (pq),(rs) matrix


def test_one_electron_and_one_hole_sectors():
    # N = 1: H is h itself.  N = 2K - 1 (one hole, spin 1/2): the energy of
    # the closed shell minus the orbital energies of the Fock operator
    # F_pq = h_pq + sum_r [2 (pq|rr) - (pr|rq)], i.e. E_full - eig(F)
    K = 3
    h, eri = W.abinitio_integrals(K, seed=7)
    st = ed.sector_states(K, 1, 1)
    H1 = ed.abinitio_hamiltonian(h, eri, st).toarray()
    np.testing.assert_allclose(np.sort(np.linalg.eigvalsh(H1)), np.sort(np.linalg.eigvalsh(h)), atol=1e-12)
    e_full = 2 * np.trace(h) + sum(2 * eri[p, p, r, r] - eri[p, r, r, p] for p in range(K) for r in range(K))
    F = h + 2 * np.einsum("pqrr->pq", eri) - np.einsum("prrq->pq", eri)
    st = ed.sector_states(K, 2 * K - 1, 1)
    Hh = ed.abinitio_hamiltonian(h, eri, st).toarray()
    np.testing.assert_allclose(np.sort(np.linalg.eigvalsh(Hh)), np.sort(e_full - np.linalg.eigvalsh(F)), atol=1e-11)
    # the full shell is one state
    st = ed.sector_states(K, 2 * K, 0)
    assert abs(ed.abinitio_hamiltonian(h, eri, st).toarray()[0, 0] - e_full) < 1e-12


def test_two_orbital_triplet_closed_form():
    # two orbitals, both alpha electrons: E = h11 + h22 + (11|22) - (12|21)
    h, eri = W.abinitio_integrals(2, seed=9)
    st = ed.sector_states(2, 2, 2)
    e = h[0, 0] + h[1, 1] + eri[0, 0, 1, 1] - eri[0, 1, 1, 0]
    Hd = mpo.mpo_to_dense(mpo.abinitio_mpo(h, eri))
    assert len(st) == 1
    assert abs(ed.abinitio_hamiltonian(h, eri, st).toarray()[0, 0] - e) < 1e-13
    assert abs(Hd[st[0], st[0]] - e) < 1e-13


def test_hamiltonian_is_spin_free():
    K = 4
    h, eri = W.abinitio_integrals(K, seed=4)
    for (N, twoM) in [(4, 0), (3, 1)]:
        st = ed.sector_states(K, N, twoM)
        H = ed.abinitio_hamiltonian(h, eri, st).toarray()
        S2 = ed.s2_operator(K, st).toarray()
        assert np.abs(H @ S2 - S2 @ H).max() < 1e-11
        assert np.abs(H - H.T).max() < 1e-12


def _ed_ground(K, N, twoM, twoS, h, eri):
    st = ed.sector_states(K, N, twoM)
    H = ed.abinitio_hamiltonian(h, eri, st)
    S2 = ed.s2_operator(K, st)
    return ed.projected_ground_energy(H, ed.lowdin_projector(S2, twoS, twoM, N))


@pytest.mark.parametrize("twoS", [0, 2])
def test_oracle_sweep_reaches_projected_ground_state(twoS):
    # full bond dimension: the one-site sweep can represent the exact state
    K, N = 4, 4
    h, eri = W.abinitio_integrals(K, seed=4)
    tab = W.make_block_table(K, N, 0, 64)
    G = q.exact_point_count(N, K, twoS, 0)
    o = mps.SPMPSOracle(tab, W.random_blocks(tab, 5), mpo.abinitio_mpo(h, eri), twoS, G)
    steps = mps.sweep(o, 3)
    e_ed = _ed_ground(K, N, 0, twoS, h, eri)
    assert abs(steps[-1]["theta"] - e_ed) < 1e-9
    E, p = o.full_contraction()
    assert abs(E - e_ed) < 1e-9 and p > 1e-3
