"""Pins of the closed-form determinant energies (oracle.slater) against exact
diagonalisation of the ab-initio Hamiltonian of Eq. [sqH] built from bit
strings, with the exact S^2 projector of Sec. 2.2 for the open-shell case."""
import numpy as np
import pytest

import workloads as W
from oracle import ed, slater


def _index(K, occ):
    """ED basis index of the determinant with spin orbitals occ (0-based p)."""
    i = 0
    for (p, s) in occ:
        k = p + 1
        i += (2 if s == 0 else 1) * 4 ** (K - k)
    return i


def _sector(K, occ):
    na = sum(1 for _, s in occ if s == 0)
    nb = len(occ) - na
    st = ed.sector_states(K, na + nb, na - nb)
    return st, {int(v): n for n, v in enumerate(st)}


def _vec(K, st, pos, occ):
    v = np.zeros(len(st))
    v[pos[_index(K, occ)]] = 1.0
    return v


K = 5
DETS = [
    [(0, 0), (0, 1), (1, 0), (1, 1)],                  # closed shell
    [(0, 0), (2, 0), (4, 0), (1, 1)],                  # same-spin exchange
    [(1, 0), (3, 1), (2, 0), (2, 1), (4, 1)],          # odd count, open shells
    [(0, 1), (1, 1), (2, 1), (3, 0), (4, 0), (4, 1)],
]


@pytest.mark.parametrize("occ", DETS)
def test_determinant_energy_is_the_diagonal_element(occ):
    h, eri = W.abinitio_integrals(K, seed=4)
    st, pos = _sector(K, occ)
    H = ed.abinitio_hamiltonian(h, eri, st)
    v = _vec(K, st, pos, occ)
    assert abs(v @ (H @ v) - slater.determinant_energy(h, eri, occ)) < 1e-12


def test_determinant_energy_detects_a_dropped_exchange_term():
    # a version without the same-spin exchange differs from the diagonal
    # element, so the pin above is sensitive to that term
    h, eri = W.abinitio_integrals(K, seed=4)
    occ = DETS[1]
    no_x = sum(h[p, p] for p, _ in occ) + 0.5 * sum(eri[p, p, q, q] for p, _ in occ for q, _ in occ)
    assert abs(no_x - slater.determinant_energy(h, eri, occ)) > 1e-3


@pytest.mark.parametrize("p,q,others", [(0, 4, [(1, 0), (2, 1), (3, 0)]), (3, 1, [(0, 0), (0, 1), (2, 1)]),
                                        (2, 3, [])])
def test_pair_transfer_coupling_matches_the_off_diagonal_element(p, q, others):
    # electrons between p and q (odd counts included) change no sign
    h, eri = W.abinitio_integrals(K, seed=4)
    a = others + [(p, 0), (p, 1)]
    b = others + [(q, 0), (q, 1)]
    st, pos = _sector(K, a)
    H = ed.abinitio_hamiltonian(h, eri, st)
    va, vb = _vec(K, st, pos, a), _vec(K, st, pos, b)
    assert abs(vb @ (H @ va) - slater.pair_transfer_coupling(eri, p, q)) < 1e-12
    # and the two-state energy of a superposition
    c1, c2 = 0.8, -0.45
    psi = c1 * va + c2 * vb
    E = psi @ (H @ psi) / (psi @ psi)
    E1, E2 = slater.determinant_energy(h, eri, a), slater.determinant_energy(h, eri, b)
    assert abs(E - slater.two_state_energy(E1, E2, slater.pair_transfer_coupling(eri, p, q), c1, c2)) < 1e-12


@pytest.mark.parametrize("core,p,q", [([1, 3], 0, 4), ([0], 2, 1), ([], 3, 0)])
def test_open_shell_singlet_projected_energy(core, p, q):
    h, eri = W.abinitio_integrals(K, seed=4)
    occ = [(c, s) for c in core for s in (0, 1)] + [(p, 0), (q, 1)]
    st, pos = _sector(K, occ)
    H = ed.abinitio_hamiltonian(h, eri, st).toarray()
    P = ed.spin_projector_dense(ed.s2_operator(K, st), 0)
    v = _vec(K, st, pos, occ)
    E_ref, norm_ref = slater.open_shell_singlet(h, eri, core, p, q)
    assert abs(v @ P @ v - norm_ref) < 1e-12
    assert abs((v @ H @ P @ v) / (v @ P @ v) - E_ref) < 1e-11
    # the triplet part lies below the determinant by the same exchange integral
    Pt = ed.spin_projector_dense(ed.s2_operator(K, st), 2)
    Et = (v @ H @ Pt @ v) / (v @ Pt @ v)
    assert abs(Et - (slater.determinant_energy(h, eri, occ) - eri[p, q, q, p])) < 1e-11


@pytest.mark.parametrize("terms", [
    [(1.0, [(0, 0), (0, 1), (1, 0), (1, 1)])],
    [(0.8, [(0, 0), (0, 1), (2, 0), (1, 1)]), (-0.45, [(4, 0), (4, 1), (2, 0), (1, 1)])],
    [(0.6, [(1, 0), (1, 1), (2, 0), (2, 1)]), (0.3, [(1, 0), (1, 1), (3, 0), (3, 1)])],
])
def test_determinant_state_inputs(terms):
    # the block-table MPS built for the GPU closed-form tests contracts to
    # the intended combination of occupation-number states
    from det_states import product_state
    from oracle import mps as omps
    n = len(terms[0][1])
    tab, blocks = product_state(terms, K, n)
    psi = ed.mps_to_dense(omps.OracleMPS(tab, blocks).A)
    ref = np.zeros(4 ** K)
    for c, occ in terms:
        ref[_index(K, occ)] += c
    np.testing.assert_allclose(psi, ref, atol=1e-15)
