"""Pins of the oracle's exact diagonalisation against closed forms."""
import json
import math
import os

import numpy as np
import pytest

from oracle import ed

ED = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "ed_energies.json")))


def _ground(L, N, twoM, U, twoS, t=1.0):
    st = ed.sector_states(L, N, twoM)
    H = ed.hubbard_hamiltonian(L, t, U, st)
    S2 = ed.s2_operator(L, st)
    return ed.projected_ground_energy(H, ed.lowdin_projector(S2, twoS, twoM, N))


@pytest.mark.parametrize("U", [0.0, 1.0, 4.0, 8.0])
def test_two_site_closed_form(U):
    # two-site Hubbard dimer, N = 2: singlet (U - sqrt(U^2 + 16 t^2))/2, triplet 0
    assert abs(_ground(2, 2, 0, U, 0) - (U - math.sqrt(U * U + 16.0)) / 2) < 1e-12
    assert abs(_ground(2, 2, 0, U, 2)) < 1e-12


@pytest.mark.parametrize("L", [4, 6, 8])
def test_free_chain_closed_form(L):
    # U = 0, N = L: eps_j = -2 cos(pi j/(L+1)); singlet fills the lowest L/2
    # levels twice, the triplet promotes one electron across the Fermi level
    eps = np.sort(-2.0 * np.cos(np.pi * np.arange(1, L + 1) / (L + 1)))
    e0 = 2.0 * eps[: L // 2].sum()
    e1 = e0 - eps[L // 2 - 1] + eps[L // 2]
    assert abs(_ground(L, L, 0, 0.0, 0) - e0) < 1e-11
    assert abs(_ground(L, L, 0, 0.0, 2) - e1) < 1e-11


def test_s2_eigenvalues_are_spin_values():
    st = ed.sector_states(4, 4, 0)
    ev = np.linalg.eigvalsh(ed.s2_operator(4, st).toarray())
    allowed = np.array([s * (s + 1) for s in (0, 1, 2)])
    assert np.all(np.min(np.abs(ev[:, None] - allowed[None, :]), axis=1) < 1e-12)


def test_hamiltonian_commutes_with_s2():
    st = ed.sector_states(4, 4, 0)
    H = ed.hubbard_hamiltonian(4, 1.0, 3.0, st).toarray()
    S2 = ed.s2_operator(4, st).toarray()
    assert np.abs(H @ S2 - S2 @ H).max() < 1e-12


def test_abinitio_reduces_to_hubbard():
    # h = -t on nearest neighbours, (pp|pp) = U only: the Hubbard chain
    L, t, U = 4, 1.0, 3.0
    h = np.zeros((L, L))
    for p in range(L - 1):
        h[p, p + 1] = h[p + 1, p] = -t
    eri = np.zeros((L, L, L, L))
    for p in range(L):
        eri[p, p, p, p] = U
    for (N, twoM) in [(4, 0), (3, 1), (5, -1)]:
        st = ed.sector_states(L, N, twoM)
        A = ed.abinitio_hamiltonian(h, eri, st).toarray()
        B = ed.hubbard_hamiltonian(L, t, U, st).toarray()
        np.testing.assert_allclose(A, B, atol=1e-13)


@pytest.mark.parametrize("case", ED["cases"])
def test_stored_ed_energies(case):
    assert abs(_ground(case["L"], case["N"], case["twoM"], case["U"], case["twoS"]) - case["E"]) < 1e-10
