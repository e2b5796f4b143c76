"""Closed-form energies of occupation-number states of the ab-initio
Hamiltonian.  Test infrastructure only.

For the second-quantised Hamiltonian of Sec. 2.1 (Eq. [sqH], chemists'
integrals (pq|rs), real orbitals) the expectation values of single
occupation-number states (Slater determinants) and the coupling of two of
them follow from the Slater-Condon rules; with the spin projector of
Sec. 2.2 (Eq. [efunctional]) an open-shell determinant of two unpaired
electrons of opposite spin has a closed-form projected energy as well.
These give exact values for the projected energy functional at any number
of orbitals, including sizes where no exact diagonalisation or dense MPO
fits (the 30-orbital workload), so they pin the library's MPO, rotated
environments and projected energy there.

Spin orbitals are (p, s): p the 0-based spatial orbital, s = 0 (alpha) or
1 (beta).  Every function is pinned against exact diagonalisation in the
tests (brute force on small orbital counts).
"""
from __future__ import annotations

import numpy as np


def determinant_energy(h: np.ndarray, eri: np.ndarray, occ) -> float:
    """<Phi|H|Phi> for the determinant with occupied spin orbitals ``occ``:
    the diagonal Slater-Condon rule,
        sum_i h_ii + 1/2 sum_{i,j} [ (ii|jj) - delta(s_i, s_j) (ij|ji) ],
    over occupied spin orbitals i = (p_i, s_i), j = (p_j, s_j) (the i = j
    terms cancel)."""
    occ = list(occ)
    if len(set(occ)) != len(occ):
        raise ValueError("a spin orbital is occupied twice")
    E = 0.0
    for (p, _) in occ:
        E += h[p, p]
    for (p, s) in occ:
        for (q, t) in occ:
            E += 0.5 * eri[p, p, q, q]
            if s == t:
                E -= 0.5 * eri[p, q, q, p]
    return float(E)


def pair_transfer_coupling(eri: np.ndarray, p: int, q: int) -> float:
    """<Phi'|H|Phi> where Phi has orbital p doubly occupied and q empty and
    Phi' is Phi with that pair moved from p to q (p != q): only the
    two-electron part connects them (a double excitation), through the term
    a+_{q alpha} a+_{q beta} a_{p beta} a_{p alpha} with coefficient
    (qp|qp) = (pq|pq).  Moving a pair past other electrons changes no sign,
    so the value is independent of the electrons in other orbitals."""
    if p == q:
        raise ValueError("p and q must differ")
    return float(eri[p, q, p, q])


def two_state_energy(E1: float, E2: float, V12: float, c1: float, c2: float) -> float:
    """<Psi|H|Psi>/<Psi|Psi> for Psi = c1 Phi1 + c2 Phi2 with orthonormal
    Phi1, Phi2, diagonal energies E1, E2 and real coupling V12."""
    return float((c1 * c1 * E1 + c2 * c2 * E2 + 2.0 * c1 * c2 * V12) / (c1 * c1 + c2 * c2))


def open_shell_singlet(h: np.ndarray, eri: np.ndarray, core, p: int, q: int):
    """Projected energy and projected norm of Phi = |core, p alpha, q beta>
    (``core``: doubly occupied spatial orbitals, p != q outside it) with the
    S = 0 projector: Phi is an equal mixture of the open-shell singlet and the
    M = 0 triplet, so <Phi|P|Phi> = 1/2 and the projected energy is the
    singlet's, E_det + (pq|qp), where E_det = <Phi|H|Phi> (the singlet lies
    above the determinant by the exchange integral, the triplet below it).
    Returns (energy, <P>)."""
    core = list(core)
    if p == q or p in core or q in core:
        raise ValueError("p, q must be distinct open-shell orbitals outside the core")
    occ = [(c, s) for c in core for s in (0, 1)] + [(p, 0), (q, 1)]
    return determinant_energy(h, eri, occ) + float(eri[p, q, q, p]), 0.5
