"""The 30-orbital ab-initio workload at its full orbital count (K=30, N=30,
S=0, G=11, the seeded integrals of the benchmark workload) against closed
forms: states made of one or two occupation-number determinants, whose
projected energy and projected norm follow from the Slater-Condon rules
(oracle.slater, pinned against exact diagonalisation).  The library builds
the full MPO (channel count about 1.9e3 at the centre), the rotated
environments of every quadrature point through all 30 sites and the
projected energy at site 1; these values check all of it at the size where
the dense oracle does not fit."""
import numpy as np
import pytest

import paper_1703_04789_amd as sp
import workloads as W
from det_states import product_state
from oracle import slater

pytestmark = pytest.mark.gpu

K, N, G = 30, 30, 11


@pytest.fixture(scope="module")
def ham():
    h, eri = W.abinitio_full().integrals()
    return h, eri, sp.mpo_abinitio(h, eri)


def _energy(ham, terms, path):
    h, eri, mpo = ham
    tab, blocks = product_state(terms, K, N)
    print(f"[case] K={K} determinants={len(terms)} path={path} bond dims "
          f"{max(tab.bond_dim(b) for b in range(K + 1))}", flush=True)
    st = sp.SPMPS(tab, blocks, mpo, 0, G, path=path)
    try:
        return st.energy()
    finally:
        st.close()


CORE = list(range(15))


@pytest.mark.parametrize("path", ["tiled", "plain"])
def test_closed_shell_determinant(ham, path):
    h, eri, _ = ham
    occ = [(p, s) for p in CORE for s in (0, 1)]
    E, normP = _energy(ham, [(1.0, occ)], path)
    assert abs(normP - 1.0) < 1e-10
    assert abs(E - slater.determinant_energy(h, eri, occ)) < 1e-8


def test_pair_transfer_superposition(ham):
    # the pair of orbital 7 moved to orbital 22: the coupling runs through
    # the centre of the chain
    h, eri, _ = ham
    p, q = 7, 22
    a = [(o, s) for o in CORE for s in (0, 1)]
    b = [(o, s) for o in CORE if o != p for s in (0, 1)] + [(q, 0), (q, 1)]
    c1, c2 = 0.8, -0.45
    E, normP = _energy(ham, [(c1, a), (c2, b)], "tiled")
    E_ref = slater.two_state_energy(slater.determinant_energy(h, eri, a), slater.determinant_energy(h, eri, b),
                                    slater.pair_transfer_coupling(eri, p, q), c1, c2)
    assert abs(normP - 1.0) < 1e-10
    assert abs(E - E_ref) < 1e-8


def test_open_shell_singlet(ham):
    # 14 doubly occupied orbitals plus 14 alpha and 20 beta: half of the
    # determinant is singlet, and the projected energy is the singlet's
    h, eri, _ = ham
    core, p, q = list(range(14)), 14, 20
    occ = [(o, s) for o in core for s in (0, 1)] + [(p, 0), (q, 1)]
    E, normP = _energy(ham, [(1.0, occ)], "tiled")
    E_ref, n_ref = slater.open_shell_singlet(h, eri, core, p, q)
    assert abs(normP - n_ref) < 1e-10
    assert abs(E - E_ref) < 1e-8


def test_full_size_state_is_projected_to_the_singlet():
    # the seeded K=30, D=500 starting state of the 30-orbital workload with
    # the S^2 operator in place of H: <S^2 P>/<P> = 0 for the S=0 projector
    # with G=11 points (above the exact count), through the full block table
    # and all 11 rotated environments
    wl = W.abinitio_full()
    tab = wl.table()
    print(f"[case] K={wl.K} D={wl.D} G={wl.G} S^2", flush=True)
    st = sp.SPMPS(tab, wl.blocks(), sp.mpo_s2(wl.K), wl.twoS, wl.G)
    try:
        s2, normP = st.energy()
    finally:
        st.close()
    assert abs(s2) < 1e-8 and 0.0 < normP < 1.0


def test_full_size_centre_products_are_symmetric():
    # H_eff and N_eff at the centre of the K=30, D=500, G=11 state (the
    # benchmark's tiled plan: 64 x 64 tiles, split channel sums) are the
    # symmetric matrices Phi^T H P Phi and Phi^T P Phi (P commutes with H and
    # is symmetric, the quadrature being exact), and N_eff is positive
    # semidefinite: <u, H v> = <v, H u>, <u, N v> = <v, N u>, <u, N u> >= 0
    import torch
    wl = W.abinitio_full()
    h, eri = wl.integrals()
    print(f"[case] K={wl.K} D={wl.D} G={wl.G} centre products", flush=True)
    st = sp.SPMPS(wl.table(), wl.blocks(), sp.mpo_abinitio(h, eri), wl.twoS, wl.G)
    try:
        kc = wl.K // 2
        for j in range(1, kc):
            st.env_update(j, +1)
        n = st.site_size(kc)
        rng = np.random.default_rng(30)
        u = torch.tensor(rng.standard_normal(n), dtype=torch.float64, device="cuda")
        v = torch.tensor(rng.standard_normal(n), dtype=torch.float64, device="cuda")
        hu, nu, hv, nv = (torch.empty_like(u) for _ in range(4))
        st.heff_apply(kc, u, hu, nu)
        st.heff_apply(kc, v, hv, nv)
        torch.cuda.synchronize()
        scale_h = float(torch.linalg.norm(u) * max(torch.linalg.norm(hu), torch.linalg.norm(hv)))
        scale_n = float(torch.linalg.norm(u) * max(torch.linalg.norm(nu), torch.linalg.norm(nv)))
        assert abs(float(u @ hv - v @ hu)) < 1e-11 * scale_h
        assert abs(float(u @ nv - v @ nu)) < 1e-11 * scale_n
        assert float(u @ nu) > -1e-11 * scale_n and float(v @ nv) > -1e-11 * scale_n
    finally:
        st.close()
