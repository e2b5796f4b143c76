"""Pins of the oracle's local matrices, rotations and MPOs against the
paper's printed matrices, library routines and brute force."""
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import ed, local_ops as lo, mpo, quadrature as q

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "local_matrices.json")))


def test_jw_matrices_match_paper():
    jw = GOLDEN["jw"]
    pairs = dict(I=lo.I2, I_tilde=lo.I_T, a_dag=lo.CDAG, a_dag_tilde=lo.CDAG_T, a=lo.C,
                 a_tilde=lo.C_T, n=lo.NUM, n_tilde=lo.NUM_T)
    for name, mat in pairs.items():
        np.testing.assert_array_equal(mat, np.array(jw[name], dtype=float), err_msg=name)


def test_spatial_spin_matrices_match_paper():
    sp_ = GOLDEN["spatial"]
    pairs = dict(I=lo.I4, S_plus=lo.S_PLUS, S_minus=lo.S_MINUS, S_z=lo.S_Z, S2=lo.S2_LOCAL)
    for name, mat in pairs.items():
        np.testing.assert_array_equal(mat, np.array(sp_[name], dtype=float), err_msg=name)


def test_rotation_matches_paper_pattern():
    beta = 0.731
    c, s = math.cos(beta / 2), math.sin(beta / 2)
    val = {"1": 1.0, "0": 0.0, "c": c, "s": s, "-s": -s}
    ref = np.array([[val[e] for e in row] for row in GOLDEN["rotation_pattern"]["matrix"]])
    np.testing.assert_allclose(lo.rotation(beta), ref, atol=1e-16)


def test_rotation_group_properties():
    a, b = 0.4, 1.3
    ra, rb = lo.rotation(a), lo.rotation(b)
    np.testing.assert_allclose(ra @ ra.T, np.eye(4), atol=1e-15)
    assert abs(np.linalg.det(ra) - 1.0) < 1e-15
    np.testing.assert_allclose(ra @ rb, lo.rotation(a + b), atol=1e-15)


@pytest.mark.parametrize("L", [1, 2, 3])
def test_product_rotation_is_exp_sy(L):
    # exp(-i beta S_y) with S_y = (S_+ - S_-)/(2i)  ->  expm(-beta/2 (S_+ - S_-)), real
    states = np.arange(4 ** L)
    Sp = np.zeros((4 ** L, 4 ** L))
    for k in range(1, L + 1):
        a, b = ed._bit(L, k, 0), ed._bit(L, k, 1)
        for i in states:
            out = ed.apply_cdag_c(int(i), a, b)
            if out is not None:
                Sp[out[0], i] += out[1]
    for beta in (0.3, 1.7, 2.9):
        R = sla.expm(-0.5 * beta * (Sp - Sp.T))
        np.testing.assert_allclose(ed.rotation_dense(L, lo.rotation(beta)), R, atol=1e-13)


@pytest.mark.parametrize("L", [2, 3, 4])
def test_hubbard_mpo_equals_ed(L):
    Hd = mpo.mpo_to_dense(mpo.hubbard_mpo(L, 1.3, 3.7))
    for N in range(0, 2 * L + 1):
        for twoM in range(-min(N, 2 * L - N), min(N, 2 * L - N) + 1, 2):
            st = ed.sector_states(L, N, twoM)
            if len(st) == 0:
                continue
            He = ed.hubbard_hamiltonian(L, 1.3, 3.7, st).toarray()
            np.testing.assert_allclose(Hd[np.ix_(st, st)], He, atol=1e-14)
    # the MPO conserves N and M: no element between different sectors
    idx = np.arange(4 ** L)
    na = sum(((idx >> (2 * (L - k))) & 3) >> 1 for k in range(1, L + 1))
    nb = sum(((idx >> (2 * (L - k))) & 3) & 1 for k in range(1, L + 1))
    diff = (na[:, None] != na[None, :]) | (nb[:, None] != nb[None, :])
    assert np.abs(Hd[diff]).max() == 0.0


@pytest.mark.parametrize("L", [2, 3, 4])
def test_s2_mpo_equals_ed(L):
    S2d = mpo.mpo_to_dense(mpo.s2_mpo(L))
    for N in range(0, 2 * L + 1):
        for twoM in range(-min(N, 2 * L - N), min(N, 2 * L - N) + 1, 2):
            st = ed.sector_states(L, N, twoM)
            S2e = ed.s2_operator(L, st).toarray()
            np.testing.assert_allclose(S2d[np.ix_(st, st)], S2e, atol=1e-14)


def _projector_quadrature_dense(L, G, twoS, twoM, st):
    t = q.projector_quadrature(G, twoS, twoM)
    P = np.zeros((len(st), len(st)))
    for g in range(G):
        R = ed.rotation_dense(L, lo.rotation(t["beta"][g]))
        P += t["coef"][g] * R[np.ix_(st, st)]
    return P


@pytest.mark.parametrize("L,N,twoM", [(3, 3, 1), (4, 4, 0), (4, 3, 1), (5, 5, 1)])
def test_quadrature_projector_exact_at_min_points(L, N, twoM):
    st = ed.sector_states(L, N, twoM)
    S2 = ed.s2_operator(L, st)
    smax = min(N, 2 * L - N)
    for twoS in range(abs(twoM), smax + 1, 2):
        Pex = ed.spin_projector_dense(S2, twoS)
        G = q.exact_point_count(N, L, twoS, twoM)
        P = _projector_quadrature_dense(L, G, twoS, twoM, st)
        np.testing.assert_allclose(P, Pex, atol=1e-13)
        np.testing.assert_allclose(P @ P, P, atol=1e-13)
        # tightness: one point fewer is not exact
        if G > 1:
            Pm = _projector_quadrature_dense(L, G - 1, twoS, twoM, st)
            assert np.abs(Pm - Pex).max() > 1e-4, (L, N, twoS)


def test_projector_multiplicities_L4():
    st = ed.sector_states(4, 4, 0)
    traces = []
    for twoS in (0, 2, 4):
        G = q.exact_point_count(4, 4, twoS)
        traces.append(round(np.trace(_projector_quadrature_dense(4, G, twoS, 0, st)), 10))
    assert traces == [20.0, 15.0, 1.0]


def test_lowdin_equals_eigen_projector():
    st = ed.sector_states(5, 5, 1)
    S2 = ed.s2_operator(5, st)
    for twoS in (1, 3, 5):
        Pex = ed.spin_projector_dense(S2, twoS)
        Pl = ed.lowdin_projector(S2, twoS, 1, 5)
        v = np.random.default_rng(0).standard_normal(len(st))
        np.testing.assert_allclose(Pl(v), Pex @ v, atol=1e-11)
