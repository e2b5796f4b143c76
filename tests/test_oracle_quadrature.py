"""Pins of the oracle's projector quadrature (Sec. 2.2, Eqs. [PSMM], [pmpo],
[exactQuadrature]) against closed forms and independent library routines."""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate

from oracle import quadrature as q

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "local_matrices.json")


@pytest.mark.parametrize("G", range(1, 14))
def test_gauss_legendre_matches_numpy(G):
    x, w = q.gauss_legendre(G)
    x2, w2 = np.polynomial.legendre.leggauss(G)
    assert np.all(np.diff(x) > 0)
    np.testing.assert_allclose(x, x2, atol=1e-14)
    np.testing.assert_allclose(w, w2, atol=1e-14)


@pytest.mark.parametrize("G", [1, 2, 5, 9, 11])
def test_gauss_legendre_exact_degree(G):
    x, w = q.gauss_legendre(G)
    assert abs(w.sum() - 2.0) < 1e-14
    for j in range(2 * G):
        exact = 2.0 / (j + 1) if j % 2 == 0 else 0.0
        assert abs(np.dot(w, x ** j) - exact) < 1e-13, j
    j = 2 * G  # first degree that a G-point rule cannot integrate
    assert abs(np.dot(w, x ** j) - 2.0 / (j + 1)) > 1e-9


@pytest.mark.parametrize("S", [0, 1, 2, 3, 4])
def test_wigner_d_m0_is_legendre(S):
    beta = np.linspace(0.0, math.pi, 17)
    d = q.wigner_small_d_diag(2 * S, 0, beta)
    ref = np.polynomial.legendre.Legendre.basis(S)(np.cos(beta))
    np.testing.assert_allclose(d, ref, atol=1e-14)


def test_wigner_d_closed_forms():
    beta = np.linspace(0.0, math.pi, 13)
    c, s = np.cos(beta / 2), np.sin(beta / 2)
    np.testing.assert_allclose(q.wigner_small_d_diag(1, 1, beta), c, atol=1e-15)
    np.testing.assert_allclose(q.wigner_small_d_diag(1, -1, beta), c, atol=1e-15)
    # d^1_11 = (1 + cos b)/2, d^{3/2}_{1/2 1/2} = c (3c^2 - 2)
    np.testing.assert_allclose(q.wigner_small_d_diag(2, 2, beta), (1 + np.cos(beta)) / 2, atol=1e-15)
    np.testing.assert_allclose(q.wigner_small_d_diag(3, 1, beta), c * (3 * c * c - 2), atol=1e-14)
    for twoJ in range(0, 9):
        for twoM in range(-twoJ, twoJ + 1, 2):
            assert abs(q.wigner_small_d_diag(twoJ, twoM, 0.0) - 1.0) < 1e-15


@pytest.mark.parametrize("twoM", [0, 1, 2])
def test_wigner_d_orthogonality(twoM):
    # int_0^pi d^S_MM d^S'_MM sin(b) db = 2 delta / (2S+1), scipy adaptive quadrature
    Js = [j for j in range(abs(twoM), 8, 2)]
    for a in Js:
        for b in Js:
            f = lambda be: (q.wigner_small_d_diag(a, twoM, be) * q.wigner_small_d_diag(b, twoM, be)
                            * math.sin(be))
            val, _ = integrate.quad(f, 0.0, math.pi, epsabs=1e-13)
            ref = 2.0 / (a + 1) if a == b else 0.0
            assert abs(val - ref) < 1e-11, (a, b)


def test_exact_point_count_printed_case():
    g = json.load(open(GOLDEN))["exact_points_4x4_hubbard"]
    assert q.exact_point_count(g["N"], g["K"], g["twoS"], g["twoM"]) == g["N_g"]


def test_exact_point_count_both_branches():
    # Omega_max = N below half filling, 2K - N above
    assert q.max_seniority(6, 0, 10) == 6
    assert q.max_seniority(14, 0, 10) == 6
    assert q.max_seniority(8, 0, 8) == 8
    assert q.exact_point_count(8, 8, 0) == 3
    assert q.exact_point_count(32, 32, 0) == 9
    assert q.exact_point_count(32, 32, 2) == 9
    assert q.exact_point_count(48, 48, 0) == 13


def test_projector_coefficients():
    t = q.projector_quadrature(9, 2, 0)
    np.testing.assert_allclose(t["c"] ** 2 + t["s"] ** 2, 1.0, atol=1e-15)
    np.testing.assert_allclose(t["c"], np.sqrt((1 + t["x"]) / 2), atol=1e-15)
    # S = 1, M = 0: coef = 3/2 w_g x_g
    np.testing.assert_allclose(t["coef"], 1.5 * t["w"] * t["x"], atol=1e-15)
