"""Quadrature for the spin projector (Sec. 2.2, Eqs. [PSMM], [pmpo],
[exactQuadrature]).  Test infrastructure only.

The projector restricted to a fixed M is written as an integral over the
rotation angle beta with weight sin(beta) d^S_MM(beta) (Eq. [PSMM]); with
x = cos(beta) the integral becomes a Gauss-Legendre sum over x (Eq. [pmpo]).
"""
from __future__ import annotations

import math

import numpy as np


def gauss_legendre(G: int):
    """Nodes and weights of the G-point Gauss-Legendre rule on [-1, 1].

    Golub-Welsch: the nodes are the eigenvalues of the symmetric tridiagonal
    Jacobi matrix of the Legendre recurrence (off-diagonal i/sqrt(4 i^2 - 1)),
    the weights are 2 times the squared first component of each normalised
    eigenvector.  Nodes ascending.
    """
    if G < 1:
        raise ValueError("G >= 1")
    i = np.arange(1, G, dtype=float)
    off = i / np.sqrt(4.0 * i * i - 1.0)
    J = np.diag(off, 1) + np.diag(off, -1)
    x, V = np.linalg.eigh(J)
    w = 2.0 * V[0, :] ** 2
    return x, w


def wigner_small_d_diag(twoJ: int, twoM: int, beta):
    """Wigner small-d element d^J_{MM}(beta) from Wigner's explicit sum.

    d^J_{MM}(b) = sum_k (-1)^k (J+M)! (J-M)! / [(J+M-k)! k! k! (J-M-k)!]
                  * cos(b/2)^(2J-2k) * sin(b/2)^(2k)
    (the diagonal case M' = M, real by the convention of Sec. 2.2).
    J and M are passed doubled so half-integers are exact.
    """
    if (twoJ - twoM) % 2 or abs(twoM) > twoJ:
        raise ValueError("need |M| <= J and J - M integer")
    jpm = (twoJ + twoM) // 2
    jmm = (twoJ - twoM) // 2
    b = np.asarray(beta, dtype=float)
    c = np.cos(b / 2.0)
    s = np.sin(b / 2.0)
    total = np.zeros_like(b)
    for k in range(0, min(jpm, jmm) + 1):
        num = math.factorial(jpm) * math.factorial(jmm)
        den = (math.factorial(jpm - k) * math.factorial(k) * math.factorial(k)
               * math.factorial(jmm - k))
        total = total + ((-1) ** k) * (num / den) * c ** (twoJ - 2 * k) * s ** (2 * k)
    return total


def max_seniority(N: int, twoM: int, K: int) -> int:
    """Largest number of singly occupied orbitals, Omega_max of
    Eq. [exactQuadrature]: min(N_a, K-N_b) + min(N_b, K-N_a)."""
    na = (N + twoM) // 2
    nb = (N - twoM) // 2
    return min(na, K - nb) + min(nb, K - na)


def exact_point_count(N: int, K: int, twoS: int, twoM: int = 0) -> int:
    """Smallest number of Gauss-Legendre points that makes the projector
    exact, Eq. [exactQuadrature]: ceil((Omega_max/2 + S + 1)/2).

    Computed in doubled units: ceil((Omega + 2S + 2)/4)."""
    om = max_seniority(N, twoM, K)
    return -(-(om + twoS + 2) // 4)


def projector_quadrature(G: int, twoS: int, twoM: int):
    """Quadrature table of the projector, Eq. [pmpo] with the (2S+1)/2
    normalisation of Eq. [PSMM]:

        P = sum_g coef_g exp(-i beta_g S_y),
        coef_g = (2S+1)/2 * w_g * d^S_MM(beta_g),  beta_g = arccos(x_g).

    Returns a dict of arrays over g in ascending x_g: x, w, beta, c, s, coef,
    with c = cos(beta/2) = sqrt((1+x)/2), s = sin(beta/2) = sqrt((1-x)/2).
    """
    x, w = gauss_legendre(G)
    beta = np.arccos(x)
    c = np.cos(beta / 2.0)
    s = np.sin(beta / 2.0)
    d = wigner_small_d_diag(twoS, twoM, beta)
    coef = (twoS + 1) / 2.0 * w * d
    return dict(x=x, w=w, beta=beta, c=c, s=s, coef=coef)
