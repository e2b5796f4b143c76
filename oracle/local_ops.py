"""Local operator matrices (Secs. 2.1 and 2.2).  Test infrastructure only.

Spin-orbital matrices in the basis {|0>, |1>} follow the Jordan-Wigner
table of Sec. 2.1 (Eq. [JWtrans]).  A spatial orbital is the merge of its
alpha and beta spin orbitals with alpha first in the Jordan-Wigner order, so
the 4-dim local index is 2*n_alpha + n_beta, i.e. the basis
(|0>, |b>, |a>, |ab>) with |ab> = a^+_alpha a^+_beta |0> (Sec. 2.2, the
basis under Eq. [Sfac]).
"""
from __future__ import annotations

import numpy as np

# --- spin-orbital (2x2) matrices, Eq. [JWtrans] ---------------------------
I2 = np.eye(2)
SZ = np.array([[1.0, 0.0], [0.0, -1.0]])      # sigma_z  = [I~]
SM = np.array([[0.0, 0.0], [1.0, 0.0]])       # sigma_-  = [a^+]
SP = np.array([[0.0, 1.0], [0.0, 0.0]])       # sigma_+  = [a]
CDAG = SM
C = SP
NUM = SM @ SP                                  # [n]
CDAG_T = SM @ SZ                               # [a^+~]
C_T = SP @ SZ                                  # [a~]
NUM_T = SM @ SP @ SZ                           # [n~]
I_T = SZ                                       # [I~]

# --- spatial orbital (4x4), alpha slower index, alpha first in JW order ----
I4 = np.eye(4)
CDAG_A = np.kron(CDAG, I2)
CDAG_B = np.kron(SZ, CDAG)
C_A = np.kron(C, I2)
C_B = np.kron(SZ, C)
N_A = np.kron(NUM, I2)
N_B = np.kron(I2, NUM)
PARITY = np.kron(SZ, SZ)                       # (-1)^(n_a + n_b)

# spin operators (Sec. 2.2, local matrices under Eq. [Sfac])
S_PLUS = CDAG_A @ C_B
S_MINUS = CDAG_B @ C_A
S_Z = 0.5 * (N_A - N_B)
S2_LOCAL = S_Z @ S_Z + 0.5 * (S_PLUS @ S_MINUS + S_MINUS @ S_PLUS)


def rotation(beta: float) -> np.ndarray:
    """Matrix of exp(-i beta S_y) on one spatial orbital, Eq. [expSy]:
    identity on |0> and |ab>, a plane rotation by beta/2 on (|b>, |a>)."""
    c = np.cos(beta / 2.0)
    s = np.sin(beta / 2.0)
    r = np.eye(4)
    r[1, 1] = c
    r[1, 2] = s
    r[2, 1] = -s
    r[2, 2] = c
    return r


def rotation_cs(c: float, s: float) -> np.ndarray:
    """Same as :func:`rotation` from c = cos(beta/2), s = sin(beta/2)."""
    r = np.eye(4)
    r[1, 1] = c
    r[1, 2] = s
    r[2, 1] = -s
    r[2, 2] = c
    return r
