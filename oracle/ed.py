"""Exact diagonalisation in the occupation-number basis.  Test
infrastructure only.

This is the plain definition of every quantity the SP-MPS method computes:
Fock-space wavefunctions (Sec. 2.1, Eq. [FSwf]), the second-quantised
Hamiltonian (Eq. [sqH]; the Hubbard model of Sec. 3 as a special case), the
total spin S^2, the exact spin projector, and the projected energy
functional (Sec. 2.2, Eq. [efunctional]).

Basis: 4^L states, index = sum_k sigma_k 4^(L-k) with site 1 the most
significant digit and sigma_k = 2 n_{k alpha} + n_{k beta}.  Spin orbitals
are ordered 1a, 1b, 2a, 2b, ... and an occupation state is the ordered
product of creators in that order acting on the vacuum; this is the ordering
that the Jordan-Wigner matrices of Sec. 2.1 encode.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def _bit(L: int, k: int, spin: int) -> int:
    """Bit position of spin orbital (k, spin), k 1-based, spin 0=alpha 1=beta.
    Earlier spin orbitals in the Jordan-Wigner order sit at higher bits."""
    return 2 * (L - k) + (1 if spin == 0 else 0)


def _above(i: int, pos: int) -> int:
    """Number of occupied spin orbitals that precede bit ``pos`` in JW order."""
    return bin(i >> (pos + 1)).count("1")


def apply_cdag_c(i: int, p: int, q: int):
    """c^+_p c_q |i>  ->  (j, sign) or None; p, q are bit positions."""
    if not (i >> q) & 1:
        return None
    s1 = _above(i, q)
    i2 = i ^ (1 << q)
    if (i2 >> p) & 1:
        return None
    s2 = _above(i2, p)
    return i2 | (1 << p), (-1) ** (s1 + s2)


def apply_ops(i: int, ops):
    """Apply a product of single creators/annihilators to |i>.

    ``ops`` lists (kind, bit) in operator-product order, leftmost first;
    kind 1 = creator, 0 = annihilator.  The rightmost acts first.  Returns
    (j, sign) or None."""
    sign = 1
    for kind, pos in reversed(ops):
        occ = (i >> pos) & 1
        if kind == 1 and occ or kind == 0 and not occ:
            return None
        if _above(i, pos) & 1:
            sign = -sign
        i ^= (1 << pos)
    return i, sign


def apply_two(i: int, p: int, r: int, s: int, q: int):
    """c^+_p c^+_r c_s c_q |i> -> (j, sign) or None (bit positions)."""
    return apply_ops(i, ((1, p), (1, r), (0, s), (0, q)))


def sector_states(L: int, N: int, twoM: int) -> np.ndarray:
    """Sorted basis indices with N electrons and n_alpha - n_beta = twoM."""
    out = []
    for i in range(4 ** L):
        na = nb = 0
        for k in range(1, L + 1):
            sgm = (i >> (2 * (L - k))) & 3
            na += sgm >> 1
            nb += sgm & 1
        if na + nb == N and na - nb == twoM:
            out.append(i)
    return np.array(out, dtype=np.int64)


def _build(states, L, terms):
    """Sparse matrix of sum_terms coef * (operator string) on a sector.
    ``terms`` yields (coef, fn) where fn(i) -> (j, sign) or None."""
    index = {int(s): n for n, s in enumerate(states)}
    rows, cols, vals = [], [], []
    for n, i in enumerate(states):
        i = int(i)
        for coef, fn in terms:
            out = fn(i)
            if out is None:
                continue
            j, sg = out
            m = index.get(j)
            if m is None:
                raise ValueError("operator leaves the sector")
            rows.append(m)
            cols.append(n)
            vals.append(coef * sg)
    dim = len(states)
    return sp.csr_matrix((vals, (rows, cols)), shape=(dim, dim))


def hubbard_hamiltonian(L: int, t: float, U: float, states) -> sp.csr_matrix:
    """Open-chain Hubbard Hamiltonian on the given sector basis."""
    terms = []
    for k in range(1, L):
        for spin in (0, 1):
            a = _bit(L, k, spin)
            b = _bit(L, k + 1, spin)
            terms.append((-t, lambda i, a=a, b=b: apply_cdag_c(i, a, b)))
            terms.append((-t, lambda i, a=a, b=b: apply_cdag_c(i, b, a)))
    for k in range(1, L + 1):
        a = _bit(L, k, 0)
        b = _bit(L, k, 1)
        terms.append((U, lambda i, a=a, b=b: (i, 1) if ((i >> a) & 1 and (i >> b) & 1) else None))
    return _build(states, L, terms)


def abinitio_hamiltonian(h: np.ndarray, eri: np.ndarray, states) -> sp.csr_matrix:
    """H = sum_pq h_pq sum_s c+_ps c_qs
         + 1/2 sum_pqrs (pq|rs) sum_{s,t} c+_ps c+_rt c_st c_qs
    (Eq. [sqH] with g_{pr,qs} = (pq|rs) in chemists' notation)."""
    K = h.shape[0]
    terms = []
    for p in range(K):
        for q in range(K):
            if h[p, q] != 0.0:
                for s in (0, 1):
                    bp, bq = _bit(K, p + 1, s), _bit(K, q + 1, s)
                    terms.append((h[p, q], lambda i, a=bp, b=bq: apply_cdag_c(i, a, b)))
    for p in range(K):
        for q in range(K):
            for r in range(K):
                for s_ in range(K):
                    v = eri[p, q, r, s_]
                    if v == 0.0:
                        continue
                    for sa in (0, 1):
                        for sb in (0, 1):
                            bp, bq = _bit(K, p + 1, sa), _bit(K, q + 1, sa)
                            br, bs = _bit(K, r + 1, sb), _bit(K, s_ + 1, sb)
                            terms.append((0.5 * v, lambda i, bp=bp, br=br, bs=bs, bq=bq:
                                          apply_two(i, bp, br, bs, bq)))
    return _build(states, K, terms)


def s2_operator(L: int, states) -> sp.csr_matrix:
    """Total spin S^2 = S_z^2 + (S_+ S_- + S_- S_+)/2 on a sector basis,
    with S_+ = sum_k c+_{k alpha} c_{k beta}."""
    terms_pm = []
    for k in range(1, L + 1):
        for l in range(1, L + 1):
            ak, bk = _bit(L, k, 0), _bit(L, k, 1)
            al, bl = _bit(L, l, 0), _bit(L, l, 1)
            # S_+^k S_-^l  and  S_-^k S_+^l
            terms_pm.append((0.5, lambda i, ak=ak, bk=bk, al=al, bl=bl:
                             _chain(i, (bl, al), (ak, bk))))
            terms_pm.append((0.5, lambda i, ak=ak, bk=bk, al=al, bl=bl:
                             _chain(i, (al, bl), (bk, ak))))
    def sz2(i):
        na = nb = 0
        for k in range(1, L + 1):
            na += (i >> _bit(L, k, 0)) & 1
            nb += (i >> _bit(L, k, 1)) & 1
        return i, 0.25 * (na - nb) ** 2
    terms = terms_pm + [(1.0, sz2)]
    return _build(states, L, terms)


def _chain(i, first, second):
    """Apply c+_{first[0]} c_{first[1]} then c+_{second[0]} c_{second[1]}."""
    out = apply_cdag_c(i, first[0], first[1])
    if out is None:
        return None
    j, s1 = out
    out2 = apply_cdag_c(j, second[0], second[1])
    if out2 is None:
        return None
    return out2[0], s1 * out2[1]


def spin_projector_dense(S2: sp.spmatrix, twoS: int) -> np.ndarray:
    """Exact projector onto total spin S in a sector: sum of v v^T over the
    eigenvectors of S^2 with eigenvalue S(S+1).  Dense; small sectors."""
    s = twoS / 2.0
    ev, V = np.linalg.eigh(S2.toarray())
    sel = np.abs(ev - s * (s + 1)) < 1e-8
    return V[:, sel] @ V[:, sel].T


def lowdin_projector(S2: sp.spmatrix, twoS: int, twoM: int, N: int):
    """Lowdin's product form of the spin projector (Sec. 2.2, Eq. [lowdin]),
    exact and applied as an operator: prod_{S' != S} (S^2 - S'(S'+1)) /
    (S(S+1) - S'(S'+1)) over every S' from |M| to N/2 in integer steps."""
    s = twoS / 2.0
    others = [x / 2.0 for x in range(abs(twoM), N + 1, 2) if x != twoS]

    def apply(v):
        out = np.array(v, dtype=float, copy=True)
        for sp_ in others:
            out = (S2 @ out - sp_ * (sp_ + 1) * out) / (s * (s + 1) - sp_ * (sp_ + 1))
        return out
    return apply


def projected_ground_energy(H: sp.spmatrix, P_apply, tol=1e-13) -> float:
    """Lowest eigenvalue of H within the range of the projector P: the
    lowest eigenvalue of P (H - c) P + c restricted to range(P), obtained
    from P (H - c) P with c above the spectrum of H."""
    c = float(abs(H).sum(axis=1).max()) + 1.0
    dim = H.shape[0]

    def mv(v):
        pv = P_apply(v)
        return P_apply(H @ pv - c * pv)
    op = spla.LinearOperator((dim, dim), matvec=mv, dtype=float)
    if dim <= 600:
        M = np.column_stack([mv(e) for e in np.eye(dim)])
        ev = np.linalg.eigvalsh(0.5 * (M + M.T))
        return float(ev[0] + c)
    rng = np.random.default_rng(0)
    v0 = P_apply(rng.standard_normal(dim))
    ev = spla.eigsh(op, k=1, which="SA", v0=v0, tol=tol, maxiter=20000,
                    return_eigenvectors=False)
    return float(ev[0] + c)


def mps_to_dense(A) -> np.ndarray:
    """Contract MPS site tensors A[k] (4, D_{k-1}, D_k) to the 4^L vector of
    Eq. [FSMPS]."""
    cur = A[0][:, 0, :]                      # (4, D1)
    for k in range(1, len(A)):
        cur = np.einsum("Sa,sab->Ssb", cur, A[k]).reshape(-1, A[k].shape[2])
    return cur[:, 0]


def rotation_dense(L: int, r: np.ndarray) -> np.ndarray:
    """Dense tensor product of the same 4x4 local matrix over L sites."""
    out = np.ones((1, 1))
    for _ in range(L):
        out = np.kron(out, r)
    return out


def projected_energy(psi_sector, H, P) -> tuple:
    """Plain definition of the projected energy functional at a fixed state,
    Eq. [efunctional] with the exact projector in place of the quadrature:
    (psi^T H P psi / psi^T P psi, psi^T P psi)."""
    ppsi = P @ psi_sector
    num = float(psi_sector @ (H @ ppsi))
    den = float(psi_sector @ ppsi)
    return num / den, den


def epq_operator(L: int, p: int, q: int, states) -> sp.csr_matrix:
    """E_pq = sum_s c+_{p s} c_{q s} on a sector basis (1-based sites)."""
    terms = []
    for spin in (0, 1):
        a, b = _bit(L, p, spin), _bit(L, q, spin)
        terms.append((1.0, lambda i, a=a, b=b: apply_cdag_c(i, a, b)))
    return _build(states, L, terms)


def spin_corr_operator(L: int, X: int, Y: int, states) -> sp.csr_matrix:
    """S_X . S_Y on a sector basis: S^z_X S^z_Y + (S^+_X S^-_Y + S^-_X S^+_Y)/2
    with S^+_k = c+_{k alpha} c_{k beta}."""
    ax, bx, ay, by = _bit(L, X, 0), _bit(L, X, 1), _bit(L, Y, 0), _bit(L, Y, 1)

    def szsz(i):
        sx = 0.5 * (((i >> ax) & 1) - ((i >> bx) & 1))
        sy = 0.5 * (((i >> ay) & 1) - ((i >> by) & 1))
        return i, sx * sy
    terms = [(1.0, szsz),
             (0.5, lambda i: _chain(i, (ay, by), (bx, ax))),   # S^+_X S^-_Y: S^-_Y acts first
             (0.5, lambda i: _chain(i, (by, ay), (ax, bx)))]   # S^-_X S^+_Y
    return _build(states, L, terms)
