"""Matrix product operators (Sec. 2.1, Eq. [FSMPO]; Sec. 2.2, Eq. [Sfac]).
Test infrastructure only.

An MPO is a list of L arrays W[k] of shape (w_left, w_right, 4, 4) with
W[k][a, b, s, t] = <s| O_ab |t>, the operator-valued matrix of the recursion
"vector of operators on sites [k, L] = W[k] times vector on [k+1, L]" used in
Sec. 2.1.  The first row of W[1] and the last column of W[L] are kept (the
boundary reading of Sec. 2.1), so W[1] has w_left = 1 and W[L] w_right = 1.
Row/column 0 carries the complete operator and the last row/column the
identity, as in Eq. [Sfac].
"""
from __future__ import annotations

import numpy as np

from . import local_ops as lo


def _trim(Ws):
    """Keep the first row of site 1 and the last column of site L."""
    Ws = [w.copy() for w in Ws]
    Ws[0] = Ws[0][:1]
    Ws[-1] = Ws[-1][:, -1:]
    return Ws


def hubbard_mpo(L: int, t: float, U: float):
    """Open-boundary 1D Hubbard chain
        H = -t sum_{k, sigma} (c+_{k sigma} c_{k+1 sigma} + h.c.)
            + U sum_k n_{k alpha} n_{k beta}
    as an MPO of bond dimension 6 built with the recursion of Sec. 2.1.

    Right-vector order (H, c_a, c_b, c+_a, c+_b, I) on sites [k+1, L].  A hop
    c+_{k s} c_{k+1 s} equals (c+_s F)_k (x) (c_s)_{k+1} and
    c+_{k+1 s} c_{k s} equals (F c_s)_k (x) (c+_s)_{k+1}, where F is the site
    parity (the Jordan-Wigner string of Eq. [JWtrans] over both spin
    orbitals of the site).
    """
    F = lo.PARITY
    w = np.zeros((6, 6, 4, 4))
    w[0, 0] = lo.I4
    w[0, 1] = -t * lo.CDAG_A @ F
    w[0, 2] = -t * lo.CDAG_B @ F
    w[0, 3] = -t * F @ lo.C_A
    w[0, 4] = -t * F @ lo.C_B
    w[0, 5] = U * lo.N_A @ lo.N_B
    w[1, 5] = lo.C_A
    w[2, 5] = lo.C_B
    w[3, 5] = lo.CDAG_A
    w[4, 5] = lo.CDAG_B
    w[5, 5] = lo.I4
    return _trim([w] * L)


def s2_mpo(L: int):
    """Total-spin S^2 as an MPO of bond dimension 5, Eq. [Sfac]:
    right-vector order (S^2, S_+, S_-, S_z, I)."""
    w = np.zeros((5, 5, 4, 4))
    w[0, 0] = lo.I4
    w[0, 1] = lo.S_MINUS
    w[0, 2] = lo.S_PLUS
    w[0, 3] = 2.0 * lo.S_Z
    w[0, 4] = lo.S2_LOCAL
    w[1, 1] = lo.I4
    w[1, 4] = lo.S_PLUS
    w[2, 2] = lo.I4
    w[2, 4] = lo.S_MINUS
    w[3, 3] = lo.I4
    w[3, 4] = lo.S_Z
    w[4, 4] = lo.I4
    return _trim([w] * L)


def _string_mpo(L, k0, k1, starts, ends, carry):
    """MPO of a sum of two-site products sum_c starts[c]_k0 (x) carry^(k1-k0-1)
    (x) ends[c]_k1 with k0 < k1, in the recursion layout: channel 0 of a
    right vector holds the complete operator of sites [k, L], channels
    1..nc an open product waiting for its left factor, the last channel the
    identity.  Built by filling that right-vector recursion directly."""
    nc = len(starts)
    w = nc + 2
    Ws = []
    for k in range(1, L + 1):
        W = np.zeros((w, w, 4, 4))
        W[0, 0] = lo.I4
        W[w - 1, w - 1] = lo.I4
        if k == k0:
            for c in range(nc):
                W[0, 1 + c] = starts[c]
        if k0 < k < k1:
            for c in range(nc):
                W[1 + c, 1 + c] = carry
        if k == k1:
            for c in range(nc):
                W[1 + c, w - 1] = ends[c]
        Ws.append(W)
    return _trim(Ws)


def site_op_mpo(L: int, p: int, op: np.ndarray):
    """A single-site operator op at site p (1-based), bond dimension 2."""
    Ws = []
    for k in range(1, L + 1):
        W = np.zeros((2, 2, 4, 4))
        W[0, 0] = lo.I4
        W[1, 1] = lo.I4
        if k == p:
            W[0, 1] = op
        Ws.append(W)
    return _trim(Ws)


def epq_mpo(L: int, p: int, q: int):
    """Spin-free one-body operator E_pq = sum_s a+_{p s} a_{q s} (Sec. 2.4).
    p == q gives n_p.  For p < q the left factor is a+_s F (F the site
    parity, the Jordan-Wigner string through the rest of site p), F is
    carried over the sites in between and a_s closes the product at q; for
    p > q the left factor is F a_s and a+_s closes it."""
    if p == q:
        return site_op_mpo(L, p, lo.N_A + lo.N_B)
    F = lo.PARITY
    if p < q:
        starts = [lo.CDAG_A @ F, lo.CDAG_B @ F]
        ends = [lo.C_A, lo.C_B]
    else:
        starts = [F @ lo.C_A, F @ lo.C_B]
        ends = [lo.CDAG_A, lo.CDAG_B]
    return _string_mpo(L, min(p, q), max(p, q), starts, ends, F)


def spin_corr_mpo(L: int, X: int, Y: int):
    """S_X . S_Y = S^z_X S^z_Y + (S^+_X S^-_Y + S^-_X S^+_Y)/2; X == Y gives
    the local S^2.  Spin operators are even: no string."""
    if X == Y:
        return site_op_mpo(L, X, lo.S2_LOCAL)
    starts = [lo.S_Z, 0.5 * lo.S_PLUS, 0.5 * lo.S_MINUS]
    ends = [lo.S_Z, lo.S_MINUS, lo.S_PLUS]
    return _string_mpo(L, min(X, Y), max(X, Y), starts, ends, lo.I4)


def identity_mpo(L: int):
    """The identity operator as a bond-dimension-1 MPO."""
    return [lo.I4.reshape(1, 1, 4, 4).copy() for _ in range(L)]


def mpo_to_dense(Ws) -> np.ndarray:
    """Contract an MPO to the dense 4^L x 4^L matrix (site 1 is the most
    significant digit of the index).  Tiny chains only."""
    L = len(Ws)
    # cur[a, S, T] accumulates operator strings over sites 1..k
    cur = Ws[0][0]                      # (w1, 4, 4)
    for k in range(1, L):
        W = Ws[k]
        cur = np.einsum("aST,abst->bSsTt", cur, W)
        b, S, s, T, tt = cur.shape
        cur = cur.reshape(b, S * s, T * tt)
    return cur[0]


def _fermion_factors(K: int, ops):
    """Site factors of a product of spin-orbital creators/annihilators.

    ``ops`` lists (site p 1-based, spin 0=alpha 1=beta, dagger) in operator
    order, leftmost first.  Under the Jordan-Wigner mapping of Sec. 2.1 one
    operator at site p is F on every earlier site, its local matrix at p and
    the identity after p (F the site parity), so the product is the site-wise
    product of these factors in operator order.  Returns K 4x4 matrices, or
    None if one of them vanishes."""
    local = {(0, 1): lo.CDAG_A, (1, 1): lo.CDAG_B, (0, 0): lo.C_A, (1, 0): lo.C_B}
    out = []
    for j in range(1, K + 1):
        m = lo.I4
        for (p, spin, dag) in ops:
            if j < p:
                m = m @ lo.PARITY
            elif j == p:
                m = m @ local[(spin, dag)]
        m = m + 0.0                       # no negative zeros in the keys below
        if not m.any():
            return None
        out.append(m)
    return out


def abinitio_terms(h: np.ndarray, eri: np.ndarray):
    """The second-quantised Hamiltonian of Eq. [sqH] for real orbitals as a
    list of (coefficient, operator product):
        sum_pq h_pq sum_s a+_ps a_qs
      + 1/2 sum_pqrs (pq|rs) sum_st a+_ps a+_rt a_st a_qs
    (chemists' notation; no core energy).  Sites are 1-based."""
    K = h.shape[0]
    terms = []
    for p in range(K):
        for q in range(K):
            if h[p, q] != 0.0:
                for s in (0, 1):
                    terms.append((h[p, q], ((p + 1, s, 1), (q + 1, s, 0))))
    for p in range(K):
        for q in range(K):
            for r in range(K):
                for s_ in range(K):
                    v = eri[p, q, r, s_]
                    if v == 0.0:
                        continue
                    for a in (0, 1):
                        for b in (0, 1):
                            terms.append((0.5 * v, ((p + 1, a, 1), (r + 1, b, 1), (s_ + 1, b, 0),
                                                    (q + 1, a, 0))))
    return terms


def terms_mpo(K: int, terms):
    """MPO of a sum of even fermionic operator products, built as the
    automaton of the right-vector recursion of Sec. 2.1: at bond k a product
    whose support [p_min, p_max] straddles the bond sits in the channel named
    by its remaining site factors on k+1..p_max (products with the same
    remainder share it), its coefficient enters at p_min, channel 0 carries
    the complete operator of the sites to the right and the last channel the
    identity.  Even products carry no string outside their support."""
    prods = []
    for coef, ops in terms:
        f = _fermion_factors(K, ops)
        if f is None:
            continue
        sup = [j for j in range(K) if not np.array_equal(f[j], lo.I4)]
        if not sup:
            raise ValueError("a constant term is not supported")
        prods.append((coef, f, sup[0], sup[-1]))

    def key(f, k, last):
        return tuple(f[j].tobytes() for j in range(k, last + 1))

    # channel index of every remainder at every inner bond k (after site k+1,
    # 0-based sites): 1..n, 0 = complete operator, n+1 = identity
    chans = [dict() for _ in range(K + 1)]
    for coef, f, lo_, hi in prods:
        for k in range(lo_, hi):            # bond after 0-based site k
            kk = key(f, k + 1, hi)
            if kk not in chans[k + 1]:
                chans[k + 1][kk] = len(chans[k + 1]) + 1
    # untrimmed widths: 2 at the outer bonds (trimmed to 1 at the end)
    wf = [2] + [len(chans[k]) + 2 for k in range(1, K)] + [2]
    Ws = [np.zeros((wf[k], wf[k + 1], 4, 4)) for k in range(K)]
    for k in range(K):
        Ws[k][0, 0] = lo.I4
        Ws[k][-1, -1] = lo.I4
    for coef, f, lo_, hi in prods:
        for k in range(lo_, hi + 1):
            a = 0 if k == lo_ else chans[k][key(f, k, hi)]
            b = wf[k + 1] - 1 if k == hi else chans[k + 1][key(f, k + 1, hi)]
            if k == lo_:
                Ws[k][a, b] += coef * f[k]
            else:
                Ws[k][a, b] = f[k]
    return _trim(Ws)


def abinitio_mpo(h: np.ndarray, eri: np.ndarray):
    """The ab-initio Hamiltonian (Eq. [sqH], chemists' integrals) as an MPO;
    see :func:`terms_mpo` for the construction."""
    return terms_mpo(h.shape[0], abinitio_terms(h, eri))


def abinitio_component_mpo(h: np.ndarray, eri: np.ndarray, p: int):
    """Energy component H_p (orbital p, 1-based) for the fragment energies
    e_p of Sec. 2.4: the terms of :func:`abinitio_terms` whose leftmost
    creator acts on orbital p,
        H_p = sum_q h_pq E_pq + 1/2 sum_qrs (pq|rs) sum_st a+_ps a+_rt a_st a_qs,
    so that sum_p H_p = H and both spin orbitals of p lie in H_p."""
    terms = [(c, ops) for (c, ops) in abinitio_terms(h, eri) if ops[0][0] == p]
    return terms_mpo(h.shape[0], terms)


def hubbard_integrals(L: int, t: float, U: float):
    """The open Hubbard chain as integrals of Eq. [sqH]: h = -t between
    nearest neighbours, (pp|pp) = U, every other integral zero."""
    h = np.zeros((L, L))
    for q in range(L - 1):
        h[q, q + 1] = h[q + 1, q] = -t
    eri = np.zeros((L, L, L, L))
    for q in range(L):
        eri[q, q, q, q] = U
    return h, eri

