"""Occupation-number states (one or two determinants) as block-table MPS
inputs: test input construction only, no arithmetic of the method."""
import numpy as np

import workloads as W

SIGMA = {(0, 0): 0, (0, 1): 1, (1, 0): 2, (1, 1): 3}  # (n_alpha, n_beta) -> local state
QN = [(0, 0), (1, -1), (1, 1), (2, 0)]                # (N, 2M) change of each local state


def sigmas(K, occ):
    """Local states of the determinant with spin orbitals occ ((p, s), p 0-based)."""
    na = np.zeros(K, dtype=int)
    nb = np.zeros(K, dtype=int)
    for p, s in occ:
        (na if s == 0 else nb)[p] += 1
    return [SIGMA[(int(na[p]), int(nb[p]))] for p in range(K)]


def product_state(terms, K, N, twoM=0):
    """Block table and packed blocks of sum_t c_t |occ_t> for one or two
    determinants with the same particle number and M, as an MPS whose bonds
    carry one state per distinct path: shared before the first and after the
    last site where the determinants differ, one per determinant between."""
    sig = [sigmas(K, o) for _, o in terms]
    diff = [k for k in range(K) if len({s[k] for s in sig}) > 1]
    d0, d1 = (diff[0], diff[-1]) if diff else (K, K)
    qn = []
    for s in sig:
        n = m = 0
        path = [(0, 0)]
        for k in range(K):
            n += QN[s[k]][0]
            m += QN[s[k]][1]
            path.append((n, m))
        qn.append(path)
    if any(path[-1] != (N, twoM) for path in qn):
        raise ValueError("every determinant must have N electrons and the given 2M")
    # state of determinant t at bond b: (sector key, index within the sector)
    bonds, state = [], []
    for b in range(K + 1):
        split = d0 < b <= d1
        keys, st = {}, []
        for t in range(len(terms)):
            key = qn[t][b]
            idx = keys.get(key, 0) if split else 0
            keys[key] = idx + 1 if split else 1
            st.append((key, idx))
        bonds.append(sorted((n, m, d) for (n, m), d in keys.items()))
        state.append(st)
    tab = W.BlockTable(K, N, twoM, bonds)
    blocks = []
    for k in range(1, K + 1):
        left, right = bonds[k - 1], bonds[k]
        loff, roff, o = {}, {}, 0
        for (n, m, d) in left:
            loff[(n, m)] = o
            o += d
        o = 0
        for (n, m, d) in right:
            roff[(n, m)] = o
            o += d
        A = np.zeros((4, sum(x[2] for x in left), sum(x[2] for x in right)))
        for t, (c, _) in enumerate(terms):
            (lk, li), (rk, ri) = state[k - 1][t], state[k][t]
            A[sig[t][k - 1], loff[lk] + li, roff[rk] + ri] = c if k - 1 == d0 else 1.0
        for (ia, s, ib, r, cc) in tab.site_blocks(k):
            lo, ro = loff[left[ia][:2]], roff[right[ib][:2]]
            blocks.append(A[s, lo:lo + r, ro:ro + cc].ravel())
    return tab, np.concatenate(blocks)
