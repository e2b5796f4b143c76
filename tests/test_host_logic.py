"""Host-side logic of the library (no GPU): exported symbols, quadrature,
MPO builders, the subspace eigensolver and argument validation, each
checked against the oracle or numpy."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1703_04789_amd as sp
import workloads as W
from oracle import mpo, quadrature as q

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "spmps.h")


def _declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:int|const char\*)\s+(sp_\w+)\s*\(", src, flags=re.M)))


def test_library_exports_every_declared_symbol():
    L = sp.lib()
    names = _declared()
    assert len(names) >= 18
    for n in names:
        assert hasattr(L, n), n
    assert sorted(sp.EXPORTS) == names


@pytest.mark.parametrize("G,twoS,twoM", [(1, 0, 0), (5, 0, 0), (9, 2, 0), (9, 0, 0), (11, 3, 1), (7, 4, -2),
                                         (13, 4, 0), (3, 1, -1)])
def test_quadrature_matches_oracle(G, twoS, twoM):
    x, w, c = sp.quadrature(G, twoS, twoM)
    t = q.projector_quadrature(G, twoS, twoM)
    np.testing.assert_allclose(x, t["x"], atol=1e-15)
    np.testing.assert_allclose(w, t["w"], atol=2e-15)
    np.testing.assert_allclose(c, t["coef"], atol=2e-15)


@pytest.mark.parametrize("N,K,twoS,twoM", [(16, 16, 0, 0), (8, 8, 0, 0), (32, 32, 2, 0), (14, 10, 0, 0),
                                           (5, 5, 1, 1), (48, 48, 4, 0)])
def test_exact_points_matches_oracle(N, K, twoS, twoM):
    assert sp.exact_points(N, K, twoS, twoM) == q.exact_point_count(N, K, twoS, twoM)


@pytest.mark.parametrize("L", [1, 2, 3, 7])
def test_mpo_builders_match_oracle(L):
    for (mine, ref) in ((sp.mpo_hubbard(L, 1.3, 3.7), mpo.hubbard_mpo(L, 1.3, 3.7)),
                        (sp.mpo_s2(L), mpo.s2_mpo(L)), (sp.mpo_identity(L), mpo.identity_mpo(L))):
        w, data = mine
        assert list(w) == [1] + [r.shape[1] for r in ref[:-1]] + [1]
        np.testing.assert_array_equal(data, np.concatenate([r.ravel() for r in ref]))


@pytest.mark.parametrize("n", [1, 2, 5, 17, 32, 64])
def test_small_eigh_matches_numpy(n):
    rng = np.random.default_rng(n)
    A = rng.standard_normal((n, n))
    A = A + A.T
    ev, V = sp.small_eigh(A)
    np.testing.assert_allclose(ev, np.linalg.eigvalsh(A), atol=1e-12 * max(1, np.abs(ev).max()))
    np.testing.assert_allclose(V @ np.diag(ev) @ V.T, A, atol=1e-12 * n)
    np.testing.assert_allclose(V.T @ V, np.eye(n), atol=1e-13 * n)


def test_small_eigh_degenerate_and_singular():
    rng = np.random.default_rng(1)
    B = rng.standard_normal((20, 4))
    A = B @ B.T
    ev, V = sp.small_eigh(A)
    assert np.abs(ev[:16]).max() < 1e-12
    np.testing.assert_allclose(V @ np.diag(ev) @ V.T, A, atol=1e-12)
    ev, V = sp.small_eigh(np.diag([2.0, 1.0, 1.0, 3.0]))
    np.testing.assert_allclose(ev, [1, 1, 2, 3])


def _canonical_lowest(H, N, drop=1e-10):
    """The subspace solve written out with numpy: eigendecompose N, keep the
    eigenvalues above drop * max, reduce H and take its lowest eigenpair."""
    lam, U = np.linalg.eigh(N)
    sel = lam > drop * lam.max()
    X = U[:, sel] / np.sqrt(lam[sel])[None, :]
    mu, C = np.linalg.eigh(X.T @ H @ X)
    return mu[0], X @ C[:, 0], int(sel.sum())


@pytest.mark.parametrize("m", [1, 2, 3, 8, 17, 32])
def test_small_gen_lowest_full_rank(m):
    rng = np.random.default_rng(10 + m)
    A = rng.standard_normal((m, m))
    H = A + A.T
    B = rng.standard_normal((m, m))
    N = B @ B.T + 0.1 * np.eye(m)
    theta, a, rank = sp.small_gen_lowest(H, N)
    t_ref, a_ref, r_ref = _canonical_lowest(H, N)
    assert rank == r_ref == m
    assert abs(theta - t_ref) < 1e-11 * max(1.0, abs(t_ref))
    assert abs(a @ N @ a - 1.0) < 1e-11
    np.testing.assert_allclose(H @ a, theta * (N @ a), atol=1e-9 * max(1.0, np.abs(H).max()))
    np.testing.assert_allclose(abs(a @ N @ a_ref), 1.0, atol=1e-9)


@pytest.mark.parametrize("m,r", [(6, 3), (20, 12), (32, 31)])
def test_small_gen_lowest_singular_metric(m, r):
    # N of rank r: the solve must stay in range(N), like the reference
    rng = np.random.default_rng(100 + m)
    B = rng.standard_normal((m, r))
    N = B @ B.T
    A = rng.standard_normal((m, m))
    H = A + A.T
    theta, a, rank = sp.small_gen_lowest(H, N)
    t_ref, a_ref, r_ref = _canonical_lowest(H, N)
    assert rank == r_ref == r
    assert abs(theta - t_ref) < 1e-9 * max(1.0, abs(t_ref))
    P = B @ np.linalg.pinv(B)  # projector on range(N)
    np.testing.assert_allclose(P @ a, a, atol=1e-8 * np.abs(a).max())


def test_small_gen_lowest_rejects_zero_metric():
    with pytest.raises(sp.SpError) as e:
        sp.small_gen_lowest(np.eye(3), np.zeros((3, 3)))
    assert e.value.code == -2


class _Tab:
    def __init__(self, L, N, twoM, bonds):
        self.L, self.N, self.twoM, self.bonds = L, N, twoM, bonds

    def flat(self):
        return W.BlockTable(self.L, self.N, self.twoM, self.bonds).flat()


def _init_rc(table, twoS, G, mpo_=None, N=None, path=sp.SP_PATH_TILED, precision=sp.SP_FP64):
    """sp_init_mps return code for host-rejected inputs (never reaches HIP)."""
    nsec, sn, s2m, sdim = (np.ascontiguousarray(a, dtype=np.int32) for a in table.flat())
    w, data = mpo_ or sp.mpo_hubbard(table.L, 1.0, 4.0)
    w = np.ascontiguousarray(w, dtype=np.int32)
    prob = sp._Problem(table.L, 4, table.N if N is None else N, twoS, table.twoM, G, precision, path)
    m = sp._Mpo(sp._iptr(w), sp._dptr(data))
    bt = sp._BlockTable(sp._iptr(nsec), sp._iptr(sn), sp._iptr(s2m), sp._iptr(sdim))
    blocks = np.zeros(max(1, W.BlockTable(table.L, table.N, table.twoM, table.bonds).total_size()))
    h = ctypes.c_void_p()
    rc = sp.lib().sp_init_mps(ctypes.byref(prob), ctypes.byref(m), ctypes.byref(bt), sp._dptr(blocks), None,
                              ctypes.byref(h))
    return rc, sp.lib().sp_last_error().decode()


def test_init_rejects_bad_spin_parity_and_range():
    tab = W.make_block_table(4, 4, 0, 8)
    assert _init_rc(tab, 1, 3)[0] == sp.SP_EINVAL            # N + 2S odd
    assert _init_rc(tab, 10, 3)[0] == sp.SP_EINVAL           # S above the largest seniority
    assert _init_rc(tab, 0, 0)[0] == sp.SP_EINVAL            # G < 1
    tab2 = W.make_block_table(4, 4, 2, 8)
    assert _init_rc(tab2, 0, 3)[0] == sp.SP_EINVAL           # |M| > S


def test_init_precision_modes():
    """SP_FP32 and SP_BF16X3 need the tiled path; unknown modes are rejected
    on the host."""
    import torch
    tab = W.make_block_table(4, 4, 0, 8)
    assert _init_rc(tab, 0, 3, precision=7)[0] == sp.SP_EINVAL
    for prec in (sp.SP_FP32, sp.SP_BF16X3):
        rc, msg = _init_rc(tab, 0, 3, precision=prec, path=sp.SP_PATH_PLAIN)
        assert rc == sp.SP_EINVAL and "tiled" in msg
        if not torch.cuda.is_available():  # accepted: the call then stops at the first HIP call
            assert _init_rc(tab, 0, 3, precision=prec)[0] == sp.SP_EHIP


def test_init_rejects_inconsistent_block_table():
    tab = W.make_block_table(4, 4, 0, 8)
    bonds = [list(b) for b in tab.bonds]
    n, m, d = bonds[2][0]
    bonds[2][0] = (n, m, d + 50)                            # wider than its support
    rc, msg = _init_rc(_Tab(4, 4, 0, bonds), 0, 3)
    assert rc == sp.SP_EINVAL and "wider" in msg
    bonds = [list(b) for b in tab.bonds]
    bonds[2] = bonds[2][::-1]                               # unsorted
    rc, msg = _init_rc(_Tab(4, 4, 0, bonds), 0, 3)
    assert rc == sp.SP_EINVAL and "sorted" in msg


def test_init_rejects_non_triangular_mpo():
    tab = W.make_block_table(3, 3, 1, 8)
    w, data = sp.mpo_hubbard(3, 1.0, 4.0)
    off = 1 * 6 * 16              # site 2 starts after site 1 (1 x 6 x 16 doubles)
    bad = data.copy()
    bad[off + ((5 * 6 + 5) * 4 + 0) * 4 + 0] = 2.0   # W[2]_{5,5} no longer the identity
    rc, msg = _init_rc(tab, 1, 3, mpo_=(w, bad))
    assert rc == sp.SP_EINVAL and "identity" in msg


@pytest.mark.parametrize("wl", [W.hubbard_small(), W.hubbard_bench(0), W.hubbard_bench(2)],
                         ids=lambda w: w.name)
def test_init_plans_pass_host_validation(wl):
    """All per-site task lists of the workload are built and bounds-checked
    on the host; without a GPU the call then stops at the first HIP call."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present: covered by the GPU tests")
    for path in (sp.SP_PATH_TILED, sp.SP_PATH_PLAIN):
        rc, msg = _init_rc(wl.table(), wl.twoS, wl.G, mpo_=sp.mpo_hubbard(wl.L, wl.t, wl.U), path=path)
        assert rc == sp.SP_EHIP, (path, msg)


def test_init_plans_pass_host_validation_odd_cases():
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present: covered by the GPU tests")
    for (L, N, twoM, D, twoS, G) in [(6, 5, 1, 12, 1, 3), (7, 6, 2, 20, 4, 4), (1, 2, 0, 4, 0, 1),
                                     (2, 2, 0, 4, 0, 2), (12, 10, 0, 128, 2, 5)]:
        tab = W.make_block_table(L, N, twoM, D)
        rc, msg = _init_rc(tab, twoS, G)
        assert rc == sp.SP_EHIP, (L, N, msg)
    tab = W.make_block_table(6, 6, 0, 20)
    rc, msg = _init_rc(tab, 2, 4, mpo_=sp.mpo_s2(6))
    assert rc == sp.SP_EHIP, msg


def _mpo_sites(w, data):
    out, pos = [], 0
    for k in range(1, len(w)):
        n = int(w[k - 1]) * int(w[k]) * 16
        out.append(data[pos:pos + n].reshape(int(w[k - 1]), int(w[k]), 4, 4))
        pos += n
    return out


@pytest.mark.parametrize("K", [2, 3, 4])
def test_abinitio_mpo_matches_exact_hamiltonian(K):
    from oracle import ed
    h, eri = W.abinitio_integrals(K, seed=11)
    w, data = sp.mpo_abinitio(h, eri)
    Hd = mpo.mpo_to_dense(_mpo_sites(w, data))
    for N in range(1, 2 * K):
        for twoM in range(-N, N + 1, 2):
            st = ed.sector_states(K, N, twoM)
            if len(st):
                np.testing.assert_allclose(Hd[np.ix_(st, st)], ed.abinitio_hamiltonian(h, eri, st).toarray(),
                                           atol=1e-12)


def test_abinitio_mpo_matches_oracle_mpo_and_is_compact():
    K = 5
    h, eri = W.abinitio_integrals(K, seed=4)
    w, data = sp.mpo_abinitio(h, eri)
    ref = mpo.abinitio_mpo(h, eri)
    np.testing.assert_allclose(mpo.mpo_to_dense(_mpo_sites(w, data)), mpo.mpo_to_dense(ref), atol=1e-12)
    # partial products named by at most two operators: O(K^2) channels, far
    # fewer than the oracle's automaton that names whole remainders
    assert max(w) < max(r.shape[1] for r in ref[:-1]) / 10
    w16, _ = sp.mpo_abinitio(*W.abinitio_integrals(16, seed=4))
    assert w16[0] == w16[16] == 1 and max(w16) <= 3 * 16 * 16


def test_abinitio_mpo_rejects_bad_sizes():
    with pytest.raises(sp.SpError):
        sp.mpo_abinitio(np.zeros((1, 1)), np.zeros((1, 1, 1, 1)))


@pytest.mark.parametrize("K,D,G", [(6, 32, 7), (8, 64, 9), (12, 128, 11)])
def test_init_abinitio_plans_pass_host_validation(K, D, G):
    """Wide MPOs: sites whose particle-number blocks do not fit the fused
    kernel get the block-product lists; every list is bounds-checked."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present: covered by the GPU tests")
    tab = W.make_block_table(K, K, 0, D)
    rc, msg = _init_rc(tab, 0, G, mpo_=sp.mpo_abinitio(*W.abinitio_integrals(K, seed=4)))
    assert rc == sp.SP_EHIP, msg
