"""The device-resident Davidson iteration: its FP64 subspace solve in one
GPU work-group against the host solve and the eigendecomposition formula,
and whole sweeps through it against the oracle and the host-driven solver.

The subspace problem (Sec. 2.3, Eq. [geproblem] in the search space): the
lowest pair of the symmetric pencil (H, N) within the span of the
eigenvectors of N above drop x lambda_max (canonical orthogonalisation).
Tolerances: Ritz values 1e-11 relative, Ritz coefficient vectors 1e-9
(up to the sign of the eigenvector); sweep energies 1e-8 (the FP64 target).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from gpu_util import make_pair  # noqa: E402

import paper_1703_04789_amd as sp  # noqa: E402
from oracle import mps as omps  # noqa: E402

pytestmark = pytest.mark.gpu


def _pencil(m, r, seed, cond=1.0):
    rng = np.random.default_rng(seed)
    H = rng.standard_normal((m, m))
    H = H + H.T
    B = rng.standard_normal((m, r)) * np.geomspace(1.0, cond, r)
    return H, B @ B.T


def _reference(H, N, drop):
    """The formula: eigenvectors of N above drop x max, X = U / sqrt(ev),
    lowest eigenpairs of X^T H X; returns Ritz values and m x rank vectors."""
    ev, U = np.linalg.eigh(0.5 * (N + N.T))
    keep = ev > drop * ev[-1]
    X = U[:, keep] / np.sqrt(ev[keep])
    mu, C = np.linalg.eigh(X.T @ (0.5 * (H + H.T)) @ X)
    return mu, X @ C


def _same_up_to_sign(a, b):
    s = 1.0 if np.dot(a, b) >= 0 else -1.0
    return np.abs(a - s * b).max() / np.abs(b).max()


@pytest.mark.parametrize("m", [1, 2, 5, 17, 32, 47])
def test_device_solve_full_rank(m):
    H, N = _pencil(m, m, 100 + m)
    theta, a, rank = sp.small_gen_lowest_gpu(H, N)
    th_h, a_h, rank_h = sp.small_gen_lowest(H, N)
    mu, Xc = _reference(H, N, 1e-10)
    assert rank == rank_h == m
    assert abs(theta - mu[0]) < 1e-11 * max(1.0, abs(mu[0]))
    assert abs(theta - th_h) < 1e-11 * max(1.0, abs(th_h))
    assert _same_up_to_sign(a, Xc[:, 0]) < 1e-9
    assert abs(a @ N @ a - 1.0) < 1e-10


@pytest.mark.parametrize("m,r", [(6, 3), (20, 13), (33, 32), (40, 8)])
def test_device_solve_singular_metric(m, r):
    # rank-deficient metric (the singular pencil of the projected problem):
    # the dropped directions carry no Ritz vector
    # (metric eigenvalues from 1 down to 1e-6: the kept basis X = U / sqrt(ev)
    # amplifies rounding by up to 1e3, so the host solve itself reaches the
    # formula only to about 2e-9 here; both sides are held to 1e-8)
    H, N = _pencil(m, r, 200 + m, cond=1e-3)
    theta, a, rank = sp.small_gen_lowest_gpu(H, N)
    th_h, a_h, rank_h = sp.small_gen_lowest(H, N)
    mu, Xc = _reference(H, N, 1e-10)
    assert rank == rank_h == Xc.shape[1] == r
    assert abs(theta - mu[0]) < 1e-8 * max(1.0, abs(mu[0]))
    assert abs(th_h - mu[0]) < 1e-8 * max(1.0, abs(mu[0]))
    assert _same_up_to_sign(a, Xc[:, 0]) < 1e-7


@pytest.mark.parametrize("m,keep", [(12, 4), (32, 8), (47, 16)])
def test_device_restart_rotation(m, keep):
    # a restart keeps the `keep` lowest Ritz vectors, orthonormalised by
    # modified Gram-Schmidt, and rotates the projected pencil onto them
    H, N = _pencil(m, m, 300 + m)
    H0, N0 = H.copy(), N.copy()
    theta, a, nk, Q, Hr, Nr = sp.small_gen_lowest_gpu(H, N, keep=keep)
    mu, Xc = _reference(H0, N0, 1e-10)
    assert nk == keep and abs(theta - mu[0]) < 1e-11 * max(1.0, abs(mu[0]))
    Qr, _ = np.linalg.qr(Xc[:, :keep])  # Gram-Schmidt of the same columns, up to signs
    D = np.sign(np.diag(Q.T @ Qr))
    assert np.abs(Q - Qr * D).max() < 1e-9
    assert np.abs(Q.T @ Q - np.eye(keep)).max() < 1e-12
    assert np.abs(Hr - Q.T @ H0 @ Q).max() < 1e-10 * np.abs(H0).max()
    assert np.abs(Nr - Q.T @ N0 @ Q).max() < 1e-10 * np.abs(N0).max()


STABLE = [  # (L, N, 2M, D, 2S, G): local problems of at most 42 elements,
    # trajectories moved by < 1e-12 under a 1e-13 change of the start
    (4, 4, 0, 16, 0, 3),
    (5, 5, 1, 8, 1, 3),
    (6, 6, 0, 8, 2, 4),
    (6, 6, 0, 8, 0, 4),
]
EXACT = dict(max_sub=47, max_iter=200)


@pytest.mark.parametrize("case", STABLE)
def test_device_sweeps_match_oracle(case):
    # every local problem fits the search space, so each solve is exact and
    # the whole trajectory is fixed by the input
    tab, gpu, orc = make_pair(*case)
    rc, steps = gpu.sweep(2, solver="device", **EXACT)
    ref = omps.sweep(orc, 2, **EXACT)
    assert rc == sp.SP_OK and len(steps) == len(ref)
    for a, b in zip(steps, ref):
        assert (a["site"], a["dir"]) == (b["site"], b["dir"])
        assert abs(a["theta"] - b["theta"]) < 1e-8, (a, b)
    E, _ = gpu.energy()
    assert abs(E - ref[-1]["theta"]) < 1e-8


def test_device_and_host_solves_agree():
    for case in STABLE:
        _, dev, _ = make_pair(*case, oracle=False)
        _, host, _ = make_pair(*case, oracle=False)
        _, sd = dev.sweep(2, solver="device", **EXACT)
        _, sh = host.sweep(2, solver="host", **EXACT)
        assert max(abs(a["theta"] - b["theta"]) for a, b in zip(sd, sh)) < 1e-9


def test_device_and_host_batches_agree():
    # the same batch through both drivers (device resident is the default
    # for batches): step energies equal to rounding
    pairs = [make_pair(*c, oracle=False) for c in STABLE]
    _, dev = sp.sweep_batch([g for _, g, _ in pairs], 2, **EXACT)
    pairs = [make_pair(*c, oracle=False) for c in STABLE]
    _, host = sp.sweep_batch([g for _, g, _ in pairs], 2, solver="host", **EXACT)
    for a, b in zip(dev, host):
        assert max(abs(x["theta"] - y["theta"]) for x, y in zip(a, b)) < 1e-9


def test_solver_option_is_checked():
    _, gpu, _ = make_pair(*STABLE[0], oracle=False)
    with pytest.raises(KeyError):
        gpu.sweep(1, solver="gpu")


def test_device_batch_matches_oracle():
    # the four states in one batch: one graph per round covers all of them
    pairs = [make_pair(*c) for c in STABLE]
    rc, batch = sp.sweep_batch([g for _, g, _ in pairs], 2, solver="device", **EXACT)
    assert rc == sp.SP_OK
    for (tab, gpu, orc), steps in zip(pairs, batch):
        ref = omps.sweep(orc, 2, **EXACT)
        assert max(abs(a["theta"] - b["theta"]) for a, b in zip(steps, ref)) < 1e-8


def test_device_restarts_reach_ed():
    # small search space (8 vectors, restart to 4) on a full-bond-dimension
    # chain: every restart runs on the device, and the energy reaches ED
    from oracle import quadrature as oq
    L, twoS = 6, 0
    G = oq.exact_point_count(L, L, twoS)
    _, gpu, _ = make_pair(L, L, 0, 64, twoS, G, oracle=False)
    rc, steps = gpu.sweep(3, max_sub=8, keep=4, max_iter=2000, tol=1e-10, solver="device")
    assert abs(steps[-1]["theta"] - (-3.092565319505379)) < 1e-9
    assert max(s["iters"] for s in steps) > 8  # restarts happened
