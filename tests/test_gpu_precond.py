"""Learned Davidson preconditioner on the HIP path against its FP64 reference
(oracle.precond and the oracle's Davidson hook).

Tolerances: model outputs 1e-6 relative to the largest output (FP64
arithmetic on FP32 weights and features, FP32 result); Adam steps 2e-7
absolute on the weights (FP32 storage after each step); recorded features
1e-5 and targets 1e-4 relative (FP32 storage; compared only where the
residual and the exact correction are not yet at the rounding level of the
trajectory: over the vector for the vector scope, over the N-block for the
per-N-block scope); sweep energies 1e-8 (converged local solves)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from gpu_util import make_pair  # noqa: E402

import paper_1703_04789_amd as sp  # noqa: E402
import workloads as W  # noqa: E402
from oracle import mps as omps, precond as pre  # noqa: E402

pytestmark = pytest.mark.gpu


def _params(H=64, seed=0):
    p = W.mlp_init(H, seed)
    rng = np.random.default_rng(seed + 7)
    p["b1"] = (0.1 * rng.standard_normal(H)).astype(np.float32)
    p["b2"] = np.float32(0.05)
    return p


def _as64(p):
    return {k: np.asarray(v, np.float64) if np.ndim(v) else float(v) for k, v in p.items()}


def test_forward_matches_reference():
    p = _params(256)
    m = sp.MLP(p)
    F = np.random.default_rng(1).standard_normal((5000, 5)).astype(np.float32)
    y = m.forward(torch.tensor(F, device="cuda")).cpu().numpy()
    ref = pre.forward(_as64(p), F.astype(np.float64))
    assert np.abs(y - ref).max() < 1e-6 * np.abs(ref).max()


def test_train_steps_match_adam_reference():
    p = _params(128, 3)
    m = sp.MLP(p)
    rng = np.random.default_rng(2)
    F = rng.standard_normal((6000, 5)).astype(np.float32)
    Y = rng.standard_normal(6000).astype(np.float32)
    Fd, Yd = torch.tensor(F, device="cuda"), torch.tensor(Y, device="cuda")
    ref, state = _as64(p), {}
    for step in range(3):
        loss = m.train_step(Fd, Yd, 1e-3)
        lref, g = pre.loss_and_grads(ref, F.astype(np.float64), Y.astype(np.float64))
        assert abs(loss - lref) < 1e-9 * lref, (step, loss, lref)
        ref = pre.adam_step(ref, g, state, 1e-3)
        # the library keeps FP32 weights: compare after the same rounding
        ref = {k: (np.asarray(v, np.float32).astype(np.float64) if np.ndim(v) else float(np.float32(v)))
               for k, v in ref.items()}
        got = m.params()
        for k in ("W1", "b1", "w2"):
            assert np.abs(np.asarray(got[k], np.float64) - ref[k]).max() < 2e-7, (step, k)
        assert abs(got["b2"] - ref["b2"]) < 2e-7


def test_recorded_pairs_match_the_oracle():
    # one sweep of the L=8, D=16, G=5 workload with recording on both sides
    wl = W.hubbard_small()
    tab, gpu, orc = make_pair(wl.L, wl.N, wl.twoM, wl.D, wl.twoS, wl.G, U=wl.U, seed=wl.seed)
    rec = sp.MLP(_params(), capacity=2_000_000)
    gpu.set_precond(record=rec)
    gpu.sweep(1, max_sub=32, max_iter=64)
    pairs = []
    omps.sweep(orc, 1, max_sub=32, max_iter=64, pairs=pairs)
    F, Y = rec.dataset()
    sizes = [len(p[1]) for p in pairs]
    assert F.shape[0] == sum(sizes), (F.shape, sum(sizes))

    def packed(k, v):  # the oracle's element order -> the library's packed order
        m = orc.mps.mask[k - 1]
        d = np.zeros(m.size)
        d[np.flatnonzero(m.ravel())] = v
        return orc.mps.site_packed(k, d.reshape(m.shape))
    off, checked = 0, 0
    for (k, r, th, x, xs, dh, dn), n in zip(pairs, sizes):
        r, x, xs, dh, dn = (packed(k, v) for v in (r, x, xs, dh, dn))
        e_raw = xs / float(x @ xs) - x
        # late iterations: the residual and the exact correction are at the
        # rounding level of the two trajectories and are not compared
        if np.linalg.norm(r) > 1e-4 and np.sqrt(np.mean(e_raw ** 2)) > 1e-4:
            fr = pre.features(r, dh, dn, th)
            blk = F[off: off + n].astype(np.float64)
            assert np.abs(blk - fr).max() < 1e-5 * max(1.0, np.abs(fr).max())
            yr = pre.target(r, x, xs)
            assert np.abs(Y[off: off + n] - yr).max() < 1e-4 * max(1.0, np.abs(yr).max())
            checked += 1
        off += n
    assert checked >= 10


def test_learned_sweep_matches_the_oracle_with_the_same_weights():
    # a briefly trained model drives both solvers; the corrections agree to
    # rounding, so do the trajectories
    wl = W.hubbard_small()
    tab, gpu, orc = make_pair(wl.L, wl.N, wl.twoM, wl.D, wl.twoS, wl.G, U=wl.U, seed=wl.seed)
    rec = sp.MLP(_params(64, 5), capacity=2_000_000)
    gpu.set_precond(record=rec)
    gpu.sweep(1)
    rec.train(3, 4096, 3e-3)
    model = rec.params()
    _, g2, o2 = make_pair(wl.L, wl.N, wl.twoM, wl.D, wl.twoS, wl.G, U=wl.U, seed=wl.seed + 1)
    g2.set_precond(use=rec)
    rc, steps = g2.sweep(2, max_sub=128, max_iter=200)
    ref = omps.sweep(o2, 2, max_sub=128, max_iter=200, model=_as64(model))
    print("[precond] iterations per step (learned):", [s["iters"] for s in steps], flush=True)
    assert all(s["converged"] for s in steps)
    assert [s["iters"] for s in steps] == [s["iters"] for s in ref]
    assert max(abs(a["theta"] - b["theta"]) for a, b in zip(steps, ref)) < 1e-8


def test_nblock_recorded_pairs_match_the_oracle():
    # per-N-block scope: block root mean squares in the features and the
    # targets; compared on the blocks whose residual and exact correction
    # are above the rounding level of the two trajectories
    wl = W.hubbard_small()
    tab, gpu, orc = make_pair(wl.L, wl.N, wl.twoM, wl.D, wl.twoS, wl.G, U=wl.U, seed=wl.seed)
    rec = sp.MLP(_params(), capacity=2_000_000, scope="nblock")
    gpu.set_precond(record=rec)
    gpu.sweep(1, max_sub=32, max_iter=64)
    pairs = []
    omps.sweep(orc, 1, max_sub=32, max_iter=64, pairs=pairs)
    F, Y = rec.dataset()
    sizes = [len(p[1]) for p in pairs]
    assert F.shape[0] == sum(sizes), (F.shape, sum(sizes))

    def packed(k, v):
        m = orc.mps.mask[k - 1]
        d = np.zeros(m.size)
        d[np.flatnonzero(m.ravel())] = v
        return orc.mps.site_packed(k, d.reshape(m.shape))
    off, checked = 0, 0
    for (k, r, th, x, xs, dh, dn), n in zip(pairs, sizes):
        grp = np.rint(packed(k, orc.mps.nblock_labels(k).astype(float))).astype(int)
        r, x, xs, dh, dn = (packed(k, v) for v in (r, x, xs, dh, dn))
        e_raw = xs / float(x @ xs) - x
        ok = (pre.rms_over(r, grp) > 1e-6) & (pre.rms_over(e_raw, grp) > 1e-6)
        if ok.sum() > n // 2:
            fr = pre.features(r, dh, dn, th, groups=grp)
            blk = F[off: off + n].astype(np.float64)
            assert np.abs(blk[ok] - fr[ok]).max() < 1e-5 * max(1.0, np.abs(fr[ok]).max())
            yr = pre.target(r, x, xs, groups=grp)
            assert np.abs(Y[off: off + n][ok] - yr[ok]).max() < 1e-4 * max(1.0, np.abs(yr[ok]).max())
            checked += 1
        off += n
    assert checked >= 10


def test_nblock_learned_sweep_matches_the_oracle_with_the_same_weights():
    wl = W.hubbard_small()
    tab, gpu, orc = make_pair(wl.L, wl.N, wl.twoM, wl.D, wl.twoS, wl.G, U=wl.U, seed=wl.seed)
    rec = sp.MLP(_params(64, 5), capacity=2_000_000, scope="nblock")
    gpu.set_precond(record=rec)
    gpu.sweep(1)
    rec.train(3, 4096, 3e-3)
    model = rec.params()
    _, g2, o2 = make_pair(wl.L, wl.N, wl.twoM, wl.D, wl.twoS, wl.G, U=wl.U, seed=wl.seed + 1)
    g2.set_precond(use=rec)
    rc, steps = g2.sweep(2, max_sub=128, max_iter=200)
    ref = omps.sweep(o2, 2, max_sub=128, max_iter=200, model=_as64(model), nblock=True)
    print("[precond] iterations per step (learned, per N-block):", [s["iters"] for s in steps], flush=True)
    assert all(s["converged"] for s in steps)
    assert [s["iters"] for s in steps] == [s["iters"] for s in ref]
    assert max(abs(a["theta"] - b["theta"]) for a, b in zip(steps, ref)) < 1e-8


def test_model_scope_rules():
    wl = W.hubbard_small()
    _, g, _ = make_pair(wl.L, wl.N, wl.twoM, wl.D, wl.twoS, wl.G, U=wl.U, seed=wl.seed, oracle=False)
    vec = sp.MLP(_params(16), capacity=100_000)
    blk = sp.MLP(_params(16), scope="nblock")
    with pytest.raises(sp.SpError):
        g.set_precond(use=blk, record=vec)
    g.set_precond(record=vec)
    g.sweep(1)
    assert vec.rows() > 0
    with pytest.raises(sp.SpError):
        vec.set_scope("nblock")
    vec.set_scope("vector")


def test_bad_model_falls_back_and_converges():
    # a model that always answers the same vector: the fallback rule hands
    # every solve back to the diagonal correction, which converges
    p = _params(16)
    p["W1"][:] = 0.0
    p["b1"][:] = 0.0
    p["w2"][:] = 0.0
    p["b2"] = np.float32(1.0)
    bad = sp.MLP(p)
    wl = W.hubbard_small()
    _, g1, _ = make_pair(wl.L, wl.N, wl.twoM, wl.D, wl.twoS, wl.G, U=wl.U, seed=wl.seed, oracle=False)
    _, g2, _ = make_pair(wl.L, wl.N, wl.twoM, wl.D, wl.twoS, wl.G, U=wl.U, seed=wl.seed, oracle=False)
    g2.set_precond(use=bad)
    r1, s1 = g1.sweep(2, max_sub=128, max_iter=200)
    r2, s2 = g2.sweep(2, max_sub=128, max_iter=200)
    assert all(s["converged"] for s in s2)
    assert abs(s1[-1]["theta"] - s2[-1]["theta"]) < 1e-8


def test_batched_sweeps_reject_models():
    wl = W.hubbard_small()
    _, g, _ = make_pair(wl.L, wl.N, wl.twoM, wl.D, wl.twoS, wl.G, U=wl.U, seed=wl.seed, oracle=False)
    g.set_precond(use=sp.MLP(_params(16)))
    with pytest.raises(sp.SpError):
        sp.sweep_batch([g], 1)
