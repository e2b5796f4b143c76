"""Pins of the learned-preconditioner reference (oracle.precond): the
back-propagated gradients against finite differences, closed forms of the
model, of Adam's first step and of the exact correction, and the solver hook
(the diagonal rule given as a preconditioner reproduces the default run)."""
import numpy as np
import pytest

import workloads as W
from oracle import mpo, mps, precond as pre, quadrature as q


def _params(hidden=16, seed=0):
    p = W.mlp_init(hidden, seed)
    rng = np.random.default_rng(seed + 1)
    p = {k: np.asarray(v, float) for k, v in p.items()}
    p["b1"] = rng.standard_normal(hidden) * 0.1
    p["b2"] = 0.3
    return p


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(4)
    p = _params()
    F = rng.standard_normal((50, 5))
    Y = rng.standard_normal(50)
    loss, g = pre.loss_and_grads(p, F, Y)
    assert abs(loss - 0.5 * np.mean((pre.forward(p, F) - Y) ** 2)) < 1e-14
    h = 1e-6
    for k in ("W1", "b1", "w2", "b2"):
        base = np.asarray(p[k], float)
        flat = base.ravel()
        for i in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            pp = dict(p)
            pm = dict(p)
            a = flat.copy()
            a[i] += h
            b_ = flat.copy()
            b_[i] -= h
            pp[k] = a.reshape(base.shape) if base.shape else float(a[0])
            pm[k] = b_.reshape(base.shape) if base.shape else float(b_[0])
            fd = (pre.loss_and_grads(pp, F, Y)[0] - pre.loss_and_grads(pm, F, Y)[0]) / (2 * h)
            an = np.asarray(g[k], float).ravel()[i]
            assert abs(fd - an) < 1e-7 * max(1.0, abs(an)), (k, i, fd, an)


def test_forward_closed_form():
    p = _params()
    p["W1"] = np.zeros_like(p["W1"])
    F = np.random.default_rng(0).standard_normal((7, 5))
    y = pre.forward(p, F)
    assert np.allclose(y, p["b2"] + np.maximum(p["b1"], 0) @ p["w2"], atol=1e-15)


def test_adam_first_step_is_a_signed_step():
    p = _params()
    F = np.random.default_rng(1).standard_normal((30, 5))
    Y = np.ones(30)
    _, g = pre.loss_and_grads(p, F, Y)
    st = {}
    out = pre.adam_step(p, g, st, lr=1e-3)
    for k in ("W1", "b1", "w2"):
        gk = np.asarray(g[k], float)
        exp = np.asarray(p[k], float) - 1e-3 * gk / (np.abs(gk) + 1e-8)
        assert np.allclose(out[k], exp, atol=1e-15)
    assert st["t"] == 1


def test_exact_correction_reaches_the_target():
    rng = np.random.default_rng(2)
    xs = rng.standard_normal(40)
    xs /= np.linalg.norm(xs)
    x = xs + 0.1 * rng.standard_normal(40)
    x /= np.linalg.norm(x)
    e = pre.exact_correction(x, xs)
    assert abs(x @ e) < 1e-12
    assert abs(np.sqrt(np.mean(e * e)) - 1.0) < 1e-12
    # x + c e is parallel to x* for the right c
    e_raw = xs / (x @ xs) - x
    y = x + e_raw
    assert np.linalg.norm(y / np.linalg.norm(y) - xs) < 1e-12


def test_features_definition():
    r = np.array([1.0, -2.0, 0.0, 3.0])
    dh = np.array([2.0, 1.0, 0.5, 1e-12])
    dn = np.array([1.0, 0.5, 0.0, 0.0])
    F = pre.features(r, dh, dn, theta=1.0)
    rms = np.sqrt(np.mean(r * r))
    assert np.allclose(F[:, 0], np.abs(r) / rms)
    assert np.allclose(F[:, 1], np.arcsinh(dh - dn))
    assert np.allclose(F[:, 2], np.arcsinh(dn))
    d = dh - dn
    d[3] = 1e-8  # floored
    assert np.allclose(F[:, 3], np.arcsinh(-(np.abs(r) / rms) / d))
    t = -r / d
    assert np.allclose(F[:, 4], np.sign(r) * t / np.sqrt(np.mean(t * t)))


def test_correction_is_odd_in_the_residual():
    p = _params()
    rng = np.random.default_rng(5)
    r, dh, dn = rng.standard_normal(20), rng.standard_normal(20) + 3, rng.random(20)
    a = pre.correction(p, r, dh, dn, 0.7)
    b = pre.correction(p, -r, dh, dn, 0.7)
    assert np.allclose(a, -b, atol=1e-15)
    x, xs = rng.standard_normal(20), rng.standard_normal(20)
    x /= np.linalg.norm(x)
    xs /= np.linalg.norm(xs)
    # flipping the Ritz vector flips r and e: the targets do not change
    assert np.allclose(pre.target(r, x, xs), pre.target(-r, -x, xs), atol=1e-12)


def test_solver_hook_with_the_diagonal_rule_reproduces_the_default():
    L = 6
    tab = W.make_block_table(L, L, 0, 16)
    G = q.exact_point_count(L, L, 0)
    runs = []
    for use_hook in (False, True):
        o = mps.SPMPSOracle(tab, W.random_blocks(tab, 3), mpo.hubbard_mpo(L, 1.0, 4.0), 0, G)
        k = 1
        m = o.mps.mask[k - 1]
        idx = np.flatnonzero(m.ravel())

        def mv(v):
            xd = np.zeros(m.size)
            xd[idx] = v
            y, ny = o.heff(k, xd.reshape(m.shape))
            return y.ravel()[idx], ny.ravel()[idx]
        dh, dn = (a.ravel()[idx] for a in o.heff_diag(k))

        def diag_rule(r, th):
            den = dh - th * dn
            den = np.where(np.abs(den) < 1e-8, np.where(den < 0, -1e-8, 1e-8), den)
            return -r / den
        rec = []
        res = mps.davidson(mv, dh, dn, o.mps.A[0].ravel()[idx], precond=diag_rule if use_hook else None,
                           record=rec)
        runs.append((res, rec))
    (a, ra), (b, rb) = runs
    assert a.iters == b.iters and abs(a.theta - b.theta) < 1e-14
    assert len(ra) == len(rb) == a.iters - 1
    r0, th0, x0, xs, _, _ = ra[0]
    assert abs(np.linalg.norm(x0) - 1) < 1e-12 and abs(np.linalg.norm(xs) - 1) < 1e-12


# --- per-N-block scope -------------------------------------------------------

def _diag_rule_model():
    # g = relu(f4) - relu(-f4) = f4: the diagonal rule written as the model
    W1 = np.zeros((2, 5))
    W1[0, 4], W1[1, 4] = 1.0, -1.0
    return {"W1": W1, "b1": np.zeros(2), "w2": np.array([1.0, -1.0]), "b2": 0.0}


def test_nblock_labels_group_by_the_particle_numbers_of_both_bonds():
    tab = W.make_block_table(6, 6, 0, 24)
    o = mps.OracleMPS(tab, W.random_blocks(tab, 1))
    for k in range(1, 7):
        m = o.mask[k - 1]
        s, a, b = np.unravel_index(np.flatnonzero(m.ravel()), m.shape)
        nl, nr = o.qn[k - 1][a, 0], o.qn[k][b, 0]
        lab = o.nblock_labels(k)
        # two elements share a label exactly when both bond particle numbers agree
        pairs = set(zip(nl.tolist(), nr.tolist()))
        assert len(np.unique(lab)) == len(pairs)
        for v in np.unique(lab):
            sel = lab == v
            assert len(set(nl[sel].tolist())) == 1 and len(set(nr[sel].tolist())) == 1
        # and merge the M sectors: some block holds both singly occupied states
        if k not in (1, 6):
            assert any(len(set(s[lab == v].tolist()) & {1, 2}) == 2 for v in np.unique(lab))


def _random_case(n=60, seed=9):
    rng = np.random.default_rng(seed)
    r = rng.standard_normal(n)
    dh = rng.standard_normal(n) + 3.0
    dn = rng.random(n)
    groups = rng.integers(0, 3, n)
    return r, dh, dn, groups


def test_block_features_with_one_block_are_the_global_ones():
    r, dh, dn, _ = _random_case()
    one = np.zeros(r.size, int)
    assert np.allclose(pre.features(r, dh, dn, 0.4, groups=one), pre.features(r, dh, dn, 0.4), atol=1e-15)
    x = np.random.default_rng(1).standard_normal(r.size)
    x /= np.linalg.norm(x)
    xs = x + 0.2 * np.random.default_rng(2).standard_normal(r.size)
    xs /= np.linalg.norm(xs)
    assert np.allclose(pre.target(r, x, xs, groups=one), pre.target(r, x, xs), atol=1e-14)


def test_block_correction_is_homogeneous_block_by_block():
    # scaling the residual of one block scales the correction there and
    # leaves the other blocks alone; a vector-wide normalisation does not
    p = _params()
    r, dh, dn, groups = _random_case()
    base = pre.correction(p, r, dh, dn, 0.4, groups=groups)
    r2 = np.where(groups == 1, 3.7 * r, r)
    scaled = pre.correction(p, r2, dh, dn, 0.4, groups=groups)
    assert np.allclose(scaled[groups == 1], 3.7 * base[groups == 1], rtol=1e-12, atol=0)
    assert np.allclose(scaled[groups != 1], base[groups != 1], rtol=1e-12, atol=0)
    g_base, g_scaled = pre.correction(p, r, dh, dn, 0.4), pre.correction(p, r2, dh, dn, 0.4)
    assert not np.allclose(g_scaled[groups != 1], g_base[groups != 1], rtol=1e-6)


def test_block_model_of_the_diagonal_rule_is_the_diagonal_correction():
    r, dh, dn, groups = _random_case()
    dh[5] = 0.4 * dn[5]  # a floored denominator
    d = dh - 0.4 * dn
    d = np.where(np.abs(d) < 1e-8, np.where(d < 0, -1e-8, 1e-8), d)
    got = pre.correction(_diag_rule_model(), r, dh, dn, 0.4, groups=groups)
    assert np.allclose(got, -r / d, rtol=1e-13, atol=0)


def test_block_targets_of_a_known_correction():
    # x = e_0 and x* = (e_0 + a u) / |.| with u orthogonal to e_0: the exact
    # correction is a u, so the target on each block is sign(r) sign(a) u
    # over the rms of u on that block
    rng = np.random.default_rng(3)
    n, a = 30, -0.35
    groups = np.repeat([0, 1, 2], 10)
    u = rng.standard_normal(n)
    u[0] = 0.0
    x = np.zeros(n)
    x[0] = 1.0
    xs = x + a * u
    xs /= np.linalg.norm(xs)
    r = rng.standard_normal(n)
    y = pre.target(r, x, xs, groups=groups)
    for g in range(3):
        sel = groups == g
        ref = np.sign(r[sel]) * np.sign(a) * u[sel] / np.sqrt(np.mean(u[sel] ** 2))
        assert np.allclose(y[sel], ref, atol=1e-12)
        assert abs(np.mean(y[sel] ** 2) - 1.0) < 1e-12


def test_block_sweep_with_the_diagonal_rule_model_reproduces_the_default():
    # the block-scoped hook with the model that equals the diagonal rule
    # follows the default solver step by step
    L = 6
    tab = W.make_block_table(L, L, 0, 16)
    G = q.exact_point_count(L, L, 0)
    runs = []
    for model in (None, _diag_rule_model()):
        o = mps.SPMPSOracle(tab, W.random_blocks(tab, 3), mpo.hubbard_mpo(L, 1.0, 4.0), 0, G)
        runs.append(mps.sweep(o, 1, model=model, nblock=True))
    a, b = runs
    assert [s["iters"] for s in a] == [s["iters"] for s in b]
    assert max(abs(x["theta"] - y["theta"]) for x, y in zip(a, b)) < 1e-10
