"""Batched sweeps (sp_sweep_batch): several states advanced together must
reproduce their single-state sweeps run by the same driver.  The batched
passes run the same per-state arithmetic in the same order, so the step
energies agree to rounding (1e-12 is asserted)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from gpu_util import make_pair  # noqa: E402

import paper_1703_04789_amd as sp  # noqa: E402
import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu

CASES = [  # (L, N, 2M, D, 2S, G)
    (8, 8, 0, 16, 0, 5),
    (6, 5, 1, 12, 1, 3),
    (10, 10, 0, 48, 2, 6),
]


def _handles(cases, **kw):
    return [make_pair(*c, oracle=False, **kw)[1] for c in cases]


@pytest.mark.parametrize("solver", ["device", "host"])
@pytest.mark.parametrize("opts", [dict(), dict(max_sub=8, keep=4, max_iter=30)])
def test_batch_matches_single_runs(opts, solver):
    # both drivers: the device-resident iteration (one graph per round for
    # all states) and the host-driven one (states advance independently)
    singles = []
    for h in _handles(CASES):
        rc, steps = h.sweep(2, solver=solver, **opts)
        singles.append(steps)
        h.close()
    hs = _handles(CASES)
    rc, batch = sp.sweep_batch(hs, 2, solver=solver, **opts)
    for one, many in zip(singles, batch):
        assert len(one) == len(many)
        for a, b in zip(one, many):
            assert (a["site"], a["dir"], a["iters"], a["matvecs"]) == (b["site"], b["dir"], b["iters"], b["matvecs"])
            assert abs(a["theta"] - b["theta"]) < 1e-12
    # the states themselves: energies at the centre after the sweeps
    for h, steps in zip(hs, batch):
        E, p = h.energy()
        assert abs(E - steps[-1]["theta"]) < 1e-10


def test_batch_fp32_matches_single_runs():
    singles = []
    for h in _handles(CASES, precision="fp32"):
        singles.append(h.sweep(1, tol=1e-5, solver="device")[1])
        h.close()
    rc, batch = sp.sweep_batch(_handles(CASES, precision="fp32"), 1, tol=1e-5)
    for one, many in zip(singles, batch):
        assert max(abs(a["theta"] - b["theta"]) for a, b in zip(one, many)) < 1e-12


def test_batch_of_neel_guesses():
    # reduced broken-symmetry instances (L 12-16, D 32-64): one sweep each,
    # batched and alone
    ws = W.hubbard_batch(4, D_choices=(32, 64))
    ws = [w for w in ws if w.L <= 16] or ws[:1]
    def mk():
        out = []
        for w in ws:
            print(f"[case] {w.name}", flush=True)
            out.append(sp.SPMPS(w.table(), w.blocks(), sp.mpo_hubbard(w.L, w.t, w.U), w.twoS, w.G))
        return out
    singles = [h.sweep(1, solver="device")[1] for h in mk()]
    rc, batch = sp.sweep_batch(mk(), 1)
    for one, many in zip(singles, batch):
        assert np.isfinite([s["theta"] for s in many]).all()
        assert max(abs(a["theta"] - b["theta"]) for a, b in zip(one, many)) < 1e-12


def test_batch_rejects_bad_input():
    a, b = _handles(CASES[:2])
    c = _handles(CASES[:1], precision="fp32")[0]
    with pytest.raises(sp.SpError):
        sp.sweep_batch([a, a], 1)
    with pytest.raises(sp.SpError):
        sp.sweep_batch([a, c], 1)
    d = _handles(CASES[:1], path="plain")[0]
    with pytest.raises(sp.SpError):
        sp.sweep_batch([b, d], 1)


def test_batched_heff_profile_reports_the_summed_work():
    ws = W.hubbard_batch(6, D_choices=(64, 128))[:3]
    hs = [sp.SPMPS(w.table(), w.blocks(), sp.mpo_hubbard(w.L, w.t, w.U), w.twoS, w.G) for w in ws]
    sites = [w.L // 2 for w in ws]
    for h, k in zip(hs, sites):
        for j in range(1, k):
            h.env_update(j, +1)
    out = sp.heff_batch_profile(hs, sites, reps=3)
    assert out["usec"] > 0 and out["workgroups"] > 0
    # the launches captured in a HIP graph: three replays, each after eager
    # work that clears the outputs, reproduce the eager partials exactly
    assert out["graph_usec"] > 0 and out["graph_max_diff"] == 0.0
    assert abs(out["flops"] - sum(h.heff_flops(k) for h, k in zip(hs, sites))) < 1.0
    with pytest.raises(sp.SpError):
        sp.heff_batch_profile([hs[0], hs[0]], [sites[0], sites[0]])


def test_batch_matches_oracle():
    # three states of different L, N, S, M and D advanced together, with
    # exact local solves (the search space covers every local problem): each
    # state's step energies follow the oracle's own sweep of that state.
    # The cases are ones whose two-sweep trajectory is stable: a 1e-13
    # relative change of the initial blocks moves the oracle's step energies
    # by at most 3e-11 (some states of tiny spin-S weight amplify it to 1e-3)
    from oracle import mps as omps
    cases = [(8, 8, 0, 16, 0, 5), (6, 5, 1, 12, 1, 3), (6, 6, 2, 16, 4, 4)]
    pairs = [make_pair(*c) for c in cases]
    opts = dict(max_sub=128, max_iter=200)
    rc, batch = sp.sweep_batch([g for _, g, _ in pairs], 2, **opts)
    assert rc == sp.SP_OK
    for (tab, gpu, orc), steps in zip(pairs, batch):
        ref = omps.sweep(orc, 2, **opts)
        assert len(steps) == len(ref) == 2 * 2 * (tab.L - 1)
        for a, b in zip(steps, ref):
            assert (a["site"], a["dir"]) == (b["site"], b["dir"])
            assert abs(a["theta"] - b["theta"]) < 1e-8, (a, b)
        E, _ = gpu.energy()
        assert abs(E - ref[-1]["theta"]) < 1e-8
