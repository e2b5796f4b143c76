"""Projected spin-free properties through the library's contractions
(sp_expect) against the oracle, FP64 (1e-10 absolute), plus the sum rules
after sweeps: sum_p <n_p> = N, sum_{XY} <S_X.S_Y> = S(S+1), sum_p e_p = E."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from gpu_util import make_pair  # noqa: E402

import paper_1703_04789_amd as sp  # noqa: E402
from oracle import mpo as om, mps as omps  # noqa: E402

pytestmark = pytest.mark.gpu

CASES = [  # (L, N, 2M, D, 2S, G)
    (8, 8, 0, 16, 0, 5),
    (6, 5, 1, 12, 1, 3),
]


@pytest.mark.parametrize("case", CASES)
def test_expectations_match_the_oracle(case):
    tab, gpu, orc = make_pair(*case)
    L, twoS, G = case[0], case[4], case[5]
    blocks = orc.mps.packed()
    for mine, ref in ((sp.mpo_epq(L, 1, 3), om.epq_mpo(L, 1, 3)),
                      (sp.mpo_epq(L, L, 2), om.epq_mpo(L, L, 2)),
                      (sp.mpo_epq(L, 2, 2), om.epq_mpo(L, 2, 2)),
                      (sp.mpo_spin_corr(L, 1, L), om.spin_corr_mpo(L, 1, L))):
        v, p = gpu.expect(mine)
        vr, pr = omps.expect(tab, blocks, ref, twoS, G)
        assert abs(v - vr) < 1e-10 and abs(p - pr) < 1e-10


def test_sum_rules_after_sweeps():
    L, N, twoM, D, twoS, G = 8, 8, 0, 16, 2, 5
    t, U = 1.0, 4.0
    tab, gpu, _ = make_pair(L, N, twoM, D, twoS, G, U=U, oracle=False)
    rc, steps = gpu.sweep(2, max_sub=64, max_iter=100)
    E, _ = gpu.energy()
    gamma = gpu.one_rdm()
    assert abs(np.trace(gamma) - N) < 1e-9
    assert np.abs(gamma - gamma.T).max() < 1e-9
    ss = gpu.spin_correlations()
    assert abs(ss.sum() - 2.0) < 1e-9
    e = gpu.hubbard_energy_components(t, U)
    print(f"[props] E {E:.10f} sum e_p {e.sum():.10f}")
    assert abs(e.sum() - E) < 1e-9


def test_energy_components_match_the_oracle():
    # e_p of Sec. 2.4 (one sp_expect per orbital with the library's H_p MPO)
    # against the oracle's expectation of its own H_p MPO, and sum_p e_p = E
    import workloads as W
    tab, gpu, orc = make_pair(8, 8, 0, 16, 0, 5)
    blocks = orc.mps.packed()
    h, eri = om.hubbard_integrals(8, 1.0, 4.0)
    e = gpu.hubbard_energy_components(1.0, 4.0)
    for p in range(1, 9):
        ref, _ = omps.expect(tab, blocks, om.abinitio_component_mpo(h, eri, p), 0, 5)
        assert abs(e[p - 1] - ref) < 1e-10, p
    E, _ = gpu.energy()
    assert abs(e.sum() - E) < 1e-10
    K = 5
    h, eri = W.abinitio_integrals(K, 4)
    tab, gpu, orc = make_pair(K, K, 1, 24, 1, 3, op="abinitio", integrals=(h, eri))
    blocks = orc.mps.packed()
    e = gpu.abinitio_energy_components(h, eri)
    for p in range(1, K + 1):
        ref, _ = omps.expect(tab, blocks, om.abinitio_component_mpo(h, eri, p), 1, 3)
        assert abs(e[p - 1] - ref) < 1e-10, p
    E, _ = gpu.energy()
    assert abs(e.sum() - E) < 1e-10


@pytest.mark.parametrize("twoS", [0, 2])
def test_bench_shape_projected_invariants(twoS):
    # L=32, U=8, D=256, G=9 (the benchmark workload, S=0 and S=1) after one
    # sweep: with the exact quadrature the projected state is a pure spin-S
    # state, so <S^2 P>/<P> = S(S+1) exactly at any bond dimension (checks
    # the rotated environments and the projector on the benchmark's own
    # state; no oracle fits this size), and the energy of the final state is
    # the last step's eigenvalue
    import workloads as W
    wl = W.hubbard_bench(twoS)
    gpu = sp.SPMPS(wl.table(), wl.blocks(), sp.mpo_hubbard(wl.L, wl.t, wl.U), wl.twoS, wl.G)
    print(f"[case] bench shape 2S={twoS}", flush=True)
    rc, steps = gpu.sweep(1)
    s2, p = gpu.expect(sp.mpo_s2(wl.L))
    S = twoS / 2
    assert abs(s2 - S * (S + 1)) < 1e-8 and 0.0 < p <= 1.0 + 1e-12
    E, _ = gpu.energy()
    assert abs(E - steps[-1]["theta"]) < 1e-8
    gpu.close()
