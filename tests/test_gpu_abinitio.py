"""Parity of the HIP path with the FP64 oracle on ab-initio Hamiltonians
(Eq. [sqH]) with seeded synthetic integrals.  The library builds its MPO with
its own O(K^2) construction, the oracle with its own automaton; both are the
same operator (pinned against exact diagonalisation on the CPU), so H_eff and
N_eff as maps on the site tensor agree whatever the MPO layout.

Cases cover the fused kernel, the LDS-tiled block products that sites too
wide for the fused kernel run (forced here with sp_set_heff_plan), the plain
path, FP32 products and batched sweeps.  Tolerances as in the Hubbard parity
tests: 1e-11 relative for products, 1e-8 for sweep energies in FP64, 1e-6 in
FP32."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from gpu_util import make_pair, rel_err  # noqa: E402

import paper_1703_04789_amd as sp  # noqa: E402
import workloads as W  # noqa: E402
from oracle import ed, mps as omps, quadrature as oq  # noqa: E402

pytestmark = pytest.mark.gpu

CASES = [  # (K, N, 2M, D, 2S)
    (4, 4, 0, 16, 0),
    (5, 4, 0, 24, 2),
    (5, 5, 1, 20, 1),
    (6, 6, 0, 32, 0),
]


def _pair(K, N, twoM, D, twoS, path="tiled", precision="fp64", oracle=True, seed=1):
    G = oq.exact_point_count(N, K, twoS, twoM)
    ints = W.abinitio_integrals(K, seed=4)
    return make_pair(K, N, twoM, D, twoS, G, seed=seed, op="abinitio", integrals=ints, path=path,
                     precision=precision, oracle=oracle)


def _dev(a):
    return torch.tensor(a, dtype=torch.float64, device="cuda")


def _force_tiled(gpu):
    for k in range(1, gpu.L + 1):
        assert gpu.set_heff_plan(k, 0) == 0


@pytest.mark.parametrize("plan", ["fused", "tiled-lists", "plain"])
@pytest.mark.parametrize("case", CASES)
def test_abinitio_heff_all_sites(case, plan):
    tab, gpu, orc = _pair(*case, path="plain" if plan == "plain" else "tiled")
    if plan == "tiled-lists":
        _force_tiled(gpu)
    rng = np.random.default_rng(3)
    for k in range(1, tab.L + 1):
        if k > 1:
            gpu.env_update(k - 1, +1)
            orc.update_left(k - 1)
        n = gpu.site_size(k)
        x = rng.standard_normal(n)
        y_ref, ny_ref = orc.heff(k, orc.mps.dense_site(k, x))
        xd = _dev(x)
        y, ny = torch.empty_like(xd), torch.empty_like(xd)
        gpu.heff_apply(k, xd, y, ny)
        dh, dn = torch.empty_like(xd), torch.empty_like(xd)
        gpu.heff_diag(k, dh, dn)
        torch.cuda.synchronize()
        assert rel_err(y.cpu().numpy(), orc.mps.site_packed(k, y_ref)) < 1e-11, k
        assert rel_err(ny.cpu().numpy(), orc.mps.site_packed(k, ny_ref)) < 1e-11, k
        dh_ref, dn_ref = orc.heff_diag(k)
        assert rel_err(dh.cpu().numpy(), orc.mps.site_packed(k, dh_ref)) < 1e-11, k
        assert rel_err(dn.cpu().numpy(), orc.mps.site_packed(k, dn_ref)) < 1e-11, k


def test_abinitio_autotuned_plans_keep_parity():
    # the autotuner chooses per site between fused plans and the tiled block
    # products; every choice must keep the products equal to the oracle's
    case = CASES[3]
    tab, gpu, orc = _pair(*case)
    choice = gpu.autotune(reps=2)
    print(f"[autotune] (budget, rows, us) {choice}", flush=True)
    assert all((b > 0 and 1 <= r <= 8) or (b == 0 and r == 0) for b, r, _ in choice)
    rng = np.random.default_rng(12)
    for k in range(1, tab.L + 1):
        if k > 1:
            gpu.env_update(k - 1, +1)
            orc.update_left(k - 1)
        x = rng.standard_normal(gpu.site_size(k))
        y_ref, ny_ref = orc.heff(k, orc.mps.dense_site(k, x))
        xd = _dev(x)
        y, ny = torch.empty_like(xd), torch.empty_like(xd)
        gpu.heff_apply(k, xd, y, ny)
        torch.cuda.synchronize()
        assert rel_err(y.cpu().numpy(), orc.mps.site_packed(k, y_ref)) < 1e-11, k
        assert rel_err(ny.cpu().numpy(), orc.mps.site_packed(k, ny_ref)) < 1e-11, k


@pytest.mark.parametrize("case", [CASES[1], CASES[3]])
def test_abinitio_tiled_product_follows_the_left_environment(case):
    """The tiled products keep the W r mixing of L[k-1] from one product to
    the next: after a new left tensor and a rebuilt L[k-1], the next product
    at the same site must use the new environment."""
    tab, gpu, orc = _pair(*case)
    _force_tiled(gpu)
    k = 3
    rng = np.random.default_rng(11)
    for j in range(1, k):
        gpu.env_update(j, +1)
        orc.update_left(j)
    for rep in range(3):
        if rep:
            a = rng.standard_normal(gpu.site_size(k - 1))
            gpu.set_site(k - 1, a)
            orc.mps.A[k - 2] = orc.mps.dense_site(k - 1, a)
            gpu.env_update(k - 1, +1)
            orc.update_left(k - 1)
        print(f"[case] K={tab.L} site={k} rebuild={rep}", flush=True)
        for _ in range(2):  # twice with the same environment, new x each time
            x = rng.standard_normal(gpu.site_size(k))
            y_ref, ny_ref = orc.heff(k, orc.mps.dense_site(k, x))
            xd = _dev(x)
            y, ny = torch.empty_like(xd), torch.empty_like(xd)
            gpu.heff_apply(k, xd, y, ny)
            torch.cuda.synchronize()
            assert rel_err(y.cpu().numpy(), orc.mps.site_packed(k, y_ref)) < 1e-11, rep
            assert rel_err(ny.cpu().numpy(), orc.mps.site_packed(k, ny_ref)) < 1e-11, rep


@pytest.mark.parametrize("case", CASES)
def test_abinitio_energy_at_centre(case):
    tab, gpu, orc = _pair(*case)
    E, p = gpu.energy()
    Ef, pf = orc.full_contraction()
    assert abs(E - Ef) < 1e-10


@pytest.mark.parametrize("plan", ["fused", "tiled-lists", "plain"])
def test_abinitio_sweep_matches_oracle(plan):
    # exact local solves, so both trajectories are the same smooth function
    # of the input
    case = (5, 4, 0, 24, 2)
    tab, gpu, orc = _pair(*case, path="plain" if plan == "plain" else "tiled")
    if plan == "tiled-lists":
        _force_tiled(gpu)
    rc, steps = gpu.sweep(2, max_sub=128, max_iter=200)
    ref = omps.sweep(orc, 2, max_sub=128, max_iter=200)
    dE = max(abs(a["theta"] - b["theta"]) for a, b in zip(steps, ref))
    assert dE < 1e-8, dE


@pytest.mark.parametrize("twoS", [0, 2])
def test_abinitio_full_bond_dimension_reaches_ed(twoS):
    K, N = 4, 4
    h, eri = W.abinitio_integrals(K, seed=4)
    st = ed.sector_states(K, N, 0)
    e_ed = ed.projected_ground_energy(ed.abinitio_hamiltonian(h, eri, st),
                                      ed.lowdin_projector(ed.s2_operator(K, st), twoS, 0, N))
    tab, gpu, _ = _pair(K, N, 0, 16, twoS, oracle=False, seed=5)
    rc, steps = gpu.sweep(3, max_sub=128, max_iter=200)
    assert abs(steps[-1]["theta"] - e_ed) < 1e-9
    E, p = gpu.energy()
    assert abs(E - e_ed) < 1e-9


def test_abinitio_fp32_products():
    # FP32 environments and accumulation: every site's products within 1e-5
    # of the FP64 oracle relative to the largest entry (the FP32 bar of the
    # Hubbard tests)
    case = (6, 6, 0, 32, 0)
    tab, gpu, orc = _pair(*case, precision="fp32")
    rng = np.random.default_rng(4)
    worst = 0.0
    for k in range(1, tab.L + 1):
        if k > 1:
            orc.mps.left_orthonormalize(k - 1)
            orc.update_left(k - 1)
            gpu.set_site(k - 1, orc.mps.site_packed(k - 1))
            gpu.set_site(k, orc.mps.site_packed(k))
            gpu.env_update(k - 1, +1)
        n = gpu.site_size(k)
        x = rng.standard_normal(n)
        y_ref, ny_ref = orc.heff(k, orc.mps.dense_site(k, x))
        xd = _dev(x)
        y, ny = torch.empty_like(xd), torch.empty_like(xd)
        gpu.heff_apply(k, xd, y, ny)
        torch.cuda.synchronize()
        e1 = rel_err(y.cpu().numpy(), orc.mps.site_packed(k, y_ref))
        e2 = rel_err(ny.cpu().numpy(), orc.mps.site_packed(k, ny_ref))
        worst = max(worst, e1, e2)
        assert e1 < 1e-5 and e2 < 1e-5, (k, e1, e2)
    print(f"[abinitio fp32] worst product error {worst:.2e}", flush=True)


def test_abinitio_fp32_sweeps_reach_the_fp64_energy():
    # K=6, N=6, D=32: ten sweeps in FP32 (solver tolerance 1e-5) and in FP64
    # (1e-9, pinned to the oracle step by step above); the energies reached
    # agree to the reduced-precision target
    case = (6, 6, 0, 32, 0)
    res = {}
    for prec, tol in (("fp64", 1e-9), ("fp32", 1e-5)):
        _, gpu, _ = _pair(*case, precision=prec, oracle=False)
        rc, steps = gpu.sweep(10, max_sub=128, max_iter=200, tol=tol)
        res[prec] = steps[-1]["theta"]
        gpu.close()
    dE = abs(res["fp32"] - res["fp64"])
    print(f"[abinitio fp32] K=6 D=32 after 10 sweeps: fp64 {res['fp64']:.10f} fp32 {res['fp32']:.10f} "
          f"|dE| {dE:.2e}", flush=True)
    assert dE < 1e-6


def test_abinitio_wide_mpo_tiled_and_plain_paths_agree():
    # K = 12, D = 128: the centre sites are too wide for the fused kernel and
    # run the tiled block products automatically; the plain path is the
    # reference here (the oracle's automaton MPO is too large at K = 12)
    wl = W.abinitio_reduced(12, 128, 11)
    h, eri = wl.integrals()
    mine = sp.mpo_abinitio(h, eri)
    tab, blocks = wl.table(), wl.blocks()
    print(f"[case] {wl.name}", flush=True)
    a = sp.SPMPS(tab, blocks, mine, wl.twoS, wl.G, path="tiled")
    b = sp.SPMPS(tab, blocks, mine, wl.twoS, wl.G, path="plain")
    Ea, _ = a.energy()
    Eb, _ = b.energy()
    assert abs(Ea - Eb) < 1e-10 * max(1.0, abs(Eb))
    rng = np.random.default_rng(2)
    for k in range(1, wl.K // 2 + 1):
        if k > 1:
            a.env_update(k - 1, +1)
            b.env_update(k - 1, +1)
        n = a.site_size(k)
        xd = _dev(rng.standard_normal(n))
        ya, nya, yb, nyb = (torch.empty_like(xd) for _ in range(4))
        a.heff_apply(k, xd, ya, nya)
        b.heff_apply(k, xd, yb, nyb)
        torch.cuda.synchronize()
        assert rel_err(ya.cpu().numpy(), yb.cpu().numpy()) < 1e-11, k
        assert rel_err(nya.cpu().numpy(), nyb.cpu().numpy()) < 1e-11, k


def test_abinitio_batched_sweeps_match_single():
    # two ab-initio states (one with every site on the tiled block products)
    # and a Hubbard state advanced together
    cases = [(5, 4, 0, 24, 2), (6, 6, 0, 32, 0)]
    singles, batch = [], []
    for i, c in enumerate(cases):
        _, s1, _ = _pair(*c, oracle=False, seed=7 + i)
        _, s2, _ = _pair(*c, oracle=False, seed=7 + i)
        if i == 0:
            _force_tiled(s1)
            _force_tiled(s2)
        singles.append(s1)
        batch.append(s2)
    _, hs1, _ = make_pair(8, 8, 0, 32, 0, 5, seed=3, oracle=False)
    _, hs2, _ = make_pair(8, 8, 0, 32, 0, 5, seed=3, oracle=False)
    singles.append(hs1)
    batch.append(hs2)
    for solver in ("device", "host"):  # each driver against its own single-state sweeps
        ref = [s.sweep(2, solver=solver)[1] for s in singles]
        rc, got = sp.sweep_batch(batch, 2, solver=solver)
        for r, g in zip(ref, got):
            assert len(r) == len(g)
            assert max(abs(a["theta"] - b["theta"]) for a, b in zip(r, g)) < 1e-10


def test_abinitio_fp32_products_on_fused_and_tiled_sites():
    # K = 12, D = 128: with SP_FP32 the fused sites use FP32 environments and
    # the sites on the tiled block products stay FP64
    wl = W.abinitio_reduced(12, 128, 11)
    mine = sp.mpo_abinitio(*wl.integrals())
    tab, blocks = wl.table(), wl.blocks()
    print(f"[case] {wl.name} fp32 vs fp64", flush=True)
    a = sp.SPMPS(tab, blocks, mine, wl.twoS, wl.G, precision="fp32")
    b = sp.SPMPS(tab, blocks, mine, wl.twoS, wl.G)
    rng = np.random.default_rng(8)
    seen = set()
    for k in range(1, wl.K // 2 + 1):
        if k > 1:
            a.env_update(k - 1, +1)
            b.env_update(k - 1, +1)
        fused = a.heff_plan(k)[0] > 0
        xd = _dev(rng.standard_normal(a.site_size(k)))
        ya, nya, yb, nyb = (torch.empty_like(xd) for _ in range(4))
        a.heff_apply(k, xd, ya, nya)
        b.heff_apply(k, xd, yb, nyb)
        torch.cuda.synchronize()
        e = max(rel_err(ya.cpu().numpy(), yb.cpu().numpy()), rel_err(nya.cpu().numpy(), nyb.cpu().numpy()))
        assert e < (1e-5 if fused else 1e-12), (k, fused, e)
        seen.add(fused)
    assert seen == {True, False}
