"""Split-BF16 block products (SP_BF16X3): the LDS-tiled products of sites
too wide for the fused kernel run on the BF16 matrix cores with each operand
split into two bf16 values and three products accumulated in FP32.  Each
operand carries about 16 significant bits, so a product is accurate to a
relative error of order 1e-5; H_eff x is a chain of two such products (the
pre-mixed environment times x, then the right environment), and the bar
below is 1e-4 relative to the largest entry against the FP64 oracle.  Sweeps
report an FP64 Rayleigh quotient per step, so the energies reached agree
with the FP64 path to the reduced-precision energy target of 1e-6."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from gpu_util import make_pair, rel_err  # noqa: E402

import paper_1703_04789_amd as sp  # noqa: E402
import workloads as W  # noqa: E402
from oracle import quadrature as oq  # noqa: E402

pytestmark = pytest.mark.gpu


def _pair(K, N, twoM, D, twoS, precision="bf16x3", oracle=True, seed=1):
    G = oq.exact_point_count(N, K, twoS, twoM)
    ints = W.abinitio_integrals(K, seed=4)
    return make_pair(K, N, twoM, D, twoS, G, seed=seed, op="abinitio", integrals=ints, precision=precision,
                     oracle=oracle)


def _force_tiled(gpu):
    for k in range(1, gpu.L + 1):
        assert gpu.set_heff_plan(k, 0) == 0


def _dev(a):
    return torch.tensor(a, dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("case", [(5, 4, 0, 24, 2), (6, 6, 0, 32, 0)])
def test_bf16x3_products_match_the_oracle(case):
    tab, gpu, orc = _pair(*case)
    _force_tiled(gpu)
    rng = np.random.default_rng(4)
    worst = 0.0
    for k in range(1, tab.L + 1):
        if k > 1:
            orc.mps.left_orthonormalize(k - 1)
            orc.update_left(k - 1)
            gpu.set_site(k - 1, orc.mps.site_packed(k - 1))
            gpu.set_site(k, orc.mps.site_packed(k))
            gpu.env_update(k - 1, +1)
        print(f"[case] K={tab.L} D={case[3]} site={k} bf16x3", flush=True)
        x = rng.standard_normal(gpu.site_size(k))
        y_ref, ny_ref = orc.heff(k, orc.mps.dense_site(k, x))
        xd = _dev(x)
        y, ny = torch.empty_like(xd), torch.empty_like(xd)
        gpu.heff_apply(k, xd, y, ny)
        torch.cuda.synchronize()
        e1 = rel_err(y.cpu().numpy(), orc.mps.site_packed(k, y_ref))
        e2 = rel_err(ny.cpu().numpy(), orc.mps.site_packed(k, ny_ref))
        worst = max(worst, e1, e2)
        assert e1 < 1e-4 and e2 < 1e-4, (k, e1, e2)
        # more accurate than plain BF16 (8 significant bits, ~4e-3)
    print(f"[bf16x3] worst product error {worst:.2e}", flush=True)


def test_bf16x3_wide_sites_against_fp64():
    # K = 12, D = 128: the centre sites run the tiled products in split BF16,
    # the fused sites in FP32; both against the FP64 path on the same input
    wl = W.abinitio_reduced(12, 128, 11)
    mine = sp.mpo_abinitio(*wl.integrals())
    tab, blocks = wl.table(), wl.blocks()
    print(f"[case] {wl.name} bf16x3 vs fp64", flush=True)
    a = sp.SPMPS(tab, blocks, mine, wl.twoS, wl.G, precision="bf16x3")
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
        print(f"[bf16x3] site {k} fused={fused} error {e:.2e}", flush=True)
        assert e < (1e-5 if fused else 1e-4), (k, fused, e)
        seen.add(fused)
    assert seen == {True, False}


def test_bf16x3_sweeps_reach_the_fp64_energy():
    # K=6, N=6, D=32 with every site on the split-BF16 products: ten sweeps
    # (solver tolerance 1e-4) against the FP64 path (1e-9)
    case = (6, 6, 0, 32, 0)
    res = {}
    for prec, tol in (("fp64", 1e-9), ("bf16x3", 1e-4)):
        _, gpu, _ = _pair(*case, precision=prec, oracle=False)
        _force_tiled(gpu)
        print(f"[case] K=6 D=32 sweeps {prec}", flush=True)
        rc, steps = gpu.sweep(10, max_sub=128, max_iter=200, tol=tol)
        res[prec] = steps[-1]["theta"]
        gpu.close()
    dE = abs(res["bf16x3"] - res["fp64"])
    print(f"[bf16x3] K=6 D=32 after 10 sweeps: fp64 {res['fp64']:.10f} bf16x3 {res['bf16x3']:.10f} "
          f"|dE| {dE:.2e}", flush=True)
    assert dE < 1e-6
