"""Reduced-precision path (SP_FP32) against the FP64 oracle.

The H_eff x / N_eff x products inside the local solves run on FP32 copies of
the environments with FP32 accumulation; everything else stays FP64, and the
energy of every site step is an FP64 Rayleigh quotient.  Tolerances:
- single products: 1e-5 relative to the largest output entry (FP32 unit
  roundoff 6e-8 times sums of up to a few hundred terms with cancellation);
- energies: 1e-6 absolute (the reduced-precision target), using a solver
  tolerance of 1e-5 on the residual (the FP32 floor of these products is
  about 1e-6).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from gpu_util import make_pair, rel_err  # noqa: E402

import workloads as W  # noqa: E402
from oracle import mps as omps, quadrature as oq  # noqa: E402

pytestmark = pytest.mark.gpu

CASES = [  # (L, N, 2M, D, 2S, G)
    (8, 8, 0, 16, 0, 5),
    (7, 6, 2, 20, 4, 4),
    (10, 10, 0, 48, 2, 6),
]
TOL_PRODUCT = 1e-5
TOL_ENERGY = 1e-6
SOLVER_TOL = 1e-5


def _dev(a):
    return torch.tensor(a, dtype=torch.float64, device="cuda")


def _move_centre(gpu, orc, k):
    """Left-orthonormalise sites 1..k-1 in the oracle (as a sweep would),
    hand the same tensors to the library and build the left environments.
    Without this the left environments of random right-canonical tensors
    grow exponentially with the site index and leave the FP32 range at the
    bench shape."""
    for j in range(1, k):
        orc.mps.left_orthonormalize(j)
        orc.update_left(j)
    for j in range(1, k + 1):
        gpu.set_site(j, orc.mps.site_packed(j))
    for j in range(1, k):
        gpu.env_update(j, +1)


@pytest.mark.parametrize("case", CASES)
def test_fp32_heff_all_sites(case):
    rng = np.random.default_rng(15)
    worst = 0.0
    L = case[0]
    for k in range(1, L + 1):
        tab, gpu, orc = make_pair(*case, precision="fp32")
        _move_centre(gpu, orc, k)
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
        assert e1 < TOL_PRODUCT and e2 < TOL_PRODUCT, (k, e1, e2)
    print(f"[fp32] worst relative product error {worst:.2e}")


def test_fp32_bench_shape_heff():
    wl = W.hubbard_bench(0)
    tab, gpu, orc = make_pair(wl.L, wl.N, wl.twoM, wl.D, wl.twoS, wl.G, U=wl.U, seed=wl.seed, precision="fp32")
    kc = wl.L // 2
    _move_centre(gpu, orc, kc)
    n = gpu.site_size(kc)
    x = np.random.default_rng(8).standard_normal(n)
    y_ref, ny_ref = orc.heff(kc, orc.mps.dense_site(kc, x))
    xd = _dev(x)
    y, ny = torch.empty_like(xd), torch.empty_like(xd)
    gpu.heff_apply(kc, xd, y, ny)
    torch.cuda.synchronize()
    e1 = rel_err(y.cpu().numpy(), orc.mps.site_packed(kc, y_ref))
    e2 = rel_err(ny.cpu().numpy(), orc.mps.site_packed(kc, ny_ref))
    print(f"[fp32] bench shape: relative error y {e1:.2e} ny {e2:.2e}")
    assert e1 < TOL_PRODUCT and e2 < TOL_PRODUCT


def test_fp32_sweeps_reach_the_fp64_energy():
    # L=8, U=4, D=16, G=5: twelve sweeps of the FP32 path (solver tolerance
    # 1e-5) against twelve of the FP64 path (1e-9), the latter being pinned
    # to the oracle step by step elsewhere.  Trajectories of truncated sweeps
    # drift apart at the 1e-6 level along the way (different local
    # tolerances); the energies they reach must agree to the FP32 target.
    wl = W.hubbard_small()
    res = {}
    for prec, tol in (("fp64", 1e-9), ("fp32", SOLVER_TOL)):
        tab, gpu, _ = make_pair(wl.L, wl.N, wl.twoM, wl.D, wl.twoS, wl.G, U=wl.U, seed=wl.seed, oracle=False,
                                precision=prec)
        rc, steps = gpu.sweep(12, max_sub=128, max_iter=200, tol=tol)
        res[prec] = steps[-1]["theta"]
        gpu.close()
    dE = abs(res["fp32"] - res["fp64"])
    print(f"[fp32] L=8 D=16 after 12 sweeps: fp64 {res['fp64']:.10f} fp32 {res['fp32']:.10f} |dE| {dE:.2e}")
    assert dE < TOL_ENERGY
    assert res["fp32"] > -4.235806999129714 - 1e-10


@pytest.mark.parametrize("L,twoS,ref", [(6, 0, -3.092565319505379), (6, 2, -2.6914960192367765)])
def test_fp32_full_bond_dimension_reaches_ed(L, twoS, ref):
    G = oq.exact_point_count(L, L, twoS)
    tab, gpu, orc = make_pair(L, L, 0, 4 ** (L // 2), twoS, G, oracle=False, precision="fp32")
    rc, steps = gpu.sweep(3, max_sub=128, max_iter=200, tol=SOLVER_TOL)
    assert abs(steps[-1]["theta"] - ref) < TOL_ENERGY
    E, p = gpu.energy()
    # the reported step energy is the FP64 Rayleigh quotient of the state
    assert abs(E - steps[-1]["theta"]) < 1e-10
