"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Element-wise comparisons at sizes the oracle finishes in seconds (several
blocks per bond, ragged sector sizes, odd electron counts, half-integer
spin), plus the bench shape (L=32, D=256, G=9) on whole site vectors.
Tolerances: 1e-11 relative for single contractions (FP64 with reductions of
a few thousand terms), 1e-8 absolute for sweep energies (the FP64 target).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from gpu_util import make_pair, rel_err  # noqa: E402

import paper_1703_04789_amd as sp  # noqa: E402
import workloads as W  # noqa: E402
from oracle import mps as omps, quadrature as oq  # noqa: E402

pytestmark = pytest.mark.gpu

CASES = [  # (L, N, 2M, D, 2S, G)
    (8, 8, 0, 16, 0, 5),
    (6, 5, 1, 12, 1, 3),
    (7, 6, 2, 20, 4, 4),
    (10, 10, 0, 48, 2, 6),
]


def _dev(a):
    return torch.tensor(a, dtype=torch.float64, device="cuda")


def _left_envs_to(gpu, orc, k):
    for j in range(1, k):
        gpu.env_update(j, +1)
        orc.update_left(j)


@pytest.mark.parametrize("case", CASES)
def test_init_right_canonical_form(case):
    tab, gpu, orc = make_pair(*case)
    for k in range(1, tab.L + 1):
        assert rel_err(gpu.get_site(k), orc.mps.site_packed(k)) < 1e-12, k
    assert gpu.center() == 1


@pytest.mark.parametrize("path", ["tiled", "plain"])
@pytest.mark.parametrize("case", CASES)
def test_heff_apply_all_sites(case, path):
    tab, gpu, orc = make_pair(*case, path=path)
    rng = np.random.default_rng(5)
    for k in range(1, tab.L + 1):
        if k > 1:
            gpu.env_update(k - 1, +1)
            orc.update_left(k - 1)
        n = gpu.site_size(k)
        x = rng.standard_normal(n)
        y_ref, ny_ref = orc.heff(k, orc.mps.dense_site(k, x))
        y_ref = orc.mps.site_packed(k, y_ref)
        ny_ref = orc.mps.site_packed(k, ny_ref)
        xd, y, ny = _dev(x), torch.empty(n, dtype=torch.float64, device="cuda"), torch.empty(
            n, dtype=torch.float64, device="cuda")
        gpu.heff_apply(k, xd, y, ny)
        torch.cuda.synchronize()
        assert rel_err(y.cpu().numpy(), y_ref) < 1e-11, k
        assert rel_err(ny.cpu().numpy(), ny_ref) < 1e-11, k
        dh, dn = torch.empty_like(y), torch.empty_like(y)
        gpu.heff_diag(k, dh, dn)
        dh_ref, dn_ref = orc.heff_diag(k)
        torch.cuda.synchronize()
        assert rel_err(dh.cpu().numpy(), orc.mps.site_packed(k, dh_ref)) < 1e-11
        assert rel_err(dn.cpu().numpy(), orc.mps.site_packed(k, dn_ref)) < 1e-11


@pytest.mark.parametrize("path", ["tiled", "plain"])
def test_heff_apply_is_deterministic(path):
    tab, gpu, orc = make_pair(*CASES[3], oracle=False, path=path)
    n = gpu.site_size(1)
    x = _dev(np.random.default_rng(0).standard_normal(n))
    outs = []
    for _ in range(3):
        y, ny = torch.empty_like(x), torch.empty_like(x)
        gpu.heff_apply(1, x, y, ny)
        torch.cuda.synchronize()
        outs.append((y.cpu().numpy(), ny.cpu().numpy()))
    for o in outs[1:]:
        assert np.array_equal(o[0], outs[0][0]) and np.array_equal(o[1], outs[0][1])


@pytest.mark.parametrize("case", CASES)
def test_energy_at_centre(case):
    tab, gpu, orc = make_pair(*case)
    E, p = gpu.energy()
    Eo, po = orc.energy(1)
    x = orc.mps.A[0]
    assert abs(E - Eo) < 1e-10
    assert abs(p - po / np.sum(x * x)) < 1e-12
    Ef, _ = orc.full_contraction()
    assert abs(E - Ef) < 1e-10


@pytest.mark.parametrize("twoS", [0, 2, 4])
def test_s2_operator_through_kernels(twoS):
    tab, gpu, orc = make_pair(6, 6, 0, 20, twoS, 4, op="s2", oracle=False)
    E, p = gpu.energy()
    s = twoS / 2
    assert p > 1e-8
    assert abs(E - s * (s + 1)) < 1e-11


@pytest.mark.parametrize("path", ["tiled", "plain"])
@pytest.mark.parametrize("case", CASES)
def test_gauge_moves_one_sweep(case, path):
    # max_iter = 1: each local solve returns its start vector, so one sweep
    # exercises every QR/LQ move and environment update of both directions
    tab, gpu, orc = make_pair(*case, path=path)
    rc, steps = gpu.sweep(1, max_iter=1)
    ref = omps.sweep(orc, 1, max_iter=1)
    for a, b in zip(steps, ref):
        assert abs(a["theta"] - b["theta"]) < 1e-10, (a, b)
    for k in range(1, tab.L + 1):
        assert rel_err(gpu.get_site(k), orc.mps.site_packed(k)) < 1e-10, k


@pytest.mark.parametrize("L,twoS,ref", [(4, 0, -1.953145308684551), (4, 2, -1.4128986959190932),
                                        (6, 0, -3.092565319505379), (6, 2, -2.6914960192367765)])
def test_sweep_full_bond_dimension_reaches_ed(L, twoS, ref):
    G = oq.exact_point_count(L, L, twoS)
    tab, gpu, orc = make_pair(L, L, 0, 4 ** (L // 2), twoS, G, oracle=False)
    rc, steps = gpu.sweep(3, max_sub=128, max_iter=200)
    assert abs(steps[-1]["theta"] - ref) < 1e-10
    E, p = gpu.energy()
    assert abs(E - ref) < 1e-10


@pytest.mark.parametrize("path", ["tiled", "plain"])
def test_sweep_small_workload_matches_oracle(path):
    # exact local solves (search space covers the local problem), so the
    # trajectory is a smooth function of the input and both sides agree
    wl = W.hubbard_small()
    tab, gpu, orc = make_pair(wl.L, wl.N, wl.twoM, wl.D, wl.twoS, wl.G, U=wl.U, seed=wl.seed, path=path)
    rc, steps = gpu.sweep(wl.sweeps, max_sub=128, max_iter=200)
    ref = omps.sweep(orc, wl.sweeps, max_sub=128, max_iter=200)
    dE = max(abs(a["theta"] - b["theta"]) for a, b in zip(steps, ref))
    assert dE < 1e-8, dE
    assert steps[-1]["theta"] > -4.235806999129714 - 1e-10


@pytest.mark.parametrize("path", ["tiled", "plain"])
def test_bench_shape_heff_parity(path):
    # L=32, U=8, D=256, G=9 (the benchmark workload): whole site vectors at the
    # first site and at the centre, plus the energy
    wl = W.hubbard_bench(0)
    tab, gpu, orc = make_pair(wl.L, wl.N, wl.twoM, wl.D, wl.twoS, wl.G, U=wl.U, seed=wl.seed, path=path)
    E, p = gpu.energy()
    Eo, po = orc.energy(1)
    assert abs(E - Eo) < 1e-9 * max(1, abs(Eo))
    rng = np.random.default_rng(7)
    kc = wl.L // 2
    for k in (1, kc):
        _left_envs_to(gpu, orc, k)  # nothing for k = 1
        n = gpu.site_size(k)
        x = rng.standard_normal(n)
        y_ref, ny_ref = orc.heff(k, orc.mps.dense_site(k, x))
        xd = _dev(x)
        y, ny = torch.empty_like(xd), torch.empty_like(xd)
        gpu.heff_apply(k, xd, y, ny)
        torch.cuda.synchronize()
        assert rel_err(y.cpu().numpy(), orc.mps.site_packed(k, y_ref)) < 1e-11
        assert rel_err(ny.cpu().numpy(), orc.mps.site_packed(k, ny_ref)) < 1e-11


def test_bond_environments_share_storage():
    # L[k] and R[k] of an interior bond live in one buffer: building L[k]
    # retires R[k], so H_eff at site k is refused until R[k] is rebuilt
    # from R[k+1], after which it again matches the oracle
    case = (8, 8, 0, 16, 0, 5)
    tab, gpu, orc = make_pair(*case)
    k = 3
    _left_envs_to(gpu, orc, k)
    rng = np.random.default_rng(17)
    x = rng.standard_normal(gpu.site_size(k))
    y_ref, ny_ref = orc.heff(k, orc.mps.dense_site(k, x))
    xd = _dev(x)
    y, ny = torch.empty_like(xd), torch.empty_like(xd)
    gpu.env_update(k, +1)
    with pytest.raises(sp.SpError) as e:
        gpu.heff_apply(k, xd, y, ny)
    assert e.value.code == sp.SP_ESTATE
    gpu.env_update(k + 1, -1)
    gpu.heff_apply(k, xd, y, ny)
    torch.cuda.synchronize()
    assert rel_err(y.cpu().numpy(), orc.mps.site_packed(k, y_ref)) < 1e-11
    assert rel_err(ny.cpu().numpy(), orc.mps.site_packed(k, ny_ref)) < 1e-11
    # the rebuilt R[k] retired L[k]: the next site's product needs it again
    with pytest.raises(sp.SpError) as e:
        gpu.heff_apply(k + 1, _dev(np.zeros(gpu.site_size(k + 1))), *(torch.empty(
            gpu.site_size(k + 1), dtype=torch.float64, device="cuda") for _ in range(2)))
    assert e.value.code == sp.SP_ESTATE


def test_zero_projected_norm_is_reported():
    # two sites, two electrons, M = 0: the MPS (|a,b> + s|b,a>) for the sign s
    # that makes it a pure triplet has no singlet component
    tab = W.make_block_table(2, 2, 0, 4)
    from oracle import ed, mpo as ompo
    st = ed.sector_states(2, 2, 0)
    P0 = ed.spin_projector_dense(ed.s2_operator(2, st), 0)
    chosen = None
    for sgn in (1.0, -1.0):
        blocks = np.zeros(tab.total_size())
        o = omps.OracleMPS(tab, blocks)
        # site 1: |b> -> (1,-1), |a> -> (1,1); site 2 completes to (2,0)
        A1 = np.zeros_like(o.A[0]); A2 = np.zeros_like(o.A[1])
        for s in (1, 2):
            for b in range(A1.shape[2]):
                if o.mask[0][s, 0, b]:
                    A1[s, 0, b] = 1.0
        for s in (1, 2):
            for a in range(A2.shape[1]):
                if o.mask[1][s, a, 0]:
                    A2[s, a, 0] = 1.0 if s == 2 else sgn
        o.A = [A1, A2]
        psi = ed.mps_to_dense(o.A)[st]
        if abs(psi @ P0 @ psi) < 1e-14 and np.linalg.norm(psi) > 0.5:
            chosen = o.packed()
    assert chosen is not None
    gpu = sp.SPMPS(tab, chosen, sp.mpo_hubbard(2, 1.0, 4.0), 0, 2)
    with pytest.raises(sp.SpError) as e:
        gpu.energy()
    assert e.value.code == sp.SP_ENORM


@pytest.mark.parametrize("path", ["tiled", "plain"])
def test_sweep_with_restarts_reaches_ed(path):
    # search space of 8 vectors (restart to 4) on a full-bond-dimension chain:
    # every local solve still converges, so the energy must reach ED
    L, twoS = 6, 0
    G = oq.exact_point_count(L, L, twoS)
    tab, gpu, orc = make_pair(L, L, 0, 64, twoS, G, oracle=False, path=path)
    rc, steps = gpu.sweep(3, max_sub=8, keep=4, max_iter=2000, tol=1e-10)
    assert abs(steps[-1]["theta"] - (-3.092565319505379)) < 1e-9


@pytest.mark.parametrize("path", ["tiled", "plain"])
def test_first_steps_with_restarts_match_oracle(path):
    # capped solves with restarts from identical inputs: the first steps agree
    # before the trajectories can separate.  The centre sites (1590 elements)
    # span two Davidson chunks while the first ones fit in one.
    tab, gpu, orc = make_pair(8, 8, 0, 64, 0, 5, U=4.0, seed=1, path=path)
    assert max(gpu.site_size(k) for k in range(1, 9)) > 1024 > gpu.site_size(1)
    rc, steps = gpu.sweep(1, max_sub=8, keep=4, max_iter=40)
    ref = omps.sweep(orc, 1, max_sub=8, keep=4, max_iter=40)
    for a, b in list(zip(steps, ref))[:5]:
        assert abs(a["theta"] - b["theta"]) < 1e-8, (a, b)


def test_autotuned_plans_keep_parity():
    # the autotuner only picks the rows per task of the fused kernel or the
    # tiled block products: the products stay equal to the oracle's at every
    # site
    tab, gpu, orc = make_pair(*CASES[3])
    choice = gpu.autotune(reps=2)
    assert len(choice) == tab.L and all((b > 0 and 1 <= r <= 8) or (b == 0 and r == 0) for b, r, _ in choice)
    rng = np.random.default_rng(9)
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
        torch.cuda.synchronize()
        assert rel_err(y.cpu().numpy(), orc.mps.site_packed(k, y_ref)) < 1e-11, k
        assert rel_err(ny.cpu().numpy(), orc.mps.site_packed(k, ny_ref)) < 1e-11, k


def test_autotune_bench_shape_runs():
    wl = W.hubbard_bench(0)
    tab, gpu, orc = make_pair(wl.L, wl.N, wl.twoM, wl.D, wl.twoS, wl.G, U=wl.U, seed=wl.seed, oracle=False)
    choice = gpu.autotune(reps=3)
    print("[autotune] site: (budget, rows, us)", {k + 1: c for k, c in enumerate(choice)})
    rc, steps = gpu.sweep(1)
    assert np.isfinite(steps[-1]["theta"])


def _largest_qr_work(tab):
    """Largest 2 rows cols over the sector factorisations of every site: QR
    of the rows gathered per right sector (right-moving) and LQ per left
    sector (left-moving).  Above 12288 doubles the factorisation runs from
    global scratch instead of LDS."""
    best = 0
    for k in range(1, tab.L + 1):
        rows_r, rows_l = {}, {}
        for ia, s, ib, r, c in tab.site_blocks(k):
            rows_r[ib] = rows_r.get(ib, 0) + r
            rows_l[ia] = rows_l.get(ia, 0) + c
        best = max([best] + [2 * r * tab.bonds[k][ib][2] for ib, r in rows_r.items()]
                   + [2 * r * tab.bonds[k - 1][ia][2] for ia, r in rows_l.items()])
    return best


@pytest.mark.parametrize("path", ["tiled", "plain"])
def test_gauge_moves_large_sectors(path):
    # L=12, D=256: some sectors are too large for the LDS-resident
    # factorisation, so those sites run the global-scratch QR/LQ kernel;
    # max_iter = 1 keeps every local solve at its start vector, and every
    # site tensor after the sweep must equal the oracle's (SVD-based) gauge
    tab, gpu, orc = make_pair(12, 12, 0, 256, 0, 4, U=4.0, seed=1, path=path)
    assert _largest_qr_work(tab) > 12288
    rc, steps = gpu.sweep(1, max_iter=1)
    assert rc == sp.SP_ENOCONV
    ref = omps.sweep(orc, 1, max_iter=1)
    assert len(steps) == len(ref) == 2 * (tab.L - 1)
    for a, b in zip(steps, ref):
        assert abs(a["theta"] - b["theta"]) < 1e-10 * max(1.0, abs(b["theta"])), (a, b)
    for k in range(1, tab.L + 1):
        assert rel_err(gpu.get_site(k), orc.mps.site_packed(k)) < 1e-10, k


@pytest.mark.parametrize("twoS", [0, 2])
def test_bench_shape_spin_targets(twoS):
    # L=32, U=8, D=256, G=9 with S=0 (seed 2) and S=1 (seed 3): energy, and
    # H_eff x, N_eff x and their diagonals at the centre site (fused plan)
    wl = W.hubbard_bench(twoS)
    tab, gpu, orc = make_pair(wl.L, wl.N, wl.twoM, wl.D, wl.twoS, wl.G, U=wl.U, seed=wl.seed)
    assert gpu.status == sp.SP_OK
    E, p = gpu.energy()
    Eo, po = orc.energy(1)
    assert abs(E - Eo) < 1e-9 * max(1, abs(Eo))
    kc = wl.L // 2
    _left_envs_to(gpu, orc, kc)
    n = gpu.site_size(kc)
    x = np.random.default_rng(11 + twoS).standard_normal(n)
    y_ref, ny_ref = orc.heff(kc, orc.mps.dense_site(kc, x))
    xd = _dev(x)
    y, ny = torch.empty_like(xd), torch.empty_like(xd)
    gpu.heff_apply(kc, xd, y, ny)
    dh, dn = torch.empty_like(xd), torch.empty_like(xd)
    gpu.heff_diag(kc, dh, dn)
    torch.cuda.synchronize()
    assert rel_err(y.cpu().numpy(), orc.mps.site_packed(kc, y_ref)) < 1e-11
    assert rel_err(ny.cpu().numpy(), orc.mps.site_packed(kc, ny_ref)) < 1e-11
    dh_ref, dn_ref = orc.heff_diag(kc)
    assert rel_err(dh.cpu().numpy(), orc.mps.site_packed(kc, dh_ref)) < 1e-11
    assert rel_err(dn.cpu().numpy(), orc.mps.site_packed(kc, dn_ref)) < 1e-11


def test_status_inexact_quadrature():
    # one point below the exact count of Eq. [exactQuadrature]: the state is
    # built (the projector is approximate) and the warning is returned
    L, N, twoS = 6, 6, 2
    G = sp.exact_points(N, L, twoS)
    assert G == oq.exact_point_count(N, L, twoS)
    _, exact, _ = make_pair(L, N, 0, 16, twoS, G, oracle=False)
    assert exact.status == sp.SP_OK
    _, short, _ = make_pair(L, N, 0, 16, twoS, G - 1, oracle=False)
    assert short.status == sp.SP_WINEXACT
    E, p = short.energy()
    assert np.isfinite(E) and p > 0


def test_status_unconverged_sweep():
    # a single Ritz evaluation per local solve cannot meet the tolerance
    # (SP_ENOCONV); exact local solves on the same state do
    tab, gpu, _ = make_pair(6, 6, 0, 16, 0, 4, oracle=False)
    rc, steps = gpu.sweep(1, max_iter=1)
    assert rc == sp.SP_ENOCONV and not any(s["converged"] for s in steps)
    rc, steps = gpu.sweep(1, max_sub=128, max_iter=200)
    assert rc == sp.SP_OK and all(s["converged"] for s in steps)


def test_verbose_sweep_prints_one_line_per_step(capfd):
    # the library reports every finished site step on stderr when asked, in
    # the order of the step reports, and stays silent otherwise
    tab, gpu, _ = make_pair(6, 6, 0, 16, 0, 4, oracle=False)
    rc, steps = gpu.sweep(1, verbose=True)
    err = capfd.readouterr().err
    lines = [ln for ln in err.splitlines() if ln.startswith("[sp_sweep]")]
    assert len(lines) == len(steps) == 2 * (tab.L - 1)
    for ln, st in zip(lines, steps):
        assert f"site {st['site']} dir {st['dir']:+d}" in ln and f"theta {st['theta']:.12f}" in ln
    gpu.sweep(1)
    assert not [ln for ln in capfd.readouterr().err.splitlines() if ln.startswith("[sp_sweep]")]
