"""sp_heff_apply_noalloc (the allocation-free H_eff x) against sp_heff_apply
through the C ABI: the same kernels run in the same order, so the outputs
must agree bit for bit.  Two calls in a row, the second on a smaller input,
on a fused-kernel site and on a block-product site."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from gpu_util import make_pair  # noqa: E402

import paper_1703_04789_amd as sp  # noqa: E402

pytestmark = pytest.mark.gpu


def _apply(gpu, k, x, noalloc):
    xd = torch.tensor(x, dtype=torch.float64, device="cuda")
    y = torch.full_like(xd, np.nan)
    ny = torch.full_like(xd, np.nan)
    (gpu.heff_apply_noalloc if noalloc else gpu.heff_apply)(k, xd, y, ny)
    torch.cuda.synchronize()
    return y.cpu().numpy(), ny.cpu().numpy()


@pytest.mark.parametrize("tiled_products", [False, True])
def test_noalloc_matches_heff_apply(tiled_products):
    # state A: L=10, D=48 (centre site), then state B: L=6, D=16 (a smaller
    # site), each call checked against the allocating entry point
    rng = np.random.default_rng(21)
    for (L, N, twoM, D, twoS, G) in [(10, 10, 0, 48, 2, 6), (6, 6, 0, 16, 0, 4)]:
        _, gpu, _ = make_pair(L, N, twoM, D, twoS, G, oracle=False)
        k = L // 2
        for j in range(1, k):
            gpu.env_update(j, +1)
        if tiled_products:
            assert gpu.set_heff_plan(k, 0) == 0
        else:
            assert gpu.heff_plan(k)[0] > 0
        x = rng.standard_normal(gpu.site_size(k))
        y0, ny0 = _apply(gpu, k, x, False)
        y1, ny1 = _apply(gpu, k, x, True)
        assert np.all(np.isfinite(y1)) and np.all(np.isfinite(ny1))
        assert np.array_equal(y0, y1) and np.array_equal(ny0, ny1), (L, D)
        gpu.close()


def test_noalloc_rejects_plain_path():
    _, gpu, _ = make_pair(6, 6, 0, 16, 0, 4, oracle=False, path="plain")
    x = torch.zeros(gpu.site_size(1), dtype=torch.float64, device="cuda")
    with pytest.raises(sp.SpError) as e:
        gpu.heff_apply_noalloc(1, x, torch.empty_like(x), torch.empty_like(x))
    assert e.value.code == sp.SP_EINVAL
