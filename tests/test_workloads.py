"""The seeded input generators (no method arithmetic): the Neel-type guesses
of the batched runs are the product states they claim to be."""
import numpy as np

import workloads as W
from oracle import ed, mps as omps  # noqa: F401


def test_neel_blocks_is_the_product_state():
    L = 6
    tab = W.make_block_table(L, L, 0, 16)
    blocks = W.neel_blocks(tab, seed=3, noise=0.0)
    m = omps.OracleMPS(tab, blocks)
    psi = ed.mps_to_dense(m.A)
    # exactly one basis state carries the weight: alpha on odd sites, beta on
    # even sites (sigma = 2 n_alpha + n_beta)
    nz = np.flatnonzero(np.abs(psi) > 1e-12)
    assert len(nz) == 1
    occ = [(int(nz[0]) >> (2 * (L - k))) & 3 for k in range(1, L + 1)]
    assert occ == [2 if k % 2 else 1 for k in range(1, L + 1)]
    assert abs(abs(psi[nz[0]]) - 1.0) < 1e-12

def test_neel_noise_is_seeded_and_small():
    tab = W.make_block_table(8, 8, 0, 16)
    a = W.neel_blocks(tab, seed=5)
    b = W.neel_blocks(tab, seed=5)
    np.testing.assert_array_equal(a, b)
    base = W.neel_blocks(tab, seed=5, noise=0.0)
    assert np.count_nonzero(base) == 8
    assert np.abs(a - base).max() < 0.1


def test_batch_instances_follow_the_recipe():
    ins = W.hubbard_batch(16)
    assert len({w.seed for w in ins}) == 16
    for w in ins:
        assert 12 <= w.L <= 32 and w.L % 2 == 0 and w.N == w.L
        assert w.U in (4.0, 8.0) and w.D in (64, 128, 256, 512) and w.G == 9 and w.twoS == 0
