"""Shared set-up of the GPU parity tests: one seeded workload fed to both the
HIP library (through its C ABI) and the oracle."""
import numpy as np

import paper_1703_04789_amd as sp
import workloads as W
from oracle import mpo as ompo, mps as omps


def make_pair(L, N, twoM, D, twoS, G, U=4.0, t=1.0, seed=1, op="hubbard", oracle=True, path="tiled",
              precision="fp64", integrals=None):
    tab = W.make_block_table(L, N, twoM, D)
    blocks = W.random_blocks(tab, seed)
    if op == "abinitio":  # integrals = (h, eri); each side builds its own MPO
        mine, ref = sp.mpo_abinitio(*integrals), (ompo.abinitio_mpo(*integrals) if oracle else None)
    elif op == "hubbard":
        mine, ref = sp.mpo_hubbard(L, t, U), ompo.hubbard_mpo(L, t, U)
    elif op == "s2":
        mine, ref = sp.mpo_s2(L), ompo.s2_mpo(L)
    else:
        mine, ref = sp.mpo_identity(L), ompo.identity_mpo(L)
    print(f"[case] L={L} N={N} 2M={twoM} D={D} 2S={twoS} G={G} seed={seed} op={op} path={path} {precision}",
          flush=True)
    gpu = sp.SPMPS(tab, blocks, mine, twoS, G, path=path, precision=precision)
    orc = omps.SPMPSOracle(tab, blocks, ref, twoS, G) if oracle else None
    return tab, gpu, orc


def rel_err(a, b):
    scale = max(np.abs(b).max(), 1e-300)
    return np.abs(a - b).max() / scale
