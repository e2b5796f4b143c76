"""Excited states through orthogonality constraints (Sec. 2.3, Eq.
[orthoB]) on the HIP path, against the FP64 oracle and exact
diagonalisation.

The lower state enters both sides as the same seeded site tensors (each side
keeps its own gauge of it; B[k] depends only on the state).  Tolerances:
1e-11 for overlaps of unit-norm states, 1e-8 for sweep energies (exact
local solves), 1e-9 against exact levels at full bond dimension."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from gpu_util import make_pair  # noqa: E402

import paper_1703_04789_amd as sp  # noqa: E402
import workloads as W  # noqa: E402
from oracle import ed, mpo as ompo, mps as omps, quadrature as oq  # noqa: E402

pytestmark = pytest.mark.gpu


def _levels(L, twoS, U, n=3):
    st = ed.sector_states(L, L, 0)
    H = ed.hubbard_hamiltonian(L, 1.0, U, st).toarray()
    ev, vec = np.linalg.eigh(ed.s2_operator(L, st).toarray())
    s = twoS / 2
    Z = vec[:, np.abs(ev - s * (s + 1)) < 1e-8]
    return np.linalg.eigvalsh(Z.T @ H @ Z)[:n]


@pytest.mark.parametrize("path", ["tiled", "plain"])
@pytest.mark.parametrize("case", [(6, 6, 0, 16, 0, 4), (7, 6, 2, 20, 2, 4)])
def test_overlap_and_constrained_sweep_match_oracle(case, path):
    L, N, twoM, D, twoS, G = case
    tab = W.make_block_table(L, N, twoM, D)
    b0 = W.random_blocks(tab, 31)
    print(f"[case] excited L={L} N={N} 2M={twoM} D={D} 2S={twoS} G={G} {path}", flush=True)
    lower = sp.SPMPS(tab, b0, sp.mpo_hubbard(L, 1.0, 4.0), twoS, G, path=path)
    tab, gpu, orc = make_pair(L, N, twoM, D, twoS, G, seed=32, path=path)
    gpu.add_orthogonality(lower)
    c = omps.OrthogonalityConstraint(orc, tab, b0)
    # normalised overlap; the oracle keeps the lower state as given
    nrm0 = float(np.linalg.norm(ed.mps_to_dense(c.psi0.A)))
    ov_gpu = gpu.orthogonality_overlaps()
    ov_orc = c.overlap(1) / nrm0 / float(np.sqrt(np.sum(orc.mps.A[0] ** 2)))
    assert abs(ov_gpu[0] - ov_orc) < 1e-11 * max(1.0, abs(ov_orc)), (ov_gpu, ov_orc)
    rc, steps = gpu.sweep(2, max_sub=128, max_iter=200)
    ref = omps.sweep(orc, 2, max_sub=128, max_iter=200, constraints=[c])
    dE = max(abs(a["theta"] - b["theta"]) for a, b in zip(steps, ref))
    assert dE < 1e-8, dE
    assert abs(gpu.orthogonality_overlaps()[0]) < 1e-10


@pytest.mark.parametrize("L,twoS", [(4, 0), (4, 2), (6, 0)])
def test_excited_states_at_full_bond_dimension_reach_exact_levels(L, twoS):
    U = 4.0
    ref = _levels(L, twoS, U)
    G = oq.exact_point_count(L, L, twoS)
    D = 4 ** (L // 2)
    tab = W.make_block_table(L, L, 0, D)
    mpo = sp.mpo_hubbard(L, 1.0, U)
    print(f"[case] excited full D L={L} 2S={twoS}", flush=True)
    s0 = sp.SPMPS(tab, W.random_blocks(tab, 1), mpo, twoS, G)
    rc, st0 = s0.sweep(3, max_sub=128, max_iter=200)
    assert abs(st0[-1]["theta"] - ref[0]) < 1e-9
    s1 = sp.SPMPS(tab, W.random_blocks(tab, 2), mpo, twoS, G)
    s1.add_orthogonality(s0)
    rc, st1 = s1.sweep(4, max_sub=128, max_iter=200)
    assert abs(st1[-1]["theta"] - ref[1]) < 1e-9, (st1[-1]["theta"], ref)
    assert abs(s1.orthogonality_overlaps()[0]) < 1e-10
    if L == 4 and twoS == 0:
        # second excited state: two constraints
        s2 = sp.SPMPS(tab, W.random_blocks(tab, 3), mpo, twoS, G)
        s2.add_orthogonality(s0)
        s2.add_orthogonality(s1)
        rc, st2 = s2.sweep(4, max_sub=128, max_iter=200)
        assert abs(st2[-1]["theta"] - ref[2]) < 1e-9, (st2[-1]["theta"], ref)
        assert np.abs(s2.orthogonality_overlaps()).max() < 1e-10


def test_constraints_reject_mismatched_states_and_batches():
    tab = W.make_block_table(6, 6, 0, 16)
    s0 = sp.SPMPS(tab, W.random_blocks(tab, 1), sp.mpo_hubbard(6, 1.0, 4.0), 0, 4)
    other = W.make_block_table(6, 6, 0, 12)
    s1 = sp.SPMPS(other, W.random_blocks(other, 2), sp.mpo_hubbard(6, 1.0, 4.0), 0, 4)
    with pytest.raises(sp.SpError):
        s1.add_orthogonality(s0)
    s2 = sp.SPMPS(tab, W.random_blocks(tab, 3), sp.mpo_hubbard(6, 1.0, 4.0), 0, 4)
    s2.add_orthogonality(s0)
    with pytest.raises(sp.SpError):
        sp.sweep_batch([s2, s0], 1)
    s2.clear_orthogonality()
    rc, st = sp.sweep_batch([s2, s0], 1)
    assert len(st) == 2


def test_abinitio_first_excited_state_at_full_bond_dimension():
    K, N, twoS = 4, 4, 0
    h, eri = W.abinitio_integrals(K, seed=4)
    st = ed.sector_states(K, N, 0)
    H = ed.abinitio_hamiltonian(h, eri, st).toarray()
    ev, vec = np.linalg.eigh(ed.s2_operator(K, st).toarray())
    Z = vec[:, np.abs(ev) < 1e-8]
    ref = np.linalg.eigvalsh(Z.T @ H @ Z)[:2]
    G = oq.exact_point_count(N, K, twoS)
    tab = W.make_block_table(K, N, 0, 16)
    mpo = sp.mpo_abinitio(h, eri)
    print("[case] ab-initio excited K=4", flush=True)
    s0 = sp.SPMPS(tab, W.random_blocks(tab, 1), mpo, twoS, G)
    s0.sweep(3, max_sub=128, max_iter=200)
    s1 = sp.SPMPS(tab, W.random_blocks(tab, 2), mpo, twoS, G)
    s1.add_orthogonality(s0)
    rc, steps = s1.sweep(4, max_sub=128, max_iter=200)
    assert abs(steps[-1]["theta"] - ref[1]) < 1e-9, (steps[-1]["theta"], ref)
    assert abs(s1.orthogonality_overlaps()[0]) < 1e-10
