"""Spin-free properties (Sec. 2.4, Eq. [PropSpinFree]) in the oracle and the
library's operator builders.

Pins: the operator MPOs contract to the Jordan-Wigner operators built
independently on the (N, M) sector; sum_{X,Y} S_X.S_Y is the total S^2;
the oracle's projected expectation equals <psi|O P|psi>/<psi|P|psi> with the
exact spin projector at a fixed random MPS; sum_p <E_pp> = N,
sum_{XY} <S_X.S_Y> = S(S+1), and the energy components add up to the energy.
"""
import numpy as np
import pytest

import paper_1703_04789_amd as sp
import workloads as W
from oracle import ed, mpo as om, mps as omps, quadrature as oq


def _sector_dense(Ws, states):
    return om.mpo_to_dense(Ws)[np.ix_(states, states)]


@pytest.mark.parametrize("L,N,twoM", [(4, 4, 0), (4, 3, 1), (5, 4, 2)])
def test_operator_mpos_are_the_jordan_wigner_operators(L, N, twoM):
    st = ed.sector_states(L, N, twoM)
    for p in range(1, L + 1):
        for q in range(1, L + 1):
            if p == q:
                ref = np.diag([((i >> ed._bit(L, p, 0)) & 1) + ((i >> ed._bit(L, p, 1)) & 1) for i in st]).astype(float)
            else:
                ref = ed.epq_operator(L, p, q, st).toarray()
            assert np.abs(_sector_dense(om.epq_mpo(L, p, q), st) - ref).max() < 1e-14, (p, q)
            sref = ed.spin_corr_operator(L, p, q, st).toarray()
            assert np.abs(_sector_dense(om.spin_corr_mpo(L, p, q), st) - sref).max() < 1e-14, (p, q)


def test_spin_correlations_add_up_to_s2():
    L = 5
    st = ed.sector_states(L, 5, 1)
    tot = sum(ed.spin_corr_operator(L, X, Y, st) for X in range(1, L + 1) for Y in range(1, L + 1))
    assert np.abs(tot.toarray() - ed.s2_operator(L, st).toarray()).max() < 1e-13


@pytest.mark.parametrize("twoS", [0, 2])
def test_oracle_expectation_is_the_projected_ratio(twoS):
    L, N = 4, 4
    tab = W.make_block_table(L, N, 0, 16)
    blocks = W.random_blocks(tab, 11)
    G = oq.exact_point_count(N, L, twoS)
    st = ed.sector_states(L, N, 0)
    P = ed.spin_projector_dense(ed.s2_operator(L, st), twoS)
    psi = ed.mps_to_dense(omps.OracleMPS(tab, blocks).A)[st]
    for Ws, dense in ((om.epq_mpo(L, 1, 3), ed.epq_operator(L, 1, 3, st)),
                      (om.epq_mpo(L, 4, 2), ed.epq_operator(L, 4, 2, st)),
                      (om.spin_corr_mpo(L, 2, 3), ed.spin_corr_operator(L, 2, 3, st))):
        val, _ = omps.expect(tab, blocks, Ws, twoS, G)
        ref, _ = ed.projected_energy(psi, dense.toarray(), P)
        assert abs(val - ref) < 1e-11


def test_property_sum_rules_at_a_random_state():
    L, N, twoS = 6, 6, 2
    tab = W.make_block_table(L, N, 0, 24)
    blocks = W.random_blocks(tab, 4)
    G = oq.exact_point_count(N, L, twoS)
    n_tot = sum(omps.expect(tab, blocks, om.epq_mpo(L, p, p), twoS, G)[0] for p in range(1, L + 1))
    assert abs(n_tot - N) < 1e-10
    ss = sum(omps.expect(tab, blocks, om.spin_corr_mpo(L, x, y), twoS, G)[0]
             for x in range(1, L + 1) for y in range(1, L + 1))
    assert abs(ss - 2.0) < 1e-10  # S(S+1) for S = 1
    t, U = 1.0, 4.0
    E, _ = omps.expect(tab, blocks, om.hubbard_mpo(L, t, U), twoS, G)
    dbl = np.zeros((4, 4))
    dbl[3, 3] = 1.0
    e = 0.0
    for p in range(1, L + 1):
        e += U * omps.expect(tab, blocks, om.site_op_mpo(L, p, dbl), twoS, G)[0]
        for q in (p - 1, p + 1):
            if 1 <= q <= L:
                e += -t * omps.expect(tab, blocks, om.epq_mpo(L, p, q), twoS, G)[0]
    assert abs(e - E) < 1e-10


def _unpack(L, mpo):
    w, data = mpo
    out, pos = [], 0
    for k in range(1, L + 1):
        n = int(w[k - 1]) * int(w[k]) * 16
        out.append(np.asarray(data[pos:pos + n]).reshape(int(w[k - 1]), int(w[k]), 4, 4))
        pos += n
    return out


@pytest.mark.parametrize("L", [1, 2, 5])
def test_library_operator_builders_match_the_oracle(L):
    op = np.arange(16, dtype=float).reshape(4, 4) / 7.0
    for p in range(1, L + 1):
        for q in range(1, L + 1):
            for mine, ref in ((sp.mpo_epq(L, p, q), om.epq_mpo(L, p, q)),
                              (sp.mpo_spin_corr(L, p, q), om.spin_corr_mpo(L, p, q))):
                for a, b in zip(_unpack(L, mine), ref):
                    assert a.shape == b.shape and np.abs(a - b).max() < 1e-15
        for a, b in zip(_unpack(L, sp.mpo_site_op(L, p, op)), om.site_op_mpo(L, p, op)):
            assert a.shape == b.shape and np.abs(a - b).max() < 1e-15


def _nn(L, p, st):
    """n_{p alpha} n_{p beta} on the sector basis (diagonal)."""
    a, b = ed._bit(L, p, 0), ed._bit(L, p, 1)
    return np.diag([float(((i >> a) & 1) and ((i >> b) & 1)) for i in st])


@pytest.mark.parametrize("L,N,twoM", [(4, 4, 0), (5, 4, 2)])
def test_hubbard_components_are_the_site_terms(L, N, twoM):
    # H_p of the Hubbard chain = -t sum_s (a+_ps a_{p+1,s} + a+_ps a_{p-1,s})
    # + U n_pa n_pb, built independently from the occupation-number operators
    t, U = 1.3, 3.7
    st = ed.sector_states(L, N, twoM)
    h, eri = om.hubbard_integrals(L, t, U)
    tot = np.zeros((len(st), len(st)))
    for p in range(1, L + 1):
        ref = U * _nn(L, p, st)
        for q in (p - 1, p + 1):
            if 1 <= q <= L:
                ref = ref - t * ed.epq_operator(L, p, q, st).toarray()
        got = _sector_dense(om.abinitio_component_mpo(h, eri, p), st)
        assert np.abs(got - ref).max() < 1e-13, p
        tot += got
    assert np.abs(tot - ed.hubbard_hamiltonian(L, t, U, st).toarray()).max() < 1e-13


def test_abinitio_components_add_up_to_the_hamiltonian():
    K = 4
    h, eri = W.abinitio_integrals(K, 7)
    for (N, twoM) in [(4, 0), (3, 1)]:
        st = ed.sector_states(K, N, twoM)
        tot = sum(_sector_dense(om.abinitio_component_mpo(h, eri, p), st) for p in range(1, K + 1))
        ref = ed.abinitio_hamiltonian(h, eri, st).toarray()
        assert np.abs(tot - ref).max() < 1e-12


@pytest.mark.parametrize("K", [3, 4])
def test_library_component_mpos_match_the_oracle(K):
    # different automata on each side: compared as operators on every
    # (N, M) sector
    h, eri = W.abinitio_integrals(K, 3)
    for p in range(1, K + 1):
        a = om.mpo_to_dense(_unpack(K, sp.mpo_abinitio_component(h, eri, p)))
        b = om.mpo_to_dense(om.abinitio_component_mpo(h, eri, p))
        assert np.abs(a - b).max() < 1e-12, p
        hh, ee = om.hubbard_integrals(K, 1.0, 4.0)
        a = om.mpo_to_dense(_unpack(K, sp.mpo_hubbard_component(K, p, 1.0, 4.0)))
        b = om.mpo_to_dense(om.abinitio_component_mpo(hh, ee, p))
        assert np.abs(a - b).max() < 1e-13, p
    with pytest.raises(sp.SpError):
        sp.mpo_abinitio_component(h, eri, K + 1)


def test_energy_components_sum_to_the_energy_at_a_random_state():
    L, N, twoS = 6, 6, 2
    tab = W.make_block_table(L, N, 0, 24)
    blocks = W.random_blocks(tab, 4)
    G = oq.exact_point_count(N, L, twoS)
    h, eri = om.hubbard_integrals(L, 1.0, 4.0)
    E, _ = omps.expect(tab, blocks, om.hubbard_mpo(L, 1.0, 4.0), twoS, G)
    e = [omps.expect(tab, blocks, om.abinitio_component_mpo(h, eri, p), twoS, G)[0] for p in range(1, L + 1)]
    assert abs(sum(e) - E) < 1e-10

