"""Seeded synthetic inputs shared by the CPU oracle and the HIP library.

This module holds no arithmetic of the spin-projected method itself.  It only
produces the *inputs* both sides consume:

* the bond block table of a matrix product state with Abelian (N, 2M)
  quantum numbers (which sectors each bond carries and how many states each
  sector keeps), and
* seeded N(0, 1) initial site tensors in the canonical packed block order,
* named workload descriptions (Hubbard chain parameters, bond dimension,
  number of quadrature points, number of sweeps, seeds).

Conventions (shared interface, stated once here):

* Sites are spatial orbitals k = 1..L with local basis index
  sigma = 2*n_alpha + n_beta, i.e. (|0>, |b>, |a>, |ab>).  The local quantum
  numbers (N, 2M) of sigma = 0, 1, 2, 3 are (0,0), (1,-1), (1,+1), (2,0).
* Bond k (k = 0..L) sits to the right of site k; its sector label q = (N, 2M)
  counts the particles and twice the spin projection of sites 1..k.  Bond 0
  is the single sector (0, 0) of dimension 1; bond L is the single sector
  (N, 2M) of dimension 1.
* Within a bond, sectors are sorted by (N, 2M) ascending; the states of one
  sector are contiguous, so the states of one particle number N form one
  contiguous range of the bond index.
* Site tensor A[k] is stored as blocks, one per pair (left sector a of bond
  k-1, sigma) whose right sector b = a + q_sigma exists in bond k.  Blocks are
  ordered by left-sector index, then sigma; each block is a dense
  dim(a) x dim(b) row-major matrix.  Sites are concatenated k = 1..L.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# local quantum numbers (N, 2M) of sigma = 2*n_alpha + n_beta
SIGMA_QN = ((0, 0), (1, -1), (1, 1), (2, 0))
D_LOCAL = 4


@dataclass
class BlockTable:
    """Bond sectors of an (N, 2M)-symmetric MPS.

    ``bonds[k]`` is a list of (N, twoM, dim) tuples sorted by (N, twoM).
    """

    L: int
    N: int
    twoM: int
    bonds: list = field(default_factory=list)

    def bond_dim(self, k: int) -> int:
        return sum(s[2] for s in self.bonds[k])

    def max_bond_dim(self) -> int:
        return max(self.bond_dim(k) for k in range(self.L + 1))

    def site_blocks(self, k: int):
        """Blocks of site k (1-based) in canonical order.

        Returns a list of (ia, sigma, ib, rows, cols) with sector indices into
        bonds[k-1] and bonds[k].
        """
        left = self.bonds[k - 1]
        right = self.bonds[k]
        index_r = {(n, m): i for i, (n, m, _) in enumerate(right)}
        out = []
        for ia, (n, m, da) in enumerate(left):
            for s, (dn, dm) in enumerate(SIGMA_QN):
                ib = index_r.get((n + dn, m + dm))
                if ib is not None:
                    out.append((ia, s, ib, da, right[ib][2]))
        return out

    def site_size(self, k: int) -> int:
        return sum(r * c for (_, _, _, r, c) in self.site_blocks(k))

    def total_size(self) -> int:
        return sum(self.site_size(k) for k in range(1, self.L + 1))

    # flat arrays in the layout the C library takes
    def flat(self):
        nsec = np.array([len(b) for b in self.bonds], dtype=np.int32)
        sec = np.array([s for b in self.bonds for s in b], dtype=np.int32).reshape(-1, 3)
        return nsec, np.ascontiguousarray(sec[:, 0]), np.ascontiguousarray(sec[:, 1]), \
            np.ascontiguousarray(sec[:, 2])


def _sector_count(nsites: int, na: int, nb: int) -> int:
    """Number of occupation states of nsites spatial orbitals with na alpha and
    nb beta electrons."""
    if na < 0 or nb < 0 or na > nsites or nb > nsites:
        return 0
    return math.comb(nsites, na) * math.comb(nsites, nb)


def _allocate(weights, caps, total):
    """Water-filling allocation of ``total`` states over sectors in proportion
    to ``weights``, each capped at ``caps``; largest-remainder rounding."""
    weights = np.asarray(weights, dtype=float)
    caps = np.asarray(caps, dtype=float)
    n = len(weights)
    alloc = np.zeros(n)
    free = np.ones(n, dtype=bool)
    remaining = float(min(total, caps.sum()))
    for _ in range(n + 1):
        w = np.where(free, weights, 0.0)
        if remaining <= 0 or w.sum() == 0:
            break
        share = remaining * w / w.sum()
        over = free & (alloc + share > caps)
        if not over.any():
            alloc += share
            remaining = 0.0
            break
        remaining -= (caps[over] - alloc[over]).sum()
        alloc[over] = caps[over]
        free &= ~over
    target = int(round(min(total, caps.sum())))
    base = np.floor(alloc + 1e-9).astype(int)
    base = np.minimum(base, caps.astype(int))
    rem = alloc - base
    order = np.argsort(-rem, kind="stable")
    short = target - base.sum()
    for i in order:
        if short <= 0:
            break
        if base[i] < caps[i]:
            base[i] += 1
            short -= 1
    return base


def make_block_table(L: int, N: int, twoM: int, D: int) -> BlockTable:
    """Bond sectors for an L-site chain with N electrons and spin projection
    twoM/2, keeping at most D states per bond.

    Each bond distributes its D states over the sectors (N_l, 2M_l) in
    proportion to dim_left * dim_right (the number of occupation states that
    realise the sector on each side), each sector capped at
    min(dim_left, dim_right).  The table is then made consistent: every
    sector keeps no more states than the neighbouring bonds can reach through
    one site.
    """
    if (N + twoM) % 2 != 0 or abs(twoM) > N:
        raise ValueError("N and twoM must have equal parity and |twoM| <= N")
    na_tot = (N + twoM) // 2
    nb_tot = (N - twoM) // 2
    if na_tot > L or nb_tot > L:
        raise ValueError("too many electrons of one spin for L orbitals")
    bonds = [[(0, 0, 1)]]
    for k in range(1, L):
        secs, w, caps = [], [], []
        for na in range(0, min(k, na_tot) + 1):
            for nb in range(0, min(k, nb_tot) + 1):
                dl = _sector_count(k, na, nb)
                dr = _sector_count(L - k, na_tot - na, nb_tot - nb)
                if dl == 0 or dr == 0:
                    continue
                secs.append((na + nb, na - nb))
                w.append(float(dl) * float(dr))
                caps.append(min(dl, dr))
        dims = _allocate(w, caps, D)
        bond = sorted((n, m, int(d)) for (n, m), d in zip(secs, dims) if d > 0)
        bonds.append(bond)
    bonds.append([(N, twoM, 1)])

    # consistency: a sector cannot hold more states than reachable from
    # either neighbour bond through one site
    def reach(bond_from, q, sign):
        tab = {(n, m): d for (n, m, d) in bond_from}
        return sum(tab.get((q[0] - sign * dn, q[1] - sign * dm), 0) for dn, dm in SIGMA_QN)

    for _ in range(4 * L):
        changed = False
        for k in range(1, L):
            nb = []
            for (n, m, d) in bonds[k]:
                lim = min(reach(bonds[k - 1], (n, m), +1), reach(bonds[k + 1], (n, m), -1))
                if lim < d:
                    changed = True
                    d = lim
                if d > 0:
                    nb.append((n, m, d))
                else:
                    changed = True
            bonds[k] = nb
        if not changed:
            break
    return BlockTable(L=L, N=N, twoM=twoM, bonds=bonds)


def random_blocks(table: BlockTable, seed: int) -> np.ndarray:
    """Seeded N(0,1) entries for every site block, in canonical packed order."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(table.total_size())


def neel_blocks(table: BlockTable, seed: int, noise: float = 1e-2) -> np.ndarray:
    """A broken-symmetry Neel-type product state embedded in the block table:
    site k holds an alpha electron for odd k and a beta electron for even k
    (N = L, N_alpha = N_beta for even L), i.e. entry (0, 0) of the block
    (left sector of the product state's prefix, sigma_k) is 1, plus seeded
    noise * N(0, 1) on every stored entry."""
    rng = np.random.default_rng(seed)
    out = noise * rng.standard_normal(table.total_size())
    off = 0
    n, m2 = 0, 0
    for k in range(1, table.L + 1):
        s_k = 2 if k % 2 == 1 else 1  # |a> on odd sites, |b> on even sites
        left = table.bonds[k - 1]
        pos = off
        for (ia, s, ib, r, c) in table.site_blocks(k):
            if s == s_k and left[ia][0] == n and left[ia][1] == m2:
                out[pos] += 1.0
            pos += r * c
        off = pos
        n += SIGMA_QN[s_k][0]
        m2 += SIGMA_QN[s_k][1]
    return out


def site_offsets(table: BlockTable):
    """Start of each site (1..L) in the concatenated packed array."""
    offs = [0]
    for k in range(1, table.L + 1):
        offs.append(offs[-1] + table.site_size(k))
    return offs


# ---------------------------------------------------------------------------
# Named workloads.  Hubbard chains: open boundary, hopping t, on-site U.


@dataclass
class HubbardWorkload:
    name: str
    L: int
    t: float
    U: float
    N: int
    twoS: int
    twoM: int
    D: int
    G: int
    sweeps: int
    seed: int
    init: str = "random"  # "random": N(0,1) entries; "neel": product state + noise
    noise: float = 1e-2

    def table(self) -> BlockTable:
        return make_block_table(self.L, self.N, self.twoM, self.D)

    def blocks(self) -> np.ndarray:
        if self.init == "neel":
            return neel_blocks(self.table(), self.seed, self.noise)
        return random_blocks(self.table(), self.seed)


def hubbard_small() -> HubbardWorkload:
    """1D Hubbard, L=8, t=1, U=4, N=8, M=0, S=0, D=16, G=5, 4 sweeps."""
    return HubbardWorkload("hubbard_L8_D16_G5", L=8, t=1.0, U=4.0, N=8, twoS=0, twoM=0,
                           D=16, G=5, sweeps=4, seed=1)


def hubbard_bench(twoS: int = 0) -> HubbardWorkload:
    """1D Hubbard, L=32, t=1, U=8, N=32, M=0, S=0 (seed 2) or S=1 (seed 3),
    D=256, G=9, 4 sweeps."""
    return HubbardWorkload(f"hubbard_L32_D256_G9_S{twoS // 2}", L=32, t=1.0, U=8.0, N=32,
                           twoS=twoS, twoM=0, D=256, G=9, sweeps=4,
                           seed=2 if twoS == 0 else 3)


def hubbard_batch(n: int = 64, seed0: int = 100, D_choices=(64, 128, 256, 512)) -> list:
    """Broken-symmetry guesses for many independent runs: instance i (seed
    seed0 + i) draws an even L in [12, 32], U in {4, 8} and D from D_choices;
    half filling N = L, M = 0, S = 0, G = 9, Neel-type initial state with
    1e-2 noise."""
    out = []
    for i in range(n):
        rng = np.random.default_rng(seed0 + i)
        L = int(rng.choice(np.arange(12, 33, 2)))
        U = float(rng.choice([4.0, 8.0]))
        D = int(rng.choice(list(D_choices)))
        out.append(HubbardWorkload(f"hubbard_batch{i}_L{L}_U{int(U)}_D{D}", L=L, t=1.0, U=U, N=L, twoS=0, twoM=0,
                                   D=D, G=9, sweeps=4, seed=seed0 + i, init="neel", noise=1e-2))
    return out


# ---------------------------------------------------------------------------
# Synthetic ab-initio-shaped Hamiltonians (real orbitals, chemists' notation).


def abinitio_integrals(K: int, seed: int, rank: int | None = None, decay: float = 4.0):
    """Seeded one- and two-electron integrals of K spatial orbitals.

    h_pq = h_qp = g_pq exp(-|p-q|/decay) with g_pq ~ N(0, 1) (upper triangle
    drawn, mirrored).  (pq|rs) = sum_l B^l_pq B^l_rs over ``rank`` (default
    2K) symmetric factors B^l_pq = g^l_pq exp(-|p-q|/decay) / sqrt(rank), so
    the tensor has the 8-fold permutational symmetry of real orbitals and is
    positive semidefinite as a (pq),(rs) matrix.  Returns (h, eri) with eri
    indexed [p, q, r, s] = (pq|rs)."""
    rank = 2 * K if rank is None else rank
    rng = np.random.default_rng(seed)
    idx = np.arange(K)
    env = np.exp(-np.abs(idx[:, None] - idx[None, :]) / decay)

    def sym(a):
        return np.triu(a) + np.triu(a, 1).T

    h = sym(rng.standard_normal((K, K))) * env
    B = np.stack([sym(rng.standard_normal((K, K))) * env for _ in range(rank)]) / math.sqrt(rank)
    eri = np.einsum("lpq,lrs->pqrs", B, B)
    return np.ascontiguousarray(h), np.ascontiguousarray(eri)


@dataclass
class AbInitioWorkload:
    name: str
    K: int
    N: int
    twoS: int
    twoM: int
    D: int
    G: int
    sweeps: int
    seed: int

    def integrals(self):
        return abinitio_integrals(self.K, self.seed)

    def table(self) -> BlockTable:
        return make_block_table(self.K, self.N, self.twoM, self.D)

    def blocks(self) -> np.ndarray:
        return random_blocks(self.table(), self.seed + 1000)


def abinitio_full() -> AbInitioWorkload:
    """K=30 orbitals, N=30, M=0, S=0, D=500, G=11, seed 4."""
    return AbInitioWorkload("abinitio_K30_D500_G11", K=30, N=30, twoS=0, twoM=0, D=500, G=11, sweeps=4, seed=4)


def abinitio_reduced(K: int = 12, D: int = 128, G: int = 11) -> AbInitioWorkload:
    """The same integral recipe at fewer orbitals and a smaller bond
    dimension: half filling, M=0, S=0, seed 4."""
    return AbInitioWorkload(f"abinitio_K{K}_D{D}_G{G}", K=K, N=K, twoS=0, twoM=0, D=D, G=G, sweeps=4, seed=4)


# ---------------------------------------------------------------------------
# Initial weights of the learned Davidson preconditioner (a two-layer MLP on
# five features per site-tensor element).


def mlp_init(hidden: int = 256, seed: int = 0, n_in: int = 5):
    """Seeded initial weights (FP32): W1 (hidden x n_in) and w2 (hidden)
    uniform in +-sqrt(6/fan_in) (He initialisation for the ReLU layer,
    +-sqrt(3/hidden) for the output), biases zero."""
    rng = np.random.default_rng(seed)
    W1 = rng.uniform(-1.0, 1.0, (hidden, n_in)) * math.sqrt(6.0 / n_in)
    w2 = rng.uniform(-1.0, 1.0, hidden) * math.sqrt(3.0 / hidden)
    return {"W1": W1.astype(np.float32), "b1": np.zeros(hidden, np.float32),
            "w2": w2.astype(np.float32), "b2": np.float32(0.0)}
