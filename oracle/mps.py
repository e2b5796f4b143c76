"""The SP-MPS one-site sweep (Sec. 2.3) in plain dense FP64.  Test
infrastructure only.

Site tensors are kept as dense arrays A[k] of shape (4, D_{k-1}, D_k) with
exact zeros outside the blocks allowed by the (N, 2M) labels of the bonds;
the allowed entries are the variational parameters of the MPS of
Eq. [SPMPS2] (definite N and M, Sec. 2.2).  No block sparsity is exploited:
every contraction is a dense einsum.

For every quadrature point g of Eq. [pmpo] the environments are built with
the bra unrotated and the ket rotated by exp(-i beta_g S_y), which is the
product of the local matrices r(beta_g) of Eq. [expSy].  H_eff and N_eff
(Eq. [geproblem], Fig. [spmpsOpt]) are then

  H_eff x = sum_g coef_g  L_g[k-1] (W[k] r_g) x R_g[k+1]   (MPO of H)
  N_eff x = sum_g coef_g  L^I_g[k-1]  r_g     x R^I_g[k+1]   (identity MPO)

followed by the projection back onto the allowed (N, M) blocks (the bra has
definite M, Sec. 2.2 below Eq. [efunctional]).
"""
from __future__ import annotations

import numpy as np

from . import local_ops as lo
from . import mpo as mpo_mod
from .quadrature import projector_quadrature

SIGMA_QN = np.array([(0, 0), (1, -1), (1, 1), (2, 0)])


class OracleMPS:
    """Dense-padded MPS over a block table (bond sector list per bond)."""

    def __init__(self, table, packed):
        self.L = table.L
        self.N = table.N
        self.twoM = table.twoM
        self.qn = []
        for k in range(self.L + 1):
            rows = []
            for (n, m, d) in table.bonds[k]:
                rows += [(n, m)] * d
            self.qn.append(np.array(rows, dtype=int).reshape(-1, 2))
        self.sectors = [list(b) for b in table.bonds]
        self.A = []
        self.mask = []
        for k in range(1, self.L + 1):
            ql, qr = self.qn[k - 1], self.qn[k]
            m = np.zeros((4, len(ql), len(qr)), dtype=bool)
            for s in range(4):
                tgt = ql + SIGMA_QN[s]
                m[s] = (tgt[:, None, 0] == qr[None, :, 0]) & (tgt[:, None, 1] == qr[None, :, 1])
            self.mask.append(m)
            self.A.append(np.zeros(m.shape))
        self.set_packed(packed)

    def nblock_labels(self, k):
        """N-block of every allowed element of site k, in the order of the
        site's non-zero dense entries: elements share a label when they
        share the particle numbers of both bonds (left N and local n fix
        the right N), whatever their M."""
        m = self.mask[k - 1]
        s, a, _ = np.unravel_index(np.flatnonzero(m.ravel()), m.shape)
        return self.qn[k - 1][a, 0] * 3 + SIGMA_QN[s, 0]

    # --- packed <-> dense, canonical block order ---------------------------
    def _ranges(self, k):
        out, off = [], 0
        for (n, m, d) in self.sectors[k]:
            out.append((n, m, off, d))
            off += d
        return out

    def site_blocks(self, k):
        """(sigma, left slice, right slice) per block of site k, canonical
        order: left sector, then sigma."""
        left = self._ranges(k - 1)
        right = {(n, m): (o, d) for (n, m, o, d) in self._ranges(k)}
        out = []
        for (n, m, o, d) in left:
            for s in range(4):
                key = (n + SIGMA_QN[s][0], m + SIGMA_QN[s][1])
                if key in right:
                    ro, rd = right[key]
                    out.append((s, slice(o, o + d), slice(ro, ro + rd)))
        return out

    def set_packed(self, packed):
        pos = 0
        for k in range(1, self.L + 1):
            A = self.A[k - 1]
            A[:] = 0.0
            for (s, sa, sb) in self.site_blocks(k):
                r = sa.stop - sa.start
                c = sb.stop - sb.start
                A[s, sa, sb] = packed[pos:pos + r * c].reshape(r, c)
                pos += r * c
        if pos != len(packed):
            raise ValueError("packed size does not match the block table")

    def dense_site(self, k, packed):
        """Dense-padded array of site k from a packed vector."""
        A = np.zeros(self.mask[k - 1].shape)
        pos = 0
        for (s, sa, sb) in self.site_blocks(k):
            r = sa.stop - sa.start
            c = sb.stop - sb.start
            A[s, sa, sb] = packed[pos:pos + r * c].reshape(r, c)
            pos += r * c
        return A

    def site_packed(self, k, A=None):
        A = self.A[k - 1] if A is None else A
        return np.concatenate([A[s, sa, sb].ravel() for (s, sa, sb) in self.site_blocks(k)])

    def packed(self):
        return np.concatenate([self.site_packed(k) for k in range(1, self.L + 1)])

    # --- canonical gauge moves (Sec. 2.3: canonical form after the local
    # solve) -----------------------------------------------------------------
    @staticmethod
    def _qr_pos(M):
        """Thin QR with a non-negative diagonal of R (the unique QR of a full
        column rank matrix)."""
        Q, R = np.linalg.qr(M, mode="reduced")
        d = np.sign(np.diag(R))
        d[d == 0] = 1.0
        return Q * d[None, :], R * d[:, None]

    def left_orthonormalize(self, k):
        """Make site k left-orthonormal per right sector; push R into site
        k+1 (or return it at the last site).  Returns the block-diagonal R."""
        A = self.A[k - 1]
        m = self.mask[k - 1]
        Db = A.shape[2]
        Rfull = np.zeros((Db, Db))
        for (n, mm, o, d) in self._ranges(k):
            cols = slice(o, o + d)
            rows = [(s, a) for s in range(4) for a in range(A.shape[1]) if m[s, a, o]]
            M = np.array([A[s, a, cols] for (s, a) in rows]).reshape(len(rows), d)
            if len(rows) < d:
                raise ValueError("bond sector wider than its left support")
            Q, R = self._qr_pos(M)
            for i, (s, a) in enumerate(rows):
                A[s, a, cols] = Q[i]
            Rfull[cols, cols] = R
        if k < self.L:
            self.A[k] = np.einsum("ab,sbc->sac", Rfull, self.A[k])
        return Rfull

    def right_orthonormalize(self, k):
        """Make site k right-orthonormal per left sector (LQ with a
        non-negative diagonal of L); push L into site k-1."""
        A = self.A[k - 1]
        m = self.mask[k - 1]
        Da = A.shape[1]
        Lfull = np.zeros((Da, Da))
        for (n, mm, o, d) in self._ranges(k - 1):
            rows = slice(o, o + d)
            cols = [(s, b) for s in range(4) for b in range(A.shape[2]) if m[s, o, b]]
            M = np.array([A[s, rows, b] for (s, b) in cols]).reshape(len(cols), d)  # = M^T
            if len(cols) < d:
                raise ValueError("bond sector wider than its right support")
            Q, R = self._qr_pos(M)          # M^T = Q R  ->  M = R^T Q^T
            for i, (s, b) in enumerate(cols):
                A[s, rows, b] = Q[i]
            Lfull[rows, rows] = R.T
        if k > 1:
            self.A[k - 2] = np.einsum("sab,bc->sac", self.A[k - 2], Lfull)
        return Lfull

    def right_canonicalize(self):
        for k in range(self.L, 1, -1):
            self.right_orthonormalize(k)


# ---------------------------------------------------------------------------
# environments


def rotated_mpo(W, r):
    """W[k] r: the rotation acts on the ket index of each site operator
    (Eq. [pmpo] folded into the MPO, one bond-dimension-1 factor per site)."""
    return [np.einsum("abst,tu->absu", w, r) for w in W]


def env_left(Lprev, A, Wt, K=None):
    """L[b, v, d] = sum A[s,a,b] Lprev[a,w,c] Wt[w,v,s,t] K[t,c,d]: bra
    tensor A, ket tensor K (default A)."""
    K = A if K is None else K
    X1 = np.einsum("awc,tcd->awtd", Lprev, K, optimize=True)
    X2 = np.einsum("awtd,wvst->avsd", X1, Wt, optimize=True)
    return np.einsum("sab,avsd->bvd", A, X2, optimize=True)


def env_right(Rnext, A, Wt, K=None):
    """R[a, w, c] = sum A[s,a,b] Wt[w,v,s,t] K[t,c,d] Rnext[b,v,d]: bra A,
    ket K (default A)."""
    K = A if K is None else K
    Y1 = np.einsum("tcd,bvd->tcbv", K, Rnext, optimize=True)
    Y2 = np.einsum("wvst,tcbv->swcb", Wt, Y1, optimize=True)
    return np.einsum("sab,swcb->awc", A, Y2, optimize=True)


def apply_local(Lenv, Wt, Renv, x):
    """y[s,a,b] = sum Lenv[a,w,c] Wt[w,v,s,t] x[t,c,d] Renv[b,v,d]."""
    X1 = np.einsum("awc,tcd->awtd", Lenv, x, optimize=True)
    X2 = np.einsum("awtd,wvst->avsd", X1, Wt, optimize=True)
    return np.einsum("avsd,bvd->sab", X2, Renv, optimize=True)


class SPMPSOracle:
    """Spin-projected sweep state: MPS, quadrature, H and identity
    environments for every quadrature point."""

    def __init__(self, table, packed, W, twoS, G, canonicalize=True):
        self.mps = OracleMPS(table, packed)
        self.L = table.L
        self.W = W
        self.twoS = twoS
        self.G = G
        self.quad = projector_quadrature(G, twoS, table.twoM)
        self.r = [lo.rotation_cs(c, s) for c, s in zip(self.quad["c"], self.quad["s"])]
        self.Wt = [rotated_mpo(W, r) for r in self.r]
        I = mpo_mod.identity_mpo(self.L)
        self.It = [rotated_mpo(I, r) for r in self.r]
        one = np.ones((1, 1, 1))
        # Lenv[g][k]: bond k, sites 1..k ; Renv[g][k]: sites k..L (bond k-1)
        self.LH = [[None] * (self.L + 2) for _ in range(G)]
        self.RH = [[None] * (self.L + 2) for _ in range(G)]
        self.LI = [[None] * (self.L + 2) for _ in range(G)]
        self.RI = [[None] * (self.L + 2) for _ in range(G)]
        for g in range(G):
            self.LH[g][0] = one.copy()
            self.LI[g][0] = one.copy()
            self.RH[g][self.L + 1] = one.copy()
            self.RI[g][self.L + 1] = one.copy()
        if canonicalize:
            self.mps.right_canonicalize()
        for k in range(self.L, 1, -1):
            self.update_right(k)

    # environment updates (Fig. [spmpsOpt]) ------------------------------
    def update_left(self, k):
        A = self.mps.A[k - 1]
        for g in range(self.G):
            self.LH[g][k] = env_left(self.LH[g][k - 1], A, self.Wt[g][k - 1])
            self.LI[g][k] = env_left(self.LI[g][k - 1], A, self.It[g][k - 1])

    def update_right(self, k):
        A = self.mps.A[k - 1]
        for g in range(self.G):
            self.RH[g][k] = env_right(self.RH[g][k + 1], A, self.Wt[g][k - 1])
            self.RI[g][k] = env_right(self.RI[g][k + 1], A, self.It[g][k - 1])

    # H_eff x and N_eff x (Eq. [geproblem]) ---------------------------------
    def heff(self, k, x):
        """(H_eff x, N_eff x) at site k for x in the dense-padded layout."""
        y = np.zeros_like(x)
        ny = np.zeros_like(x)
        for g in range(self.G):
            cg = self.quad["coef"][g]
            y += cg * apply_local(self.LH[g][k - 1], self.Wt[g][k - 1], self.RH[g][k + 1], x)
            ny += cg * apply_local(self.LI[g][k - 1], self.It[g][k - 1], self.RI[g][k + 1], x)
        m = self.mps.mask[k - 1]
        return np.where(m, y, 0.0), np.where(m, ny, 0.0)

    def heff_diag(self, k):
        """Diagonals of H_eff and N_eff at site k (preconditioner)."""
        shape = self.mps.A[k - 1].shape
        dh = np.zeros(shape)
        dn = np.zeros(shape)
        for g in range(self.G):
            cg = self.quad["coef"][g]
            Ld = np.einsum("awa->aw", self.LH[g][k - 1])
            Rd = np.einsum("bvb->bv", self.RH[g][k + 1])
            Wd = np.einsum("wvss->wvs", self.Wt[g][k - 1])
            dh += cg * np.einsum("aw,wvs,bv->sab", Ld, Wd, Rd)
            Ld = np.einsum("awa->aw", self.LI[g][k - 1])
            Rd = np.einsum("bvb->bv", self.RI[g][k + 1])
            Wd = np.einsum("wvss->wvs", self.It[g][k - 1])
            dn += cg * np.einsum("aw,wvs,bv->sab", Ld, Wd, Rd)
        m = self.mps.mask[k - 1]
        return np.where(m, dh, 0.0), np.where(m, dn, 0.0)

    def energy(self, k):
        """Projected energy functional (Eq. [efunctional]) evaluated at
        site k with the current environments: (E, <P>)."""
        x = self.mps.A[k - 1]
        y, ny = self.heff(k, x)
        num = float(np.sum(x * y))
        den = float(np.sum(x * ny))
        return num / den, den

    def full_contraction(self):
        """<HP> and <P> by contracting left environments over the whole
        chain, independent of the canonical form."""
        num = den = 0.0
        for g in range(self.G):
            Lh = np.ones((1, 1, 1))
            Li = np.ones((1, 1, 1))
            for k in range(1, self.L + 1):
                A = self.mps.A[k - 1]
                Lh = env_left(Lh, A, self.Wt[g][k - 1])
                Li = env_left(Li, A, self.It[g][k - 1])
            num += self.quad["coef"][g] * Lh[0, 0, 0]
            den += self.quad["coef"][g] * Li[0, 0, 0]
        return num / den, den


# ---------------------------------------------------------------------------
# Davidson for the singular pencil H_eff x = theta N_eff x (Eq. [geproblem]).
# The paper does not state the local solver; this is the reading used by both
# the oracle and the library (see the design notes): one target vector,
# Euclidean-orthonormal search space, canonical orthogonalisation of the
# projected metric, diagonal preconditioner, restart to the lowest Ritz
# vectors.


class DavidsonResult:
    def __init__(self, theta, x, rnorm, iters, converged, pnorm):
        self.theta = theta
        self.x = x
        self.rnorm = rnorm
        self.iters = iters
        self.converged = converged
        self.pnorm = pnorm


def davidson(matvec, dH, dN, x0, tol=1e-9, max_iter=64, max_sub=32, keep=8,
             drop=1e-10, floor=1e-8, C=None, precond=None, record=None):
    """Lowest theta of H x = theta N x within range(N).

    matvec(v) -> (H v, N v) on flat vectors.  Returns a DavidsonResult with
    x normalised to unit Euclidean norm and pnorm = x^T N x.

    C (n x c, orthonormal columns) restricts the search to the complement of
    span(C) (the constraints of Eq. [orthoB]): with Q = 1 - C C^T the
    pencil becomes (Q H Q, Q N Q), i.e. the start vector, every H v, N v and
    every correction are multiplied by Q (twice, for rounding), so the
    residual is the projected one.

    precond(r, theta) -> t replaces the diagonal correction (a learned
    preconditioner); it is abandoned for the rest of the solve once the
    residual norm has failed three times in a row to reach a new minimum, or
    has fallen by less than a factor of two over the last four iterations.
    record (a list) receives, after a converged solve, one (r_j, theta_j,
    x_j, x*, dH, dN) tuple per iteration but the last (training pairs).
    """
    if C is not None and C.shape[1] > 0:
        def proj(u):
            for _ in range(2):
                u = u - C @ (C.T @ u)
            return u
    else:
        def proj(u):
            return u
    v = proj(x0)
    v = v / np.linalg.norm(v)
    V = [v]
    HV, NV = [], []
    hv, nv = matvec(v)
    hv, nv = proj(hv), proj(nv)
    HV.append(hv)
    NV.append(nv)
    theta = 0.0
    x = v
    rn = np.inf
    it = 0
    use_model, best, stall, hist = precond is not None, np.inf, 0, []
    trail = []
    for it in range(1, max_iter + 1):
        Vm = np.array(V).T
        Hm = np.array(HV).T
        Nm = np.array(NV).T
        Ht = Vm.T @ Hm
        Nt = Vm.T @ Nm
        Ht = 0.5 * (Ht + Ht.T)
        Nt = 0.5 * (Nt + Nt.T)
        lam, Uv = np.linalg.eigh(Nt)
        lmax = lam.max()
        if not lmax > 1e-12:
            raise FloatingPointError("projected norm vanishes in the search space")
        sel = lam > drop * lmax
        X = Uv[:, sel] / np.sqrt(lam[sel])[None, :]
        mu, Cm = np.linalg.eigh(X.T @ Ht @ X)
        theta = float(mu[0])
        a = X @ Cm[:, 0]
        x = Vm @ a
        hx = Hm @ a
        nx = Nm @ a
        nrm = np.linalg.norm(x)
        x, hx, nx = x / nrm, hx / nrm, nx / nrm
        r = hx - theta * nx
        rn = float(np.linalg.norm(r))
        if rn <= tol or it == max_iter:
            break
        if record is not None:
            trail.append((r.copy(), theta, x.copy()))
        if use_model:
            t = proj(np.asarray(precond(r, theta), dtype=float))
            # the residual norms seen so far decide the next iterations
            if rn < best:
                best, stall = rn, 0
            else:
                stall += 1
            hist.append(rn)
            slow = len(hist) >= 5 and rn > 0.5 * hist[-5]
            use_model = stall < 3 and not slow
        else:
            den = dH - theta * dN
            den = np.where(np.abs(den) < floor, np.where(den < 0, -floor, floor), den)
            t = proj(-r / den)
        if len(V) >= max_sub:
            nk = min(keep, Cm.shape[1])
            Ak = X @ Cm[:, :nk]
            Qk, _ = np.linalg.qr(Ak)
            V = list((Vm @ Qk).T)
            HV = list((Hm @ Qk).T)
            NV = list((Nm @ Qk).T)
            Vm = np.array(V).T
        for _ in range(2):
            t = t - Vm @ (Vm.T @ t)
        tn = np.linalg.norm(t)
        if tn < 1e-14:
            break
        t = t / tn
        V.append(t)
        hv, nv = matvec(t)
        hv, nv = proj(hv), proj(nv)
        HV.append(hv)
        NV.append(nv)
    pn = float(x @ nx)
    if record is not None and rn <= tol:
        record.extend((r_, th_, x_, x.copy(), dH, dN) for (r_, th_, x_) in trail)
    return DavidsonResult(theta, x, rn, it, rn <= tol, pn)


def orthonormal_constraints(vectors, rel_drop=1e-10):
    """Orthonormal basis of the constraint vectors B_j (Eq. [orthoB]) by
    Gram-Schmidt in the given order, each projection done twice; a vector
    whose remainder falls below rel_drop times its own norm is dependent on
    the earlier ones and dropped.  Returns an n x c array."""
    cols = []
    for b in vectors:
        nb = float(np.linalg.norm(b))
        u = np.array(b, dtype=float)
        for _ in range(2):
            for c in cols:
                u = u - c * float(c @ u)
        nu = float(np.linalg.norm(u))
        if nb > 0.0 and nu > rel_drop * nb:
            cols.append(u / nu)
    n = len(vectors[0]) if len(vectors) else 0
    return np.array(cols).T if cols else np.zeros((n, 0))


class OrthogonalityConstraint:
    """Orthogonality of the optimised state Psi to a fixed state Psi_0 in the
    projected metric, <Psi_0|P|Psi> = 0 (Sec. 2.3, Eq. [orthoB]).

    Keeps, for every quadrature point, the environments of
    <Psi|R(beta_g)|Psi_0> (bra: the optimised state, ket: Psi_0, the rotated
    identity MPO between them), updated as the sweep changes Psi, and builds
    B[k] = sum_g coef_g L_g[k-1] (r_g Psi_0[k]) R_g[k+1], the derivative of
    <Psi|P|Psi_0> = <Psi_0|P|Psi> with respect to Psi's site tensor k.  Psi_0
    keeps the gauge it is given in."""

    def __init__(self, state: SPMPSOracle, table, packed0):
        self.state = state
        self.psi0 = OracleMPS(table, packed0)
        L, G = state.L, state.G
        one = np.ones((1, 1, 1))
        self.Le = [[None] * (L + 2) for _ in range(G)]
        self.Re = [[None] * (L + 2) for _ in range(G)]
        for g in range(G):
            self.Le[g][0] = one.copy()
            self.Re[g][L + 1] = one.copy()
        for k in range(L, 1, -1):
            self.update_right(k)

    def update_left(self, k):
        A, K = self.state.mps.A[k - 1], self.psi0.A[k - 1]
        for g in range(self.state.G):
            self.Le[g][k] = env_left(self.Le[g][k - 1], A, self.state.It[g][k - 1], K)

    def update_right(self, k):
        A, K = self.state.mps.A[k - 1], self.psi0.A[k - 1]
        for g in range(self.state.G):
            self.Re[g][k] = env_right(self.Re[g][k + 1], A, self.state.It[g][k - 1], K)

    def vector(self, k):
        """B[k] in Psi's dense-padded site layout."""
        out = np.zeros(self.state.mps.A[k - 1].shape)
        for g in range(self.state.G):
            out += self.state.quad["coef"][g] * apply_local(self.Le[g][k - 1], self.state.It[g][k - 1],
                                                             self.Re[g][k + 1], self.psi0.A[k - 1])
        return np.where(self.state.mps.mask[k - 1], out, 0.0)

    def overlap(self, k):
        """<Psi_0|P|Psi> from the environments around site k."""
        return float(np.sum(self.vector(k) * self.state.mps.A[k - 1]))


def sweep(state: SPMPSOracle, n_sweeps: int, tol=1e-9, max_iter=64, max_sub=32,
          keep=8, record=None, constraints=(), model=None, pairs=None, nblock=False):
    """One-site sweeps (Sec. 2.3): right-moving k = 1..L-1 then left-moving
    k = L..2.  Each step solves the local problem, restores the canonical
    form with a positive-diagonal QR (right-moving) or LQ (left-moving) and
    updates the environments of the bond it leaves behind.  With
    ``constraints`` (OrthogonalityConstraint objects built on this state)
    every local solve is restricted to the complement of the B[k] vectors
    of Eq. [orthoB] (excited states).  ``model`` (weights of the learned
    preconditioner, see oracle.precond; per N-block with ``nblock``)
    replaces the diagonal correction;
    ``pairs`` (a list) collects the solver's training pairs as (site,) +
    the tuples of :func:`davidson` (vectors in the order of the site's
    non-zero dense entries).

    Returns a list of per-step dicts (sweep, site, dir, theta, pnorm, rnorm,
    iters)."""
    L = state.L
    steps = []
    mps = state.mps
    for sw in range(n_sweeps):
        order = [(k, +1) for k in range(1, L)] + [(k, -1) for k in range(L, 1, -1)]
        for (k, d) in order:
            m = mps.mask[k - 1]
            shape = m.shape
            idx = np.flatnonzero(m.ravel())

            def mv(v, k=k, idx=idx, shape=shape):
                xd = np.zeros(int(np.prod(shape)))
                xd[idx] = v
                y, ny = state.heff(k, xd.reshape(shape))
                return y.ravel()[idx], ny.ravel()[idx]
            dh, dn = state.heff_diag(k)
            x0 = mps.A[k - 1].ravel()[idx]
            C = orthonormal_constraints([c.vector(k).ravel()[idx] for c in constraints]) if constraints else None
            dhv, dnv = dh.ravel()[idx], dn.ravel()[idx]
            pc = None
            if model is not None:
                from . import precond as pre

                grp = mps.nblock_labels(k) if nblock else None

                def pc(r, th, dhv=dhv, dnv=dnv, grp=grp):
                    return pre.correction(model, r, dhv, dnv, th, groups=grp)
            rec_k = [] if pairs is not None else None
            res = davidson(mv, dhv, dnv, x0, tol=tol, max_iter=max_iter, max_sub=max_sub, keep=keep, C=C,
                           precond=pc, record=rec_k)
            if pairs is not None:
                pairs.extend((k,) + e for e in rec_k)
            xd = np.zeros(int(np.prod(shape)))
            xd[idx] = res.x
            mps.A[k - 1] = xd.reshape(shape)
            if d > 0:
                mps.left_orthonormalize(k)
                state.update_left(k)
                for c in constraints:
                    c.update_left(k)
            else:
                mps.right_orthonormalize(k)
                state.update_right(k)
                for c in constraints:
                    c.update_right(k)
            steps.append(dict(sweep=sw, site=k, dir=d, theta=res.theta, pnorm=res.pnorm,
                              rnorm=res.rnorm, iters=res.iters, converged=res.converged))
            if record is not None:
                record(steps[-1])
    return steps


def expect(table, packed, O, twoS, G):
    """Projected expectation value of a spin-free operator O (an MPO),
    Eq. [PropSpinFree]: <Psi|O P|Psi> / <Psi|P|Psi> for the MPS of the packed
    site tensors, with the quadrature projector of (twoS, G).  Returns
    (<O>, <P>/<Psi|Psi>)."""
    st = SPMPSOracle(table, packed, O, twoS, G)
    val, den = st.energy(1)
    x = st.mps.A[0]
    return val, den / float(np.sum(x * x))
