"""Python binding of libspmps.so, the spin-projected MPS (SP-MPS) hot path on
an AMD MI355X (gfx950).

Argument marshalling only: every step of the method runs in the HIP library
(``csrc/``); see ``include/spmps.h`` for the contract of each call.  Device
buffers are torch tensors on the current HIP device; host inputs are NumPy
arrays.  The library must be built first (``paper_1703_04789_amd/build.py``);
importing works without it, but every call raises if it is missing.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspmps.so")

SP_OK, SP_ENOCONV, SP_WINEXACT = 0, 1, 2
SP_EINVAL, SP_ENORM, SP_EHIP, SP_ENOMEM, SP_ESTATE, SP_ENAN = -1, -2, -3, -4, -5, -6
SP_FP64 = 0
SP_FP32 = 1
SP_BF16X3 = 2
SP_PATH_TILED, SP_PATH_PLAIN = 0, 1
SOLVERS = {"auto": 0, "host": 1, "device": 2}

EXPORTS = ["sp_init_mps", "sp_env_update", "sp_heff_apply", "sp_heff_diag", "sp_sweep", "sp_energy",
           "sp_destroy", "sp_site_size", "sp_get_site", "sp_set_site", "sp_center", "sp_heff_flops",
           "sp_heff_profile",
           "sp_last_error", "sp_quadrature", "sp_exact_points", "sp_mpo_hubbard", "sp_mpo_s2",
           "sp_mpo_identity", "sp_small_eigh", "sp_small_gen_lowest", "sp_sweep_batch", "sp_autotune",
           "sp_mpo_site_op", "sp_mpo_epq", "sp_mpo_spin_corr", "sp_expect",
           "sp_mpo_abinitio", "sp_set_heff_plan", "sp_heff_plan", "sp_add_orthogonality",
           "sp_clear_orthogonality", "sp_orthogonality_overlaps", "sp_mlp_create", "sp_mlp_set_scope",
           "sp_mlp_destroy", "sp_mlp_get", "sp_mlp_dataset", "sp_mlp_forward", "sp_mlp_train_step", "sp_mlp_train",
           "sp_set_precond", "sp_heff_batch_profile", "sp_heff_apply_noalloc",
           "sp_mpo_abinitio_component", "sp_mpo_hubbard_component", "sp_small_gen_lowest_gpu"]


class SpError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class _Problem(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int), ("d", ctypes.c_int), ("N", ctypes.c_int), ("twoS", ctypes.c_int),
                ("twoM", ctypes.c_int), ("G", ctypes.c_int), ("precision", ctypes.c_int),
                ("path", ctypes.c_int)]


class _Mpo(ctypes.Structure):
    _fields_ = [("w", ctypes.POINTER(ctypes.c_int)), ("data", ctypes.POINTER(ctypes.c_double))]


class _BlockTable(ctypes.Structure):
    _fields_ = [("nsec", ctypes.POINTER(ctypes.c_int)), ("sec_n", ctypes.POINTER(ctypes.c_int)),
                ("sec_2m", ctypes.POINTER(ctypes.c_int)), ("sec_dim", ctypes.POINTER(ctypes.c_int))]


class _SweepOpts(ctypes.Structure):
    _fields_ = [("n_sweeps", ctypes.c_int), ("tol", ctypes.c_double), ("max_iter", ctypes.c_int),
                ("max_sub", ctypes.c_int), ("keep", ctypes.c_int), ("solver", ctypes.c_int),
                ("verbose", ctypes.c_int)]


class _StepReport(ctypes.Structure):
    _fields_ = [("sweep", ctypes.c_int), ("site", ctypes.c_int), ("dir", ctypes.c_int), ("iters", ctypes.c_int),
                ("converged", ctypes.c_int), ("matvecs", ctypes.c_int), ("theta", ctypes.c_double),
                ("pnorm", ctypes.c_double), ("rnorm", ctypes.c_double), ("usec", ctypes.c_double)]


class _SweepReport(ctypes.Structure):
    _fields_ = [("capacity", ctypes.c_int), ("n_steps", ctypes.c_int), ("steps", ctypes.POINTER(_StepReport))]


_lib = None


def lib():
    """Load libspmps.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1703_04789_amd/build.py")
    # PyTorch ships its own HIP runtime: load it first so that the library
    # binds to the same runtime instance (one device context per process)
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp, ip, dp = ctypes.c_void_p, P(ctypes.c_int), P(ctypes.c_double)
    fp = P(ctypes.c_float)
    sig = {
        "sp_init_mps": [P(_Problem), P(_Mpo), P(_BlockTable), dp, vp, P(vp)],
        "sp_env_update": [vp, ctypes.c_int, ctypes.c_int],
        "sp_heff_apply": [vp, ctypes.c_int, vp, vp, vp],
        "sp_heff_apply_noalloc": [vp, ctypes.c_int, vp, vp, vp],
        "sp_heff_diag": [vp, ctypes.c_int, vp, vp],
        "sp_sweep": [vp, P(_SweepOpts), P(_SweepReport)],
        "sp_sweep_batch": [P(vp), ctypes.c_int, P(_SweepOpts), P(_SweepReport)],
        "sp_autotune": [vp, ctypes.c_int, ip, ip, dp],
        "sp_set_heff_plan": [vp, ctypes.c_int, ctypes.c_int, ip],
        "sp_heff_plan": [vp, ctypes.c_int, ip, ip],
        "sp_add_orthogonality": [vp, vp],
        "sp_clear_orthogonality": [vp],
        "sp_orthogonality_overlaps": [vp, dp],
        "sp_mlp_create": [ctypes.c_int, fp, ctypes.c_longlong, P(vp)],
        "sp_mlp_set_scope": [vp, ctypes.c_int],
        "sp_mlp_destroy": [vp],
        "sp_mlp_get": [vp, fp, P(ctypes.c_longlong)],
        "sp_mlp_dataset": [vp, ctypes.c_longlong, ctypes.c_longlong, fp, fp],
        "sp_mlp_forward": [vp, vp, ctypes.c_longlong, vp, vp],
        "sp_mlp_train_step": [vp, vp, vp, ctypes.c_longlong, ctypes.c_double, dp, vp],
        "sp_mlp_train": [vp, ctypes.c_int, ctypes.c_longlong, ctypes.c_double, dp, vp],
        "sp_set_precond": [vp, vp, vp],
        "sp_heff_batch_profile": [P(vp), ctypes.c_int, ip, ctypes.c_int, dp],
        "sp_mpo_site_op": [ctypes.c_int, ctypes.c_int, dp, ip, dp, P(ctypes.c_longlong)],
        "sp_mpo_epq": [ctypes.c_int, ctypes.c_int, ctypes.c_int, ip, dp, P(ctypes.c_longlong)],
        "sp_mpo_spin_corr": [ctypes.c_int, ctypes.c_int, ctypes.c_int, ip, dp, P(ctypes.c_longlong)],
        "sp_mpo_abinitio": [ctypes.c_int, dp, dp, ip, dp, P(ctypes.c_longlong)],
        "sp_mpo_abinitio_component": [ctypes.c_int, ctypes.c_int, dp, dp, ip, dp, P(ctypes.c_longlong)],
        "sp_mpo_hubbard_component": [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, ip, dp,
                                     P(ctypes.c_longlong)],
        "sp_expect": [vp, P(_Mpo), dp, dp],
        "sp_energy": [vp, dp, dp],
        "sp_destroy": [vp],
        "sp_site_size": [vp, ctypes.c_int, P(ctypes.c_longlong)],
        "sp_get_site": [vp, ctypes.c_int, dp],
        "sp_set_site": [vp, ctypes.c_int, dp],
        "sp_center": [vp, ip],
        "sp_heff_flops": [vp, ctypes.c_int, dp],
        "sp_heff_profile": [vp, ctypes.c_int, ctypes.c_int, vp, vp, vp, dp],
        "sp_quadrature": [ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp, dp],
        "sp_exact_points": [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int],
        "sp_mpo_hubbard": [ctypes.c_int, ctypes.c_double, ctypes.c_double, ip, dp, P(ctypes.c_longlong)],
        "sp_mpo_s2": [ctypes.c_int, ip, dp, P(ctypes.c_longlong)],
        "sp_mpo_identity": [ctypes.c_int, ip, dp, P(ctypes.c_longlong)],
        "sp_small_eigh": [ctypes.c_int, dp, dp, dp],
        "sp_small_gen_lowest": [ctypes.c_int, dp, dp, ctypes.c_double, dp, dp, ctypes.POINTER(ctypes.c_int)],
        "sp_small_gen_lowest_gpu": [ctypes.c_int, dp, dp, ctypes.c_double, ctypes.c_int, ctypes.c_int, dp, dp, dp,
                                    ctypes.POINTER(ctypes.c_int)],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    L.sp_last_error.argtypes = []
    L.sp_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(rc):
    if rc < 0:
        raise SpError(rc, lib().sp_last_error().decode())
    return rc


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _fptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def _dev32(t):
    """Device pointer of a contiguous float32 torch tensor."""
    if t.dtype.__str__() != "torch.float32" or not t.is_cuda or not t.is_contiguous():
        raise ValueError("model buffers must be contiguous float32 tensors on the GPU")
    return ctypes.c_void_p(t.data_ptr())


def _iptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _dev(t):
    """Device pointer of a contiguous float64 torch tensor."""
    if t.dtype.__str__() != "torch.float64" or not t.is_cuda or not t.is_contiguous():
        raise ValueError("device buffers must be contiguous float64 tensors on the GPU")
    return ctypes.c_void_p(t.data_ptr())


# ---- host-only helpers ---------------------------------------------------

def quadrature(G, twoS, twoM):
    x, w, c = np.zeros(G), np.zeros(G), np.zeros(G)
    _check(lib().sp_quadrature(G, twoS, twoM, _dptr(x), _dptr(w), _dptr(c)))
    return x, w, c


def exact_points(N, K, twoS, twoM=0):
    return lib().sp_exact_points(N, K, twoS, twoM)


def _mpo(fn, L, *args):
    w = np.zeros(L + 1, dtype=np.int32)
    n = ctypes.c_longlong(0)
    _check(fn(L, *args, _iptr(w), None, ctypes.byref(n)))
    data = np.zeros(n.value)
    _check(fn(L, *args, _iptr(w), _dptr(data), ctypes.byref(n)))
    return w, data


def mpo_hubbard(L, t, U):
    return _mpo(lib().sp_mpo_hubbard, L, ctypes.c_double(t), ctypes.c_double(U))


def mpo_s2(L):
    return _mpo(lib().sp_mpo_s2, L)


def mpo_identity(L):
    return _mpo(lib().sp_mpo_identity, L)


def mpo_site_op(L, p, op):
    op = np.ascontiguousarray(op, dtype=np.float64).reshape(16)
    return _mpo(lib().sp_mpo_site_op, L, ctypes.c_int(p), _dptr(op))


def mpo_epq(L, p, q):
    """E_pq = sum_sigma a+_{p sigma} a_{q sigma} (1-based sites)."""
    return _mpo(lib().sp_mpo_epq, L, ctypes.c_int(p), ctypes.c_int(q))


def mpo_spin_corr(L, X, Y):
    """S_X . S_Y (1-based sites)."""
    return _mpo(lib().sp_mpo_spin_corr, L, ctypes.c_int(X), ctypes.c_int(Y))


def mpo_abinitio(h, eri):
    """The ab-initio Hamiltonian of K real orbitals from h[p, q] and
    eri[p, q, r, s] = (pq|rs)."""
    h = np.ascontiguousarray(h, dtype=np.float64)
    eri = np.ascontiguousarray(eri, dtype=np.float64)
    K = h.shape[0]
    if h.shape != (K, K) or eri.shape != (K, K, K, K):
        raise ValueError("h must be K x K and eri K x K x K x K")
    return _mpo(lib().sp_mpo_abinitio, K, _dptr(h), _dptr(eri))


def mpo_abinitio_component(h, eri, p):
    """Energy component H_p (orbital p, 1-based) of the ab-initio
    Hamiltonian: the terms whose first creator acts on p (sum_p H_p = H)."""
    h = np.ascontiguousarray(h, dtype=np.float64)
    eri = np.ascontiguousarray(eri, dtype=np.float64)
    K = h.shape[0]
    if h.shape != (K, K) or eri.shape != (K, K, K, K):
        raise ValueError("h must be K x K and eri K x K x K x K")
    return _mpo(lib().sp_mpo_abinitio_component, K, ctypes.c_int(p), _dptr(h), _dptr(eri))


def mpo_hubbard_component(L, p, t, U):
    """Energy component H_p of the open Hubbard chain (site p, 1-based):
    -t sum_s (a+_ps a_{p+1,s} + a+_ps a_{p-1,s}) + U n_pa n_pb."""
    return _mpo(lib().sp_mpo_hubbard_component, L, ctypes.c_int(p), ctypes.c_double(t), ctypes.c_double(U))


def heff_batch_profile(states, sites, reps=20):
    """One batched fused H_eff launch over the states at the given sites,
    eager and as a captured HIP graph: dict(usec, flops, bytes, workgroups,
    graph_usec, graph_max_diff)."""
    hs = (ctypes.c_void_p * len(states))(*[st._h.value for st in states])
    ks = np.ascontiguousarray(sites, dtype=np.int32)
    out = np.zeros(6)
    _check(lib().sp_heff_batch_profile(hs, len(states), _iptr(ks), reps, _dptr(out)))
    return {"usec": out[0], "flops": out[1], "bytes": out[2], "workgroups": int(out[3]),
            "graph_usec": out[4], "graph_max_diff": out[5]}


def small_eigh(a):
    a = np.ascontiguousarray(a, dtype=np.float64).copy()
    n = a.shape[0]
    ev, vec = np.zeros(n), np.zeros((n, n))
    _check(lib().sp_small_eigh(n, _dptr(a), _dptr(ev), _dptr(vec)))
    return ev, vec


def small_gen_lowest_gpu(H, N, drop=1e-10, keep=0):
    """The device-resident iteration's subspace solve on the current GPU:
    (theta, a, rank) and, with keep > 0 (a restart), also (Qk, H', N') with
    the orthonormalised lowest Ritz vectors and the rotated pencil."""
    H = np.array(H, dtype=np.float64, order="C")
    N = np.array(N, dtype=np.float64, order="C")
    m = H.shape[0]
    theta, a, rank = ctypes.c_double(0), np.zeros(m), ctypes.c_int(0)
    Qk = np.zeros(m * max(1, keep))
    _check(lib().sp_small_gen_lowest_gpu(m, _dptr(H), _dptr(N), drop, 1 if keep else 0, max(1, keep),
                                         ctypes.byref(theta), _dptr(a), _dptr(Qk), ctypes.byref(rank)))
    if not keep:
        return theta.value, a, rank.value
    nk = rank.value
    return theta.value, a, nk, Qk[: m * nk].reshape(m, nk), H[:nk, :nk].copy(), N[:nk, :nk].copy()


def small_gen_lowest(H, N, drop=1e-10):
    """Lowest (theta, a, rank) of the pencil (H, N) within the span of N's
    eigenvectors above drop * max (the Davidson subspace solve)."""
    H = np.ascontiguousarray(H, dtype=np.float64)
    N = np.ascontiguousarray(N, dtype=np.float64)
    m = H.shape[0]
    theta = np.zeros(1)
    a = np.zeros(m)
    rank = ctypes.c_int(0)
    _check(lib().sp_small_gen_lowest(m, _dptr(H), _dptr(N), float(drop), _dptr(theta), _dptr(a), ctypes.byref(rank)))
    return float(theta[0]), a, rank.value


# ---- the SP-MPS state ------------------------------------------------------

MLP_IN = 5  # features per element of the learned preconditioner


def pack_mlp(p):
    """Packed FP32 weights W1 (H x 5) | b1 | w2 | b2 from a dict."""
    return np.concatenate([np.asarray(p["W1"], np.float32).ravel(), np.asarray(p["b1"], np.float32),
                           np.asarray(p["w2"], np.float32), np.asarray([p["b2"]], np.float32)])


def unpack_mlp(w, H):
    w = np.asarray(w, np.float32)
    k = MLP_IN
    return {"W1": w[: k * H].reshape(H, k), "b1": w[k * H: (k + 1) * H], "w2": w[(k + 1) * H: (k + 2) * H],
            "b2": float(w[(k + 2) * H])}


class MLP:
    """A learned Davidson preconditioner (sp_mlp) on the current device."""

    def __init__(self, params, capacity=0, scope="vector"):
        """scope: "vector" (SP_MLP_VECTOR) or "nblock" (SP_MLP_NBLOCK)."""
        import torch
        self._torch = torch
        self.hidden = int(np.asarray(params["W1"]).shape[0])
        w = pack_mlp(params)
        h = ctypes.c_void_p()
        _check(lib().sp_mlp_create(self.hidden, _fptr(w), int(capacity), ctypes.byref(h)))
        self._h = h
        self.scope = scope
        if scope != "vector":
            self.set_scope(scope)

    def set_scope(self, scope):
        _check(lib().sp_mlp_set_scope(self._h, {"vector": 0, "nblock": 1}[scope]))
        self.scope = scope

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(lib().sp_mlp_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self):
        w = np.zeros((MLP_IN + 2) * self.hidden + 1, np.float32)
        _check(lib().sp_mlp_get(self._h, _fptr(w), None))
        return unpack_mlp(w, self.hidden)

    def rows(self):
        n = ctypes.c_longlong(0)
        _check(lib().sp_mlp_get(self._h, None, ctypes.byref(n)))
        return n.value

    def dataset(self, first=0, count=None):
        count = self.rows() - first if count is None else count
        F = np.zeros((count, MLP_IN), np.float32)
        Y = np.zeros(count, np.float32)
        _check(lib().sp_mlp_dataset(self._h, first, count, _fptr(F), _fptr(Y)))
        return F, Y

    def forward(self, F):
        """F: float32 (n x 5) CUDA tensor -> float32 CUDA tensor of n."""
        y = self._torch.empty(F.shape[0], dtype=self._torch.float32, device=F.device)
        _check(lib().sp_mlp_forward(self._h, _dev32(F), F.shape[0], _dev32(y),
                                    ctypes.c_void_p(self._torch.cuda.current_stream().cuda_stream)))
        return y

    def train_step(self, F, Y, lr):
        loss = ctypes.c_double(0.0)
        _check(lib().sp_mlp_train_step(self._h, _dev32(F), _dev32(Y), F.shape[0], lr, ctypes.byref(loss),
                                       ctypes.c_void_p(self._torch.cuda.current_stream().cuda_stream)))
        return loss.value

    def train(self, epochs, batch, lr):
        out = np.zeros(max(1, epochs))
        _check(lib().sp_mlp_train(self._h, epochs, batch, lr, _dptr(out),
                                  ctypes.c_void_p(self._torch.cuda.current_stream().cuda_stream)))
        return out[:epochs]


class SPMPS:
    """Handle of one SP-MPS state on the current HIP device.

    ``table``: an object with ``flat()`` returning (nsec, sec_n, sec_2m,
    sec_dim) and attributes L, N, twoM; ``blocks``: packed initial site
    tensors; ``mpo``: (w, data) as returned by :func:`mpo_hubbard`.
    """

    def __init__(self, table, blocks, mpo, twoS, G, stream=None, path="tiled", precision="fp64"):
        import torch
        self._torch = torch
        nsec, sn, s2m, sdim = (np.ascontiguousarray(a, dtype=np.int32) for a in table.flat())
        self._keep = (nsec, sn, s2m, sdim)
        self.L, self.N, self.twoM, self.twoS, self.G = table.L, table.N, table.twoM, twoS, G
        self.path = path
        self.precision = precision
        prob = _Problem(self.L, 4, self.N, twoS, self.twoM, G, {"fp64": SP_FP64, "fp32": SP_FP32, "bf16x3": SP_BF16X3}[precision],
                        {"tiled": SP_PATH_TILED, "plain": SP_PATH_PLAIN}[path])
        w, data = mpo
        w = np.ascontiguousarray(w, dtype=np.int32)
        data = np.ascontiguousarray(data, dtype=np.float64)
        m = _Mpo(_iptr(w), _dptr(data))
        bt = _BlockTable(_iptr(nsec), _iptr(sn), _iptr(s2m), _iptr(sdim))
        blocks = np.ascontiguousarray(blocks, dtype=np.float64)
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self.stream = stream
        h = ctypes.c_void_p()
        self.status = _check(lib().sp_init_mps(ctypes.byref(prob), ctypes.byref(m), ctypes.byref(bt), _dptr(blocks),
                                               ctypes.c_void_p(stream), ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(lib().sp_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def site_size(self, k):
        n = ctypes.c_longlong(0)
        _check(lib().sp_site_size(self._h, k, ctypes.byref(n)))
        return n.value

    def get_site(self, k):
        out = np.zeros(self.site_size(k))
        _check(lib().sp_get_site(self._h, k, _dptr(out)))
        return out

    def set_site(self, k, host):
        host = np.ascontiguousarray(host, dtype=np.float64)
        _check(lib().sp_set_site(self._h, k, _dptr(host)))

    def env_update(self, k, direction):
        _check(lib().sp_env_update(self._h, k, direction))

    def heff_apply(self, k, x, y, ny):
        _check(lib().sp_heff_apply(self._h, k, _dev(x), _dev(y), _dev(ny)))

    def heff_apply_noalloc(self, k, x, y, ny):
        """As heff_apply, with the library's fixed device scratch (no
        allocation in the call)."""
        _check(lib().sp_heff_apply_noalloc(self._h, k, _dev(x), _dev(y), _dev(ny)))

    def heff_diag(self, k, dh, dn):
        _check(lib().sp_heff_diag(self._h, k, _dev(dh), _dev(dn)))

    def heff_flops(self, k):
        f = ctypes.c_double(0)
        _check(lib().sp_heff_flops(self._h, k, ctypes.byref(f)))
        return f.value

    def heff_profile(self, k, x, y, ny, reps=20):
        """Per-launch timing of H_eff x at site k: dict of (ms, flops, bytes)
        for the left product, the mixing and the right product (plain path),
        or for the product, the once-per-local-problem pre-mixing of the left
        environment (block-product sites; not part of the product's time)
        and the g sum (tiled path)."""
        out = np.zeros(9)
        _check(lib().sp_heff_profile(self._h, k, reps, _dev(x), _dev(y), _dev(ny), _dptr(out)))
        names = (("left_product", "mixing", "right_product") if self.path == "plain"
                 else ("fused_heff", "premix_once", "g_sum"))
        return {n: dict(ms=out[i], flops=out[3 + i], bytes=out[6 + i]) for i, n in enumerate(names) if n}

    def center(self):
        c = ctypes.c_int(0)
        _check(lib().sp_center(self._h, ctypes.byref(c)))
        return c.value

    def energy(self):
        E, p = ctypes.c_double(0), ctypes.c_double(0)
        _check(lib().sp_energy(self._h, ctypes.byref(E), ctypes.byref(p)))
        return E.value, p.value

    def expect(self, mpo):
        """<O P>/<P> of a spin-free operator (an MPO as returned by the
        mpo_* builders) in the current projected state, and <P>."""
        w, data = mpo
        w = np.ascontiguousarray(w, dtype=np.int32)
        data = np.ascontiguousarray(data, dtype=np.float64)
        m = _Mpo(_iptr(w), _dptr(data))
        val, normp = np.zeros(1), np.zeros(1)
        _check(lib().sp_expect(self._h, ctypes.byref(m), _dptr(val), _dptr(normp)))
        return float(val[0]), float(normp[0])

    def one_rdm(self):
        """Spin-free one-body density matrix gamma_pq = <E_pq> (L x L)."""
        return np.array([[self.expect(mpo_epq(self.L, p, q))[0] for q in range(1, self.L + 1)]
                         for p in range(1, self.L + 1)])

    def spin_correlations(self):
        """<S_X . S_Y> for all site pairs (L x L)."""
        return np.array([[self.expect(mpo_spin_corr(self.L, x, y))[0] for y in range(1, self.L + 1)]
                         for x in range(1, self.L + 1)])

    def hubbard_energy_components(self, t, U):
        """e_p = <H_p P>/<P> of Sec. 2.4 for the open Hubbard chain, one
        sp_expect per site with the library's H_p MPO (sum_p e_p = E)."""
        return np.array([self.expect(mpo_hubbard_component(self.L, p, t, U))[0] for p in range(1, self.L + 1)])

    def abinitio_energy_components(self, h, eri):
        """e_p = <H_p P>/<P> of Sec. 2.4 for an ab-initio Hamiltonian."""
        return np.array([self.expect(mpo_abinitio_component(h, eri, p))[0] for p in range(1, self.L + 1)])

    def autotune(self, reps=5):
        """Pick the fused-kernel LDS budget (rows per task) of every site by
        timing; returns per-site (budget in doubles, rows, microseconds)."""
        b = np.zeros(self.L, dtype=np.int32)
        r = np.zeros(self.L, dtype=np.int32)
        us = np.zeros(self.L)
        _check(lib().sp_autotune(self._h, reps, _iptr(b), _iptr(r), _dptr(us)))
        return [(int(b[i]), int(r[i]), float(us[i])) for i in range(self.L)]

    def add_orthogonality(self, lower):
        """Keep this state orthogonal to ``lower`` (an SPMPS) in the projected
        metric in later sweeps (excited states)."""
        _check(lib().sp_add_orthogonality(self._h, lower._h))
        self._n_cons = getattr(self, "_n_cons", 0) + 1

    def clear_orthogonality(self):
        _check(lib().sp_clear_orthogonality(self._h))
        self._n_cons = 0

    def orthogonality_overlaps(self):
        """<lower_j|P|this> for every constraint, in the order added."""
        out = np.zeros(max(1, getattr(self, "_n_cons", 0)))
        _check(lib().sp_orthogonality_overlaps(self._h, _dptr(out)))
        return out[: getattr(self, "_n_cons", 0)]

    def set_precond(self, use=None, record=None):
        """Correct local solves with the MLP ``use`` (None: diagonal rule) and
        record training pairs into the MLP ``record`` (None: no recording)."""
        _check(lib().sp_set_precond(self._h, use._h if use is not None else None,
                                    record._h if record is not None else None))
        self._models = (use, record)  # keep them alive while attached

    def heff_plan(self, site):
        """(rows per task, LDS doubles) of the site's fused plan; (0, 0) when
        the site runs the tiled block products or the plain path."""
        rows, lds = ctypes.c_int(0), ctypes.c_int(0)
        _check(lib().sp_heff_plan(self._h, site, ctypes.byref(rows), ctypes.byref(lds)))
        return rows.value, lds.value

    def set_heff_plan(self, site, lds_budget):
        """Fused kernel with this LDS budget (doubles) at ``site``, or 0 for
        the tiled block products; returns the rows per task (0: tiled)."""
        rows = ctypes.c_int(0)
        _check(lib().sp_set_heff_plan(self._h, site, lds_budget, ctypes.byref(rows)))
        return rows.value

    def sweep(self, n_sweeps, tol=1e-9, max_iter=64, max_sub=32, keep=8, solver="auto", verbose=False):
        """Run sweeps; returns (status, list of per-step dicts).  solver:
        "host" (subspace solve on a host core), "device" (device-resident
        iteration replayed from a HIP graph) or "auto" (host for one state).
        verbose: the library prints a line per site step on stderr."""
        return sweep_batch([self], n_sweeps, tol, max_iter, max_sub, keep, _single=True, solver=solver,
                           verbose=verbose)


def _steps_out(steps, n):
    out = []
    for i in range(n):
        s = steps[i]
        out.append(dict(sweep=s.sweep, site=s.site, dir=s.dir, iters=s.iters, converged=bool(s.converged),
                        matvecs=s.matvecs, theta=s.theta, pnorm=s.pnorm, rnorm=s.rnorm, usec=s.usec))
    return out


def sweep_batch(states, n_sweeps, tol=1e-9, max_iter=64, max_sub=32, keep=8, _single=False, solver="auto",
                verbose=False):
    """Sweeps of several SPMPS states (``sp_sweep_batch``; one state:
    ``sp_sweep``).  solver: "auto" (device-resident iteration for two or more
    states, host-driven for one), "host" or "device".  Returns (status,
    per-state lists of step dicts); for a single state with _single=True,
    (status, step dicts)."""
    opts = _SweepOpts(n_sweeps, tol, max_iter, max_sub, keep, SOLVERS[solver], int(bool(verbose)))
    caps = [max(1, n_sweeps * max(1, 2 * (st.L - 1))) for st in states]
    bufs = [(_StepReport * c)() for c in caps]
    reps = (_SweepReport * len(states))(*[_SweepReport(c, 0, b) for c, b in zip(caps, bufs)])
    if _single:
        rc = _check(lib().sp_sweep(states[0]._h, ctypes.byref(opts), ctypes.byref(reps[0])))
        return rc, _steps_out(bufs[0], reps[0].n_steps)
    hs = (ctypes.c_void_p * len(states))(*[st._h.value for st in states])
    rc = _check(lib().sp_sweep_batch(hs, len(states), ctypes.byref(opts), reps))
    return rc, [_steps_out(bufs[i], reps[i].n_steps) for i in range(len(states))]
