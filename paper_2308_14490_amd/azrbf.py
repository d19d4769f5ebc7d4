"""Python binding of the azrbf C ABI (argument marshalling only).

Blocks of vectors are torch tensors on the GPU of shape (nvec, length), one
vector per row, unit stride along the row: as a column-major matrix that is
length x nvec with leading dimension ``t.stride(0)``, which is what the C
functions take.  Every computation runs in the HIP library; this module only
checks shapes and passes pointers and the current torch stream.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np
import torch   # imported before the library: the process keeps one HIP runtime

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libazrbf.so")

OK, EINVAL, EUNSUPPORTED, ENOMEM, EHIP, ERANK, ESTATE, ESCRATCH = 0, -1, -2, -3, -4, -5, -6, -7
OP_APPROX, OP_BVP = 0, 1


class AzrbfError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__(f"{where}: {_lib().azrbf_strerror(code).decode()} ({code})")


class _Problem(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32), ("n", ctypes.c_int32), ("s", ctypes.c_int32),
        ("T", ctypes.c_double), ("eps", ctypes.c_double), ("tau0", ctypes.c_double),
        ("op", ctypes.c_int32), ("k2", ctypes.c_double),
        ("mask", ctypes.POINTER(ctypes.c_uint8)), ("nb", ctypes.c_int64),
        ("bpts", ctypes.POINTER(ctypes.c_double)), ("bweight", ctypes.c_double),
        ("tau", ctypes.c_double), ("tauZ", ctypes.c_double), ("k", ctypes.c_int32),
        ("refine", ctypes.c_int32), ("seed", ctypes.c_uint64), ("ny", ctypes.c_int32), ("Ty", ctypes.c_double),
        ("btype", ctypes.POINTER(ctypes.c_uint8)), ("bnormal", ctypes.POINTER(ctypes.c_double)),
    ]


class _Info(ctypes.Structure):
    _fields_ = [
        ("N", ctypes.c_int64), ("M", ctypes.c_int64), ("Mb", ctypes.c_int64), ("L", ctypes.c_int64),
        ("k", ctypes.c_int32), ("rank", ctypes.c_int32), ("eps", ctypes.c_double),
        ("normA", ctypes.c_double), ("normZ", ctypes.c_double), ("zeroed", ctypes.c_int32),
        ("factored", ctypes.c_int32), ("sweeps", ctypes.c_int32), ("device_bytes", ctypes.c_int64),
    ]


_LIB = None
_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_D = ctypes.c_double

EXPORTS = {
    "azrbf_plan": (ctypes.c_int, [ctypes.POINTER(_Problem), _P, ctypes.POINTER(_P)]),
    "azrbf_plan_info": (ctypes.c_int, [_P, ctypes.POINTER(_Info)]),
    "azrbf_plan_dims": (ctypes.c_int, [_P, ctypes.POINTER(_I64)]),
    "azrbf_apply_A": (ctypes.c_int, [_P, _P, _I64, _I64, _D, _D, _P, _I64, _P]),
    "azrbf_apply_Zstar": (ctypes.c_int, [_P, _P, _I64, _I64, _D, _D, _P, _I64, _P]),
    "azrbf_rhs": (ctypes.c_int, [_P, _P, _I64, _P, _I64, _I64, _P, _I64, _P]),
    "azrbf_apply_AZstar": (ctypes.c_int, [_P, _P, _I64, _I64, _D, _D, _P, _I64, _P]),
    "azrbf_factor": (ctypes.c_int, [_P, _P]),
    "azrbf_solve": (ctypes.c_int, [_P, _P, _I64, _I64, _P, _I64, _P, _P]),
    "azrbf_solve_many": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(_P), ctypes.POINTER(_P),
                                        ctypes.POINTER(_I64), ctypes.POINTER(_I64), ctypes.POINTER(_P),
                                        ctypes.POINTER(_I64), ctypes.POINTER(_P), _P]),
    "azrbf_solve_batched": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(_P), ctypes.POINTER(_P),
                                           ctypes.POINTER(_I64), ctypes.POINTER(_I64), ctypes.POINTER(_P),
                                           ctypes.POINTER(_I64), ctypes.POINTER(_P), _P]),
    "azrbf_footprint_bytes": (ctypes.c_int64, [ctypes.POINTER(_Problem), _I64]),
    "azrbf_get_factor": (ctypes.c_int, [_P, ctypes.c_int32, _P, _I64, _P]),
    "azrbf_gaussian": (ctypes.c_int, [ctypes.c_uint64, _I64, _I64, _P, _I64, _P]),
    "azrbf_dgemm": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, _I64, _I64, _I64, _D, _P, _I64, _P, _I64,
                                   _D, _P, _I64, _P]),
    "azrbf_dgemm_noalloc": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, _I64, _I64, _I64, _D, _P, _I64, _P,
                                           _I64, _D, _P, _I64, _P]),
    "azrbf_autotune": (ctypes.c_int, [_P, _I64, _P, ctypes.c_char_p, _I64]),
    "azrbf_tune_table": (ctypes.c_int, [ctypes.c_char_p, _I64]),
    "azrbf_tune_load": (ctypes.c_int, [ctypes.c_char_p]),
    "azrbf_profile_enable": (ctypes.c_int, [ctypes.c_int32]),
    "azrbf_profile_report": (ctypes.c_int, [ctypes.c_char_p, _I64]),
    "azrbf_destroy": (None, [_P]),
    "azrbf_release_cached_memory": (ctypes.c_int, []),
    "azrbf_strerror": (ctypes.c_char_p, [ctypes.c_int]),
}


def _lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2308_14490_amd/build.py "
                              "(or __graft_entry__.build())")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _LIB = lib
    return _LIB


def _check(rc, where):
    if rc != OK:
        raise AzrbfError(rc, where)


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _vecs(t, length, name):
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda:
        raise TypeError(f"{name} must be a float64 CUDA tensor")
    if t.dim() == 1:
        t = t.view(1, -1)
    if t.dim() != 2 or t.shape[1] != length or t.stride(1) != 1:
        raise ValueError(f"{name} must have shape (nvec, {length}) with unit row stride")
    return t, t.shape[0], max(t.stride(0), length)


# ------------------------------------------------------------------ grids

def fine_grid(n, s, T):
    """x~_i = -T + i * 2T/(s n), i = 0..s n - 1 (eq. set_Xtilde)."""
    L = s * n
    return -T + np.arange(L, dtype=np.float64) * (2.0 * T / L)


def make_mask(dim, n, s, T, contains, ny=None, Ty=None):
    """Collocation mask on the fine grid: 1 where ``contains`` holds (2D:
    ix*Ly + iy; the y axis has ny centres on [-Ty, Ty), default n and T)."""
    xt = fine_grid(n, s, T)
    if dim == 1:
        return np.ascontiguousarray(contains(xt), dtype=np.uint8)
    yt = fine_grid(ny or n, s, Ty or T)
    X, Y = np.meshgrid(xt, yt, indexing="ij")
    return np.ascontiguousarray(contains(X, Y), dtype=np.uint8).ravel()


def collocation_points(dim, n, s, T, mask, ny=None, Ty=None):
    """Coordinates of the collocation rows, (M, dim), in row order."""
    xt = fine_grid(n, s, T)
    idx = np.nonzero(np.asarray(mask).ravel())[0]
    if dim == 1:
        return xt[idx][:, None]
    yt = fine_grid(ny or n, s, Ty or T)
    Ly = yt.size
    return np.stack([xt[idx // Ly], yt[idx % Ly]], axis=1)


# ------------------------------------------------------------------ plan

class Plan:
    """An azrbf plan (owns device memory until ``destroy`` or garbage collection)."""

    def __init__(self, dim, n, s, T, mask, eps=0.0, tau0=0.0, op=OP_APPROX, k2=0.0, bpts=None,
                 bweight=1.0, tau=1e-12, tauZ=1e-12, k=0, refine=1, seed=42, stream=None, ny=0, Ty=0.0,
                 btype=None, bnormal=None):
        """ny, Ty: the y axis of a 2D box (0: the same as n, T).  btype: per
        boundary point 0 (Dirichlet) or 1 (Neumann; None: all Dirichlet);
        bnormal: (nb, dim) unit outward normals, needed at Neumann points."""
        lib = _lib()
        self.dim, self.n, self.s, self.T = dim, n, s, T
        self.ny, self.Ty = int(ny or 0), float(Ty or 0.0)
        self._mask = np.ascontiguousarray(mask, dtype=np.uint8).ravel()
        bp = np.zeros((0, dim)) if bpts is None else np.ascontiguousarray(bpts, dtype=np.float64)
        self._bpts = np.ascontiguousarray(bp.reshape(-1, dim))
        pr = _Problem()
        pr.dim, pr.n, pr.s, pr.T = dim, n, s, float(T)
        pr.eps, pr.tau0, pr.op, pr.k2 = float(eps), float(tau0), op, float(k2)
        pr.mask = self._mask.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
        pr.nb = self._bpts.shape[0]
        pr.bpts = self._bpts.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if pr.nb else None
        pr.bweight, pr.tau, pr.tauZ = float(bweight), float(tau), float(tauZ)
        pr.k, pr.refine, pr.seed = int(k), int(refine), int(seed)
        pr.ny, pr.Ty = self.ny, self.Ty
        self._btype = self._bnormal = None
        if btype is not None and pr.nb:
            self._btype = np.ascontiguousarray(btype, dtype=np.uint8).ravel()
            if self._btype.size != pr.nb:
                raise ValueError("btype needs one entry per boundary point")
            pr.btype = self._btype.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
        if bnormal is not None and pr.nb:
            self._bnormal = np.ascontiguousarray(np.asarray(bnormal, dtype=np.float64).reshape(-1, dim))
            if self._bnormal.shape[0] != pr.nb:
                raise ValueError("bnormal needs one normal per boundary point")
            pr.bnormal = self._bnormal.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        self._prob = pr
        h = ctypes.c_void_p()
        _check(lib.azrbf_plan(ctypes.byref(pr), _stream(stream), ctypes.byref(h)), "azrbf_plan")
        self._h = h
        self.N, self.M, self.Mb, _, self.k = self.dims()
        self.Mt = self.M + self.Mb

    def dims(self):
        """(N, M, Mb, L, k) without waiting for the device."""
        d = (_I64 * 5)()
        _check(_lib().azrbf_plan_dims(self._h, d), "azrbf_plan_dims")
        return tuple(int(v) for v in d)

    def info(self):
        inf = _Info()
        _check(_lib().azrbf_plan_info(self._h, ctypes.byref(inf)), "azrbf_plan_info")
        return {f: getattr(inf, f) for f, _ in _Info._fields_}

    def destroy(self):
        if getattr(self, "_h", None):
            _lib().azrbf_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def points(self):
        return collocation_points(self.dim, self.n, self.s, self.T, self._mask, self.ny, self.Ty)


def plan(*args, **kw):
    return Plan(*args, **kw)


def apply_A(p, X, Y=None, alpha=1.0, beta=0.0, stream=None):
    """Y = alpha * A X + beta * Y; X (nvec, N) -> Y (nvec, M + Mb)."""
    X, nvec, ldx = _vecs(X, p.N, "X")
    if Y is None:
        Y = torch.empty((nvec, p.Mt), dtype=torch.float64, device=X.device)
    Y, nv2, ldy = _vecs(Y, p.Mt, "Y")
    if nv2 != nvec:
        raise ValueError("X and Y hold different numbers of vectors")
    _check(_lib().azrbf_apply_A(p.handle, X.data_ptr(), ldx, nvec, alpha, beta, Y.data_ptr(), ldy,
                                _stream(stream)), "azrbf_apply_A")
    return Y


def apply_Zstar(p, R, Z=None, alpha=1.0, beta=0.0, stream=None):
    """Z = alpha * Z* R + beta * Z; R (nvec, M + Mb) -> Z (nvec, N)."""
    R, nvec, ldr = _vecs(R, p.Mt, "R")
    if Z is None:
        Z = torch.empty((nvec, p.N), dtype=torch.float64, device=R.device)
    Z, nv2, ldz = _vecs(Z, p.N, "Z")
    if nv2 != nvec:
        raise ValueError("R and Z hold different numbers of vectors")
    _check(_lib().azrbf_apply_Zstar(p.handle, R.data_ptr(), ldr, nvec, alpha, beta, Z.data_ptr(), ldz,
                                    _stream(stream)), "azrbf_apply_Zstar")
    return Z


def apply_AZstar(p, R, Y=None, alpha=1.0, beta=0.0, stream=None):
    """Y = alpha * A Z* R + beta * Y; R (nvec, M + Mb) -> Y (nvec, M + Mb)."""
    R, nvec, ldr = _vecs(R, p.Mt, "R")
    if Y is None:
        Y = torch.empty((nvec, p.Mt), dtype=torch.float64, device=R.device)
    Y, nv2, ldy = _vecs(Y, p.Mt, "Y")
    if nv2 != nvec:
        raise ValueError("R and Y hold different numbers of vectors")
    _check(_lib().azrbf_apply_AZstar(p.handle, R.data_ptr(), ldr, nvec, alpha, beta, Y.data_ptr(), ldy,
                                     _stream(stream)), "azrbf_apply_AZstar")
    return Y


def factor(p, stream=None):
    """Factor the sketch; returns the retained rank (raises on errors other than ERANK)."""
    rc = _lib().azrbf_factor(p.handle, _stream(stream))
    if rc not in (OK, ERANK):
        _check(rc, "azrbf_factor")
    inf = p.info()
    p.k = inf["k"]          # the width may have grown
    return inf["rank"]


def rhs(p, F, G=None, B=None, stream=None):
    """Right-hand sides from interior data F (nrhs, M) and boundary data G
    (nrhs, Mb) (azrbf_rhs); returns B (nrhs, M + Mb)."""
    F, nrhs, ldf = _vecs(F, p.M, "F")
    if p.Mb:
        if G is None:
            raise ValueError("boundary data G is required for a plan with boundary rows")
        G, ng, ldg = _vecs(G, p.Mb, "G")
        if ng != nrhs:
            raise ValueError("F and G hold different numbers of vectors")
        gp = G.data_ptr()
    else:
        gp, ldg = None, 0
    if B is None:
        B = torch.empty((nrhs, p.Mt), dtype=torch.float64, device=F.device)
    B, nb2, ldb = _vecs(B, p.Mt, "B")
    if nb2 != nrhs:
        raise ValueError("F and B hold different numbers of vectors")
    _check(_lib().azrbf_rhs(p.handle, F.data_ptr(), ldf, gp, ldg, nrhs, B.data_ptr(), ldb, _stream(stream)),
           "azrbf_rhs")
    return B


def solve(p, B, X=None, relres=None, stream=None):
    """Least-squares solve A X = B; B (nrhs, M + Mb) -> X (nrhs, N).  Returns (X, relres)."""
    B, nrhs, ldb = _vecs(B, p.Mt, "B")
    if X is None:
        X = torch.empty((nrhs, p.N), dtype=torch.float64, device=B.device)
    X, nv2, ldx = _vecs(X, p.N, "X")
    if nv2 != nrhs:
        raise ValueError("B and X hold different numbers of vectors")
    if relres is None:
        relres = torch.empty(nrhs, dtype=torch.float64, device=B.device)
    if (relres.dtype != torch.float64 or not relres.is_cuda or not relres.is_contiguous()
            or relres.numel() < nrhs):
        raise ValueError(f"relres must be a contiguous float64 CUDA tensor of at least {nrhs} entries")
    _check(_lib().azrbf_solve(p.handle, B.data_ptr(), ldb, nrhs, X.data_ptr(), ldx, relres.data_ptr(),
                              _stream(stream)), "azrbf_solve")
    p.k = p.dims()[4]       # a first solve factors, and the width may have grown
    return X, relres


def _many_args(plans, Bs, Xs, rels):
    n = len(plans)
    hp = (ctypes.c_void_p * n)(*[p.handle.value for p in plans])
    bp = (ctypes.c_void_p * n)()
    xp = (ctypes.c_void_p * n)()
    rp = (ctypes.c_void_p * n)()
    ldb = (ctypes.c_int64 * n)()
    ldx = (ctypes.c_int64 * n)()
    nr = (ctypes.c_int64 * n)()
    for i, (p, B, X, r) in enumerate(zip(plans, Bs, Xs, rels)):
        B, nrhs, lb = _vecs(B, p.Mt, "B")
        X, _, lx = _vecs(X, p.N, "X")
        bp[i], xp[i], rp[i] = B.data_ptr(), X.data_ptr(), r.data_ptr()
        ldb[i], ldx[i], nr[i] = lb, lx, nrhs
    return hp, bp, ldb, nr, xp, ldx, rp


def solve_batched(plans, Bs, Xs=None, rels=None, stream=None):
    """Grouped solve of many (possibly repeated) plans in one call, each with
    its own right-hand sides; returns (Xs, relres list)."""
    n = len(plans)
    Xs = Xs or [torch.empty((B.shape[0], p.N), dtype=torch.float64, device=B.device) for p, B in zip(plans, Bs)]
    rels = rels or [torch.empty(B.shape[0], dtype=torch.float64, device=B.device) for B in Bs]
    args = _many_args(plans, Bs, Xs, rels)
    _check(_lib().azrbf_solve_batched(n, *args, _stream(stream)), "azrbf_solve_batched")
    for p in plans:
        p.k = p.dims()[4]
    return Xs, rels


def solve_many(plans, Bs, Xs=None, stream=None):
    """Solve several factored problems in one call; returns (Xs, relres list)."""
    n = len(plans)
    Xs = Xs or [torch.empty((B.shape[0], p.N), dtype=torch.float64, device=B.device) for p, B in zip(plans, Bs)]
    rels = [torch.empty(B.shape[0], dtype=torch.float64, device=B.device) for B in Bs]
    hp = (ctypes.c_void_p * n)(*[p.handle.value for p in plans])
    bp = (ctypes.c_void_p * n)()
    xp = (ctypes.c_void_p * n)()
    rp = (ctypes.c_void_p * n)()
    ldb = (ctypes.c_int64 * n)()
    ldx = (ctypes.c_int64 * n)()
    nr = (ctypes.c_int64 * n)()
    for i, (p, B, X, r) in enumerate(zip(plans, Bs, Xs, rels)):
        B, nrhs, lb = _vecs(B, p.Mt, "B")
        X, _, lx = _vecs(X, p.N, "X")
        bp[i], xp[i], rp[i] = B.data_ptr(), X.data_ptr(), r.data_ptr()
        ldb[i], ldx[i], nr[i] = lb, lx, nrhs
    _check(_lib().azrbf_solve_many(n, hp, bp, ldb, nr, xp, ldx, rp, _stream(stream)), "azrbf_solve_many")
    for p in plans:
        p.k = p.dims()[4]
    return Xs, rels


def footprint_bytes(p_or_prob, max_rhs=64):
    pr = p_or_prob._prob if isinstance(p_or_prob, Plan) else p_or_prob
    return int(_lib().azrbf_footprint_bytes(ctypes.byref(pr), int(max_rhs)))


def get_factor(p, which, stream=None):
    """which: 'omega' (k, N), 'Q' (k, M+Mb), 'R' (k, k) column j in row j, 'sigma' (k,)."""
    k = p.k
    dev = torch.device("cuda", torch.cuda.current_device())
    if which == "omega":
        out, code, ld = torch.empty((k, p.N), dtype=torch.float64, device=dev), 0, p.N
    elif which == "Q":
        out, code, ld = torch.empty((k, p.Mt), dtype=torch.float64, device=dev), 1, p.Mt
    elif which == "R":
        out, code, ld = torch.empty((k, k), dtype=torch.float64, device=dev), 2, k
    elif which == "sigma":
        out, code, ld = torch.empty(k, dtype=torch.float64, device=dev), 3, k
    else:
        raise ValueError(which)
    _check(_lib().azrbf_get_factor(p.handle, code, out.data_ptr(), ld, _stream(stream)), "azrbf_get_factor")
    return out


def gaussian(seed, rows, cols, stream=None):
    """The sketch generator: returns (cols, rows), row c holding column c."""
    dev = torch.device("cuda", torch.cuda.current_device())
    out = torch.empty((cols, rows), dtype=torch.float64, device=dev)
    _check(_lib().azrbf_gaussian(int(seed), rows, cols, out.data_ptr(), rows, _stream(stream)), "azrbf_gaussian")
    return out


def _colmajor(t, name):
    """A column-major matrix held as a (cols, rows) tensor: (rows, cols, ld)."""
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda or t.dim() != 2:
        raise TypeError(f"{name} must be a 2-D float64 CUDA tensor")
    if t.stride(1) != 1:
        raise ValueError(f"{name} must have unit row stride")
    return t.shape[1], t.shape[0], max(t.stride(0), t.shape[1], 1)


def dgemm(A, B, C=None, transa=False, transb=False, alpha=1.0, beta=0.0, stream=None, noalloc=False):
    """C = alpha op(A) op(B) + beta C on the matrix cores.  Matrices are
    column-major, held as (cols, rows) tensors (tensor row j = column j).
    noalloc: use azrbf_dgemm_noalloc (no device allocation; C must be given)."""
    ra, ca, lda = _colmajor(A, "A")
    rb, cb, ldb = _colmajor(B, "B")
    m, k = (ca, ra) if transa else (ra, ca)
    kb, n = (cb, rb) if transb else (rb, cb)
    if k != kb:
        raise ValueError(f"inner dimensions differ: {k} vs {kb}")
    if C is None:
        C = torch.zeros((n, m), dtype=torch.float64, device=A.device)
    rc_, cc_, ldc = _colmajor(C, "C")
    if (rc_, cc_) != (m, n):
        raise ValueError(f"C must hold a {m} x {n} matrix")
    fn = _lib().azrbf_dgemm_noalloc if noalloc else _lib().azrbf_dgemm
    _check(fn(int(bool(transa)), int(bool(transb)), m, n, k, float(alpha), A.data_ptr(), lda,
              B.data_ptr(), ldb, float(beta), C.data_ptr(), ldc, _stream(stream)),
           "azrbf_dgemm_noalloc" if noalloc else "azrbf_dgemm")
    return C


def autotune(p, nvec, stream=None):
    """Times the engine's tile shapes on the plan's operator; returns the report dict."""
    import json
    buf = ctypes.create_string_buffer(1 << 16)
    _check(_lib().azrbf_autotune(p.handle, int(nvec), _stream(stream), buf, len(buf)), "azrbf_autotune")
    return json.loads(buf.value.decode())


def tune_table():
    """The process-wide tile-shape table: {key: (C, rows, pairs)}."""
    buf = ctypes.create_string_buffer(1 << 16)
    _check(_lib().azrbf_tune_table(buf, len(buf)), "azrbf_tune_table")
    out = {}
    for line in buf.value.decode().splitlines():
        key, c, l, ch = line.split()
        out[key] = (int(c), int(l), int(ch))
    return out


def tune_load(table):
    """Loads {key: (C, rows, pairs)} into the process-wide table."""
    text = "".join(f"{k} {c} {l} {ch}\n" for k, (c, l, ch) in table.items())
    _check(_lib().azrbf_tune_load(text.encode()), "azrbf_tune_load")


def tune_save_file(path):
    import json
    with open(path, "w") as f:
        json.dump({k: list(v) for k, v in tune_table().items()}, f, indent=1, sort_keys=True)


def tune_load_file(path):
    import json
    with open(path) as f:
        tune_load({k: tuple(v) for k, v in json.load(f).items()})


def profile_enable(on=True):
    _check(_lib().azrbf_profile_enable(1 if on else 0), "azrbf_profile_enable")


def profile_report():
    """Per-kernel totals since the last report: list of dicts (name, calls, ms, max_ms, bytes)."""
    import json
    buf = ctypes.create_string_buffer(1 << 20)
    _check(_lib().azrbf_profile_report(buf, len(buf)), "azrbf_profile_report")
    return json.loads(buf.value.decode())


def release_cached_memory():
    _check(_lib().azrbf_release_cached_memory(), "azrbf_release_cached_memory")


def exported_symbols():
    return list(EXPORTS)
