"""Thin ctypes binding of libglass.so (include/glass.h).

The ``glass_*`` functions carry the C names and argument order and only
marshal arguments: a torch tensor becomes its device pointer, ``force``
becomes a ``glass_placement_t``, ``stream=None`` becomes torch's current
stream.  They return the integer status.  The short helpers below them
(``gemm``, ``posv``, ...) check dtype / device / contiguity / shape, allocate
outputs with torch and raise :class:`GlassError` on a nonzero status.

Importing this module loads the built library and raises ImportError when it
is missing: there is no fallback path.

torch is imported before the library is loaded.  torch's HIP build asks for
its own copy of the HIP runtime by the unversioned file name; were the
library (which asks for ``libamdhip64.so.7``) loaded first, the process would
hold two runtimes, and torch's streams and allocations would belong to the
other one (launches then fail with hipErrorNoDevice).  Loaded after torch,
the library binds to torch's runtime.
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (must precede the CDLL below, see above)

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libglass.so")

OK, ERR_INVALID_VALUE, ERR_UNSUPPORTED, ERR_INFEASIBLE_PLACEMENT, ERR_LAUNCH = 0, -1, -2, -3, -4
OP_GEMM, OP_GEMV, OP_POTRF, OP_POTRS, OP_POSV, OP_TRSV, OP_SE3_COMPOSE, OP_SE3_INVERSE, OP_POSV_ADJOINT = range(9)
SCOPE_THREAD, SCOPE_WAVE, SCOPE_WORKGROUP, SCOPE_SUBWAVE = 0, 1, 2, 3
OPS = {"gemm": OP_GEMM, "gemv": OP_GEMV, "potrf": OP_POTRF, "potrs": OP_POTRS, "posv": OP_POSV,
       "trsv": OP_TRSV, "se3_compose": OP_SE3_COMPOSE, "se3_inverse": OP_SE3_INVERSE}
SCOPES = {"thread": SCOPE_THREAD, "wave": SCOPE_WAVE, "workgroup": SCOPE_WORKGROUP, "subwave": SCOPE_SUBWAVE}
SCOPE_NAMES = {v: k for k, v in SCOPES.items()}
RAGGED_SCOPES = SCOPES


class Placement(ctypes.Structure):
    _fields_ = [("scope", ctypes.c_int32), ("pack", ctypes.c_int32),
                ("wg_threads", ctypes.c_int32), ("problems_per_wg", ctypes.c_int32)]

    def __repr__(self):
        return (f"Placement({SCOPE_NAMES.get(self.scope, self.scope)}, P={self.pack}, "
                f"threads={self.wg_threads}, problems/wg={self.problems_per_wg})")


class GlassError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        super().__init__(f"{what}: {status_string(status)} ({status})")


if not os.path.exists(LIB_PATH):
    raise ImportError(f"libglass.so is not built ({LIB_PATH}); run __graft_entry__.build()")
_lib = ctypes.CDLL(LIB_PATH)

_i, _f, _p = ctypes.c_int, ctypes.c_float, ctypes.c_void_p
_PP = ctypes.POINTER(Placement)
_SIGS = {
    "glass_gemm_batched": [_i, _i, _i, _i, _f, _p, _p, _f, _p, _PP, _p],
    "glass_gemm_batched_ex": [_i, _i, _i, _i, _i, _i, _f, _p, _p, _f, _p, _PP, _p],
    "glass_gemv_batched": [_i, _i, _i, _f, _p, _p, _f, _p, _PP, _p],
    "glass_potrf_batched": [_i, _i, _p, _p, _PP, _p],
    "glass_potrs_batched": [_i, _i, _i, _p, _p, _PP, _p],
    "glass_posv_batched": [_i, _i, _i, _p, _p, _p, _PP, _p],
    "glass_trsv_batched": [_i, _i, _i, _p, _p, _PP, _p],
    "glass_se3_batched": [_i, _i, _p, _p, _p, _PP, _p],
    "glass_posv_adjoint_batched": [_i, _i, _i, _p, _p, _p, _p, _p, _PP, _p],
    "glass_posv_ragged": [_i, _p, _p, _p, _p, _p, _p, _p, _p, ctypes.c_size_t, _p, _p],
    "glass_posv_ragged_noalloc": [_i, _p, _p, _p, _p, _p, _p, _p, _p, _p],
    "glass_posv_ragged_noalloc_max_count": [],
    "glass_posv_ragged_workspace_size": [_i],
    "glass_posv_ragged_perm_offset": [_i],
    "glass_stream_probe": [_i, _p, _p, _p, ctypes.c_longlong, _i, _p],
    "glass_riccati_gain_batched": [_i, _i, _i, _p, _p, _p, _p, _p, _p, _PP, _p],
    "glass_riccati_feasible": [_i, _i, _i],
    "glass_riccati_placement_feasible": [_i, _i, _i, _i],
    "glass_ragged_table_provenance": [],
    "glass_last_launch_error": [],
    "glass_hip_error_name": [_i],
    "glass_mlp_num_params": [_i],
    "glass_mlp_forward": [_i, _i, _p, _p, _p, _p, _p, _p],
    "glass_mlp_backward_workspace_size": [_i, _i],
    "glass_mlp_backward": [_i, _i, _p, _p, _p, _p, _p, _p, _p, _p, ctypes.c_size_t, _p],
    "glass_mlp_adam": [_i, _p, _p, _p, _p, _i, _f, _f, _f, _f, _p],
    "glass_query_placement": [_i, _i, _i, _PP],
    "glass_placement_feasible": [_i, _i, _i, _i, _i],
    "glass_table_provenance": [],
    "glass_status_string": [_i],
}
for _name, _args in _SIGS.items():
    _fn = getattr(_lib, _name)
    _fn.argtypes = _args
    _fn.restype = ctypes.c_char_p if _name in ("glass_table_provenance", "glass_status_string",
                                               "glass_hip_error_name", "glass_ragged_table_provenance") \
        else ctypes.c_int
    if _name in ("glass_posv_ragged_workspace_size", "glass_posv_ragged_perm_offset", "glass_mlp_num_params",
                 "glass_mlp_backward_workspace_size"):
        _fn.restype = ctypes.c_size_t

EXPORTED = tuple(_SIGS)


# ----------------------------------------------------------------- marshalling
def _ptr(t):
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _force(force):
    if force is None:
        return None
    if isinstance(force, Placement):
        return ctypes.byref(force)
    scope, pack = force
    if isinstance(scope, str):
        scope = SCOPES[scope]
    return ctypes.byref(Placement(scope, pack, 0, 0))


# ------------------------------------------------------------ C-named wrappers
def glass_gemm_batched(m, n, k, batch, alpha, A, B, beta, C, force=None, stream=None) -> int:
    return _lib.glass_gemm_batched(m, n, k, batch, alpha, _ptr(A), _ptr(B), beta, _ptr(C), _force(force),
                                   _stream(stream))


def glass_gemm_batched_ex(transa, transb, m, n, k, batch, alpha, A, B, beta, C, force=None, stream=None) -> int:
    return _lib.glass_gemm_batched_ex(transa, transb, m, n, k, batch, alpha, _ptr(A), _ptr(B), beta, _ptr(C),
                                      _force(force), _stream(stream))


def glass_gemv_batched(m, n, batch, alpha, A, x, beta, y, force=None, stream=None) -> int:
    return _lib.glass_gemv_batched(m, n, batch, alpha, _ptr(A), _ptr(x), beta, _ptr(y), _force(force),
                                   _stream(stream))


def glass_potrf_batched(n, batch, A, info=None, force=None, stream=None) -> int:
    return _lib.glass_potrf_batched(n, batch, _ptr(A), _ptr(info), _force(force), _stream(stream))


def glass_potrs_batched(n, nrhs, batch, L, B, force=None, stream=None) -> int:
    return _lib.glass_potrs_batched(n, nrhs, batch, _ptr(L), _ptr(B), _force(force), _stream(stream))


def glass_posv_batched(n, nrhs, batch, A, B, info=None, force=None, stream=None) -> int:
    return _lib.glass_posv_batched(n, nrhs, batch, _ptr(A), _ptr(B), _ptr(info), _force(force), _stream(stream))


def glass_trsv_batched(n, batch, trans, L, x, force=None, stream=None) -> int:
    return _lib.glass_trsv_batched(n, batch, trans, _ptr(L), _ptr(x), _force(force), _stream(stream))


def glass_se3_batched(op, batch, Ta, Tb, Tout, force=None, stream=None) -> int:
    return _lib.glass_se3_batched(op, batch, _ptr(Ta), _ptr(Tb), _ptr(Tout), _force(force), _stream(stream))


def glass_posv_adjoint_batched(n, nrhs, batch, L, X, G, dB, dA, force=None, stream=None) -> int:
    return _lib.glass_posv_adjoint_batched(n, nrhs, batch, _ptr(L), _ptr(X), _ptr(G), _ptr(dB), _ptr(dA),
                                           _force(force), _stream(stream))


def glass_posv_ragged(count, n, nrhs, offA, offB, A, B, info, workspace, workspace_bytes, class_scope=None,
                      stream=None) -> int:
    cs = None
    if class_scope is not None:
        vals = [RAGGED_SCOPES[v] if isinstance(v, str) else int(v) for v in class_scope]
        cs = (ctypes.c_int32 * 8)(*vals)
    return _lib.glass_posv_ragged(count, _ptr(n), _ptr(nrhs), _ptr(offA), _ptr(offB), _ptr(A), _ptr(B), _ptr(info),
                                  _ptr(workspace), workspace_bytes, cs, _stream(stream))


def glass_posv_ragged_noalloc(count, n, nrhs, offA, offB, A, B, info, class_scope=None, stream=None) -> int:
    cs = None
    if class_scope is not None:
        vals = [RAGGED_SCOPES[v] if isinstance(v, str) else int(v) for v in class_scope]
        cs = (ctypes.c_int32 * 8)(*vals)
    return _lib.glass_posv_ragged_noalloc(count, _ptr(n), _ptr(nrhs), _ptr(offA), _ptr(offB), _ptr(A), _ptr(B),
                                          _ptr(info), cs, _stream(stream))


def glass_posv_ragged_noalloc_max_count() -> int:
    return _lib.glass_posv_ragged_noalloc_max_count()


def glass_posv_ragged_workspace_size(count) -> int:
    return _lib.glass_posv_ragged_workspace_size(count)


def glass_posv_ragged_perm_offset(count) -> int:
    return _lib.glass_posv_ragged_perm_offset(count)


def glass_riccati_gain_batched(nx, nu, batch, A, B, P, R, K, info=None, force=None, stream=None) -> int:
    return _lib.glass_riccati_gain_batched(nx, nu, batch, _ptr(A), _ptr(B), _ptr(P), _ptr(R), _ptr(K), _ptr(info),
                                           _force(force), _stream(stream))


def glass_stream_probe(kind, a, b, c, n4, blocks, stream=None) -> int:
    return _lib.glass_stream_probe(kind, _ptr(a), _ptr(b), _ptr(c), n4, blocks, _stream(stream))


def glass_riccati_feasible(nx, nu, pack) -> int:
    return _lib.glass_riccati_feasible(nx, nu, pack)


def glass_riccati_placement_feasible(nx, nu, scope, pack) -> int:
    return _lib.glass_riccati_placement_feasible(nx, nu, scope, pack)


def glass_ragged_table_provenance() -> str:
    return _lib.glass_ragged_table_provenance().decode()


def glass_last_launch_error() -> int:
    return _lib.glass_last_launch_error()


def glass_hip_error_name(code) -> str:
    return _lib.glass_hip_error_name(code).decode()


def glass_mlp_num_params(d) -> int:
    return _lib.glass_mlp_num_params(d)


def glass_mlp_forward(N, d, X, params, H1, H2, y, stream=None) -> int:
    return _lib.glass_mlp_forward(N, d, _ptr(X), _ptr(params), _ptr(H1), _ptr(H2), _ptr(y), _stream(stream))


def glass_mlp_backward_workspace_size(N, d) -> int:
    return _lib.glass_mlp_backward_workspace_size(N, d)


def glass_mlp_backward(N, d, X, params, H1, H2, y, t, grad, workspace, workspace_bytes, stream=None) -> int:
    return _lib.glass_mlp_backward(N, d, _ptr(X), _ptr(params), _ptr(H1), _ptr(H2), _ptr(y), _ptr(t), _ptr(grad),
                                   _ptr(workspace), workspace_bytes, _stream(stream))


def glass_mlp_adam(P, params, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None) -> int:
    return _lib.glass_mlp_adam(P, _ptr(params), _ptr(grad), _ptr(m), _ptr(v), step, lr, beta1, beta2, eps,
                               _stream(stream))


def glass_query_placement(op, n, batch) -> Placement:
    out = Placement()
    st = _lib.glass_query_placement(op, n, batch, ctypes.byref(out))
    if st != OK:
        raise GlassError(st, "glass_query_placement")
    return out


def glass_placement_feasible(op, n, nrhs, scope, pack) -> int:
    return _lib.glass_placement_feasible(op, n, nrhs, scope, pack)


def glass_table_provenance() -> str:
    return _lib.glass_table_provenance().decode()


def status_string(status: int) -> str:
    return _lib.glass_status_string(status).decode()


# ----------------------------------------------------------- checked helpers
def _check(t, name, shape=None, dtype=None):
    import torch
    dtype = dtype or torch.float32
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


def _raise(st, what):
    if st == ERR_LAUNCH:
        code = _lib.glass_last_launch_error()
        raise GlassError(st, f"{what} [HIP {_lib.glass_hip_error_name(code).decode()} ({code})]")
    if st != OK:
        raise GlassError(st, what)


def gemm(A, B, C=None, alpha=1.0, beta=0.0, force=None):
    import torch
    b, m, k = A.shape
    n = B.shape[2]
    _check(A, "A", (b, m, k))
    _check(B, "B", (b, k, n))
    if C is None:
        C = torch.empty((b, m, n), dtype=torch.float32, device=A.device)
    _check(C, "C", (b, m, n))
    _raise(glass_gemm_batched(m, n, k, b, alpha, A, B, beta, C, force), "gemm")
    return C


def gemv(A, x, y=None, alpha=1.0, beta=0.0, force=None):
    import torch
    b, m, n = A.shape
    _check(A, "A", (b, m, n))
    _check(x, "x", (b, n))
    if y is None:
        y = torch.empty((b, m), dtype=torch.float32, device=A.device)
    _check(y, "y", (b, m))
    _raise(glass_gemv_batched(m, n, b, alpha, A, x, beta, y, force), "gemv")
    return y


def potrf_(A, info=None, force=None):
    """In place: A <- L (strict upper +0).  Returns (A, info)."""
    import torch
    b, n, _ = A.shape
    _check(A, "A", (b, n, n))
    if info is None:
        info = torch.empty((b,), dtype=torch.int32, device=A.device)
    _check(info, "info", (b,), torch.int32)
    _raise(glass_potrf_batched(n, b, A, info, force), "potrf")
    return A, info


def potrs_(L, B, force=None):
    b, n, _ = L.shape
    _check(L, "L", (b, n, n))
    _check(B, "B", (b, n, B.shape[2]))
    _raise(glass_potrs_batched(n, B.shape[2], b, L, B, force), "potrs")
    return B


def posv_(A, B, info=None, force=None):
    import torch
    b, n, _ = A.shape
    _check(A, "A", (b, n, n))
    _check(B, "B", (b, n, B.shape[2]))
    if info is None:
        info = torch.empty((b,), dtype=torch.int32, device=A.device)
    _check(info, "info", (b,), torch.int32)
    _raise(glass_posv_batched(n, B.shape[2], b, A, B, info, force), "posv")
    return A, B, info


def trsv_(L, x, trans=0, force=None):
    b, n, _ = L.shape
    _check(L, "L", (b, n, n))
    _check(x, "x", (b, n))
    _raise(glass_trsv_batched(n, b, trans, L, x, force), "trsv")
    return x


def se3_compose(Ta, Tb, out=None, force=None):
    import torch
    b = Ta.shape[0]
    _check(Ta, "Ta", (b, 4, 4))
    _check(Tb, "Tb", (b, 4, 4))
    if out is None:
        out = torch.empty_like(Ta)
    _check(out, "out", (b, 4, 4))
    _raise(glass_se3_batched(OP_SE3_COMPOSE, b, Ta, Tb, out, force), "se3_compose")
    return out


def se3_inverse(Ta, out=None, force=None):
    import torch
    b = Ta.shape[0]
    _check(Ta, "Ta", (b, 4, 4))
    if out is None:
        out = torch.empty_like(Ta)
    _check(out, "out", (b, 4, 4))
    _raise(glass_se3_batched(OP_SE3_INVERSE, b, Ta, None, out, force), "se3_inverse")
    return out


def posv_adjoint(L, X, G, force=None):
    """(dB, dA) = (A^{-1} G, -(dB X^T + X dB^T) / 2) for A = L L^T."""
    import torch
    b, n, _ = L.shape
    r = X.shape[2]
    _check(L, "L", (b, n, n))
    _check(X, "X", (b, n, r))
    _check(G, "G", (b, n, r))
    dB = torch.empty_like(X)
    dA = torch.empty_like(L)
    _raise(glass_posv_adjoint_batched(n, r, b, L, X, G, dB, dA, force), "posv_adjoint")
    return dB, dA


class Ragged:
    """A packed ragged batch on the device plus its workspace (tensors kept)."""

    def __init__(self, case: dict, device="cuda:0"):
        import torch
        self.count = len(case["n"])
        t = lambda a: torch.from_numpy(a).to(device)
        self.n, self.nrhs, self.offA, self.offB = t(case["n"]), t(case["nrhs"]), t(case["offA"]), t(case["offB"])
        self.A, self.B = t(case["A"]), t(case["B"])
        self.info = torch.zeros(self.count, dtype=torch.int32, device=device)
        self.ws_bytes = glass_posv_ragged_workspace_size(self.count)
        self.ws = torch.empty((self.ws_bytes + 3) // 4, dtype=torch.int32, device=device)

    def solve(self, class_scope=None, stream=None):
        _raise(glass_posv_ragged(self.count, self.n, self.nrhs, self.offA, self.offB, self.A, self.B, self.info,
                                 self.ws, self.ws_bytes, class_scope, stream), "posv_ragged")

    def perm(self):
        off = glass_posv_ragged_perm_offset(self.count) // 4
        return self.ws[off:off + self.count]
