"""Shared helpers of the GPU parity tests: run one (op, n, batch, placement)
case through the C-ABI and the same inputs through the FP64 oracle, and the
error metric.

Error metric (one reading of "within 1e-4 relative error"): per problem,
max |gpu - oracle| / max(max |oracle|, 2^-126) over the output elements the
contract defines, then the maximum over problems.
"""
from __future__ import annotations

import numpy as np

import oracle
from paper_2609_28179_amd import inputs

TOL = 1e-4
PACKS = (1, 2, 4, 8)
SCOPES = ("thread", "wave", "workgroup", "subwave")


def normwise(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    b = ref.shape[0]
    g = got.reshape(b, -1)
    r = ref.reshape(b, -1)
    den = np.maximum(np.max(np.abs(r), axis=1), 2.0 ** -126)
    return np.max(np.abs(g - r), axis=1) / den


def guarded(torch, arr_np, dev, pad=64):
    return _guarded(torch, arr_np, dev, pad)


def _guarded(torch, arr_np, dev, pad):
    """Device copy of arr with NaN guard bands of `pad` floats on each side.
    Returns (full_buffer, view); pad keeps 256-byte alignment."""
    flat = np.ascontiguousarray(arr_np).reshape(-1)
    full = torch.full((flat.size + 2 * pad,), float("nan"), dtype=torch.float32, device=dev)
    full[pad:pad + flat.size] = torch.from_numpy(flat.astype(np.float32)).to(dev)
    view = full[pad:pad + flat.size].view(arr_np.shape)
    return full, view


def guards_intact(full, pad=64):
    h = full.detach().cpu().numpy()
    return bool(np.isnan(h[:pad]).all() and np.isnan(h[-pad:]).all())


def run_case(glass, torch, op, n, batch, scope, pack, nrhs=1, trans=0, seed_extra=0, dev="cuda:0",
             case=None, check_guards=True, shift=0):
    """Run one case on the GPU and on the oracle.  Returns a dict with 'err'
    (max normwise error), 'status', and bit-exact flags where they apply.
    shift > 0 starts every operand `shift` floats past a 256-byte boundary
    (4-byte aligned only; the contract allows it)."""
    if case is None:
        case = inputs.make_case(op, n, batch, cfg=100, nrhs=nrhs, extra=seed_extra)
    force = (scope, pack)
    out = {"status": None}
    bufs = []
    pad = 64 + shift

    def guarded(torch, arr_np, dev):
        return _guarded(torch, arr_np, dev, pad)

    def g(name):
        full, view = guarded(torch, case[name], dev)
        bufs.append(full)
        return view

    if op == "gemm":
        A, B = g("A"), g("B")
        C_full, C = guarded(torch, np.zeros((batch, n, n), np.float32), dev)
        bufs.append(C_full)
        out["status"] = glass.glass_gemm_batched(n, n, n, batch, 1.0, A, B, 0.0, C, force)
        torch.cuda.synchronize()
        ref = oracle.gemm(case["A"], case["B"])
        out["err"] = normwise(C.cpu().numpy(), ref).max()
        out["out"] = C.cpu().numpy()
    elif op == "gemv":
        A, x = g("A"), g("x")
        y_full, y = guarded(torch, np.zeros((batch, n), np.float32), dev)
        bufs.append(y_full)
        out["status"] = glass.glass_gemv_batched(n, n, batch, 1.0, A, x, 0.0, y, force)
        torch.cuda.synchronize()
        ref = oracle.gemv(case["A"], case["x"])
        out["err"] = normwise(y.cpu().numpy(), ref).max()
        out["out"] = y.cpu().numpy()
    elif op in ("potrf", "posv"):
        A = g("A")
        info = torch.full((batch,), -7, dtype=torch.int32, device=dev)
        if op == "potrf":
            out["status"] = glass.glass_potrf_batched(n, batch, A, info, force)
            torch.cuda.synchronize()
            L_ref, info_ref = oracle.potrf(case["A"])
            Lg = A.cpu().numpy()
            out["err"] = normwise(np.tril(Lg), L_ref).max()
            out["out"] = Lg
        else:
            B = g("B")
            out["status"] = glass.glass_posv_batched(n, nrhs, batch, A, B, info, force)
            torch.cuda.synchronize()
            L_ref, X_ref, info_ref = oracle.posv(case["A"], case["B"])
            Lg = A.cpu().numpy()
            Xg = B.cpu().numpy()
            out["err"] = max(normwise(np.tril(Lg), L_ref).max(), normwise(Xg, X_ref).max())
            out["out"] = np.concatenate([Lg.reshape(batch, -1), Xg.reshape(batch, -1)], axis=1)
        iu = np.triu_indices(n, 1)
        up = Lg[:, iu[0], iu[1]]
        out["upper_pos_zero"] = bool((up == 0).all() and not np.signbit(up).any())
        out["info_exact"] = bool(np.array_equal(info.cpu().numpy(), info_ref))
    elif op == "potrs":
        L, B = g("L"), g("B")
        out["status"] = glass.glass_potrs_batched(n, nrhs, batch, L, B, force)
        torch.cuda.synchronize()
        ref = oracle.potrs(case["L"], case["B"])
        out["err"] = normwise(B.cpu().numpy(), ref).max()
        out["out"] = B.cpu().numpy()
    elif op == "trsv":
        L, x = g("L"), g("x")
        out["status"] = glass.glass_trsv_batched(n, batch, trans, L, x, force)
        torch.cuda.synchronize()
        ref = oracle.trsv(case["L"], case["x"], trans)
        out["err"] = normwise(x.cpu().numpy(), ref).max()
        out["out"] = x.cpu().numpy()
    elif op in ("se3_compose", "se3_inverse"):
        Ta = g("Ta")
        T_full, T = guarded(torch, np.zeros((batch, 4, 4), np.float32), dev)
        bufs.append(T_full)
        if op == "se3_compose":
            Tb = g("Tb")
            out["status"] = glass.glass_se3_batched(glass.OP_SE3_COMPOSE, batch, Ta, Tb, T, force)
            ref = oracle.se3_compose(case["Ta"], case["Tb"])
        else:
            out["status"] = glass.glass_se3_batched(glass.OP_SE3_INVERSE, batch, Ta, None, T, force)
            ref = oracle.se3_inverse(case["Ta"])
        torch.cuda.synchronize()
        Tg = T.cpu().numpy()
        out["err"] = normwise(Tg[:, :3, :], ref[:, :3, :]).max()
        out["row3_exact"] = bool(np.array_equal(Tg[:, 3, :], np.broadcast_to([0, 0, 0, 1], (batch, 4))))
        out["out"] = Tg
    else:
        raise ValueError(op)
    if check_guards:
        out["guards"] = all(guards_intact(b, pad) for b in bufs)
    return out
