"""SPCG (Sequential Preconditioned Conjugate Gradient) on MI355X / gfx950.

Python binding of the C ABI in ``include/spcg.h``: the functions below carry
the ABI's names and only marshal arguments (torch tensors give device
pointers and the stream); every step of the method runs in the HIP library
``libspcg.so``.  There is no fallback: if the library is not built, the
first call raises.
"""
import ctypes

import numpy as np
import torch

from . import _lib as L
from ._lib import (SPCG_BF16, SPCG_E_BREAKDOWN, SPCG_E_DTYPE, SPCG_E_HIP, SPCG_E_INVALID_ARG,
                   SPCG_E_NOMEM, SPCG_E_RANK, SPCG_E_SHAPE, SPCG_F32, SPCG_F64, SPCG_FP8E4M3,
                   SPCG_METHOD_FULL_PCG, SPCG_METHOD_SPCG, SPCG_OK, SPCG_W_NOT_CONVERGED)

__all__ = ["Context", "SpcgError", "spcg_sketch", "spcg_precond_build", "spcg_precond_from_r",
           "spcg_pcg_stage", "spcg_pcg_stage_noalloc", "spcg_solve", "spcg_solve_batched", "spcg_sketch_tables_host",
           "spcg_mlp_forward", "spcg_mlp_loss_grad", "spcg_mlp_adam", "mat", "load"]

_DTYPES = {
    torch.float64: SPCG_F64,
    torch.float32: SPCG_F32,
    torch.bfloat16: SPCG_BF16,
    torch.float8_e4m3fn: SPCG_FP8E4M3,
}


def load():
    return L.load()


class SpcgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"SPCG error {code}: {msg}")
        self.code = code


def mat(t, col_scale=None):
    """spcg_mat view of a 2-D device tensor with unit column stride."""
    if t.dim() == 1:
        t = t.unsqueeze(1)
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError("matrices must be 2-D row-major with unit column stride")
    if t.dtype not in _DTYPES:
        raise TypeError(f"unsupported dtype {t.dtype}")
    m = L.SpcgMat()
    m.data = t.data_ptr() if t.numel() else None
    m.dtype = _DTYPES[t.dtype]
    m.rows, m.cols = t.shape
    m.ld = max(t.stride(0), t.shape[1])
    m.col_scale = col_scale.data_ptr() if col_scale is not None else None
    return m


class Context:
    """spcg_ctx bound to a device and the current torch stream."""

    def __init__(self, device=0, stream=None):
        lib = load()
        dev = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        self.device = dev
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        h = ctypes.c_void_p()
        rc = lib.spcg_ctx_create(dev.index or 0, ctypes.c_void_p(self.stream.cuda_stream),
                                 ctypes.byref(h))
        if rc != SPCG_OK:
            raise SpcgError(rc, "spcg_ctx_create failed")
        self.h = h
        self.lib = lib

    def check(self, rc):
        if rc < 0:
            raise SpcgError(rc, self.lib.spcg_last_error(self.h).decode())
        return rc

    def close(self):
        if getattr(self, "h", None):
            self.lib.spcg_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Sketch:
    def __init__(self, ctx, h, keep):
        self.ctx, self.h, self._keep = ctx, h, keep
        info = L.SketchInfo()
        ctx.check(ctx.lib.spcg_sketch_get_info(h, ctypes.byref(info)))
        self.info = info
        self.sizes = [info.m[i] for i in range(info.K)]

    def view(self, stage):
        """(A, b, c2) spcg_mat views of sketched stage ``stage`` (-1: S_hat)."""
        A, b, c2 = L.SpcgMat(), L.SpcgMat(), ctypes.c_double()
        self.ctx.check(self.ctx.lib.spcg_sketch_view(self.h, stage, ctypes.byref(A),
                                                     ctypes.byref(b), ctypes.byref(c2)))
        return A, b, c2.value

    def view_tensor(self, stage):
        """Copies of the stored (unscaled) sketch rows of a stage as tensors."""
        A, b, c2 = self.view(stage)
        dt = {SPCG_F64: torch.float64, SPCG_F32: torch.float32, SPCG_BF16: torch.bfloat16}[A.dtype]
        es = {SPCG_F64: 8, SPCG_F32: 4, SPCG_BF16: 2}[A.dtype]
        Ah = _tensor_from_ptr(A.data, (A.rows, A.ld), dt, es, self.ctx.device)[:, :A.cols]
        bh = None
        if b.data:
            bh = _tensor_from_ptr(b.data, (b.rows, b.ld), torch.float64, 8,
                                  self.ctx.device)[:, :b.cols]
        return Ah.clone(), (bh.clone() if bh is not None else None), c2

    def export(self):
        info = self.info
        mK = self.sizes[-1] if self.sizes else 0
        slot = np.zeros(max(mK, 1), np.int32)
        hat = np.zeros(info.r, np.int32)
        perm = np.zeros(info.Np, np.int32)
        sign = np.zeros(max(info.Np // 8, 1), np.uint8)
        self.ctx.check(self.ctx.lib.spcg_sketch_export(
            self.ctx.h, self.h, slot.ctypes.data, hat.ctypes.data, perm.ctypes.data,
            sign.ctypes.data))
        return {"slot_rows": slot[:mK], "hat_rows": hat, "input_perm": perm, "sign_bits": sign}

    def free(self):
        if self.h:
            self.ctx.lib.spcg_sketch_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def _tensor_from_ptr(ptr, shape, dtype, es, device):
    n = int(np.prod(shape))
    if n == 0:
        return torch.empty(shape, dtype=dtype, device=device)
    # wrap the device pointer without copying via a DLPack-free route:
    # allocate a tensor and copy with the HIP runtime through torch
    out = torch.empty(shape, dtype=dtype, device=device)
    hip = ctypes.CDLL("libamdhip64.so.7")
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    torch.cuda.current_stream(device).synchronize()
    rc = hip.hipMemcpy(ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(ptr), n * es, 3)
    if rc != 0:
        raise SpcgError(-6, f"hipMemcpy failed ({rc})")
    return out


class Precond:
    def __init__(self, ctx, h, d):
        self.ctx, self.h, self.d = ctx, h, d

    def export(self):
        R = np.zeros((self.d, self.d), np.float64)
        passes = ctypes.c_int32()
        self.ctx.check(self.ctx.lib.spcg_precond_export(self.ctx.h, self.h, R.ctypes.data,
                                                        ctypes.byref(passes)))
        return R, passes.value

    def free(self):
        if self.h:
            self.ctx.lib.spcg_precond_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def _sketch_kind(kind):
    if kind in ("srht", L.SPCG_SKETCH_SRHT):
        return L.SPCG_SKETCH_SRHT
    if kind in ("cs", "count", L.SPCG_SKETCH_COUNT):
        return L.SPCG_SKETCH_COUNT
    raise ValueError(f"unknown sketch kind {kind!r}")


def _sizes(m_list):
    if not m_list:
        return None, 0
    arr = (ctypes.c_int64 * len(m_list))(*[int(m) for m in m_list])
    return arr, len(m_list)


def spcg_sketch(ctx, X, Y=None, seed=1, m0=0, m_max=0, r=0, growth=2, hat_only=False,
                col_scale=None, stage_dtype=0, transform_segment=0, kind="srht", m_list=None):
    sizes, n_sizes = _sizes(m_list)
    o = L.SketchOpts(seed=seed, m0=m0, m_max=m_max, r=r, growth=growth, hat_only=int(hat_only),
                     stage_dtype=stage_dtype, transform_segment=transform_segment, kind=_sketch_kind(kind))
    if sizes is not None:
        o.m_list = ctypes.cast(sizes, ctypes.POINTER(ctypes.c_int64))
        o.m_list_len = n_sizes
    Xm = mat(X, col_scale)
    Ym = mat(Y) if Y is not None else None
    h = ctypes.c_void_p()
    ctx.check(ctx.lib.spcg_sketch(ctx.h, ctypes.byref(Xm), ctypes.byref(Ym) if Ym else None,
                                  ctypes.byref(o), ctypes.byref(h)))
    return Sketch(ctx, h, (X, Y, col_scale))


def spcg_precond_build(ctx, sketch, qr_passes=0):
    h = ctypes.c_void_p()
    o = L.PrecondOpts(qr_passes=qr_passes)
    ctx.check(ctx.lib.spcg_precond_build(ctx.h, sketch.h, ctypes.byref(o), ctypes.byref(h)))
    return Precond(ctx, h, sketch.info.d)


def spcg_precond_from_r(ctx, R):
    R = R.to(device=ctx.device, dtype=torch.float64).contiguous()
    h = ctypes.c_void_p()
    ctx.check(ctx.lib.spcg_precond_from_r(ctx.h, ctypes.c_void_p(R.data_ptr()), R.shape[0],
                                          ctypes.byref(h)))
    torch.cuda.current_stream(ctx.device).synchronize()
    return Precond(ctx, h, R.shape[0])


def _as_mat(a, col_scale=None):
    return a if isinstance(a, L.SpcgMat) else mat(a, col_scale)


def spcg_pcg_stage(ctx, A, b, c2, precond, beta, iters, tol=0.0, refresh=False, check_every=1,
                   col_scale=None):
    """PCG on c2 A^T A x = c2 A^T b from x = beta (updated in place)."""
    Am, bm = _as_mat(A, col_scale), _as_mat(b)
    o = L.StageOpts(iters=iters, refresh_gradient=int(refresh), tol=tol, check_every=check_every)
    st = L.StageStats()
    rc = ctx.check(ctx.lib.spcg_pcg_stage(ctx.h, ctypes.byref(Am), ctypes.byref(bm), c2, precond.h,
                                          ctypes.c_void_p(beta.data_ptr()), ctypes.byref(o),
                                          ctypes.byref(st)))
    return {"iters": st.iters, "converged": bool(st.converged), "rho0": st.rho0, "rho": st.rho,
            "ax_norm": st.ax_norm, "resid_norm2": st.resid_norm2, "rc": rc}


def spcg_pcg_stage_noalloc(ctx, A, b, c2, precond, beta, iters, tol=0.0, refresh=False,
                           check_every=1, col_scale=None):
    """spcg_pcg_stage on the library's static scratch (k = 1, d <= 1024): the
    call allocates no device memory."""
    Am, bm = _as_mat(A, col_scale), _as_mat(b)
    o = L.StageOpts(iters=iters, refresh_gradient=int(refresh), tol=tol, check_every=check_every)
    st = L.StageStats()
    rc = ctx.check(ctx.lib.spcg_pcg_stage_noalloc(ctx.h, ctypes.byref(Am), ctypes.byref(bm), c2,
                                                  precond.h, ctypes.c_void_p(beta.data_ptr()),
                                                  ctypes.byref(o), ctypes.byref(st)))
    return {"iters": st.iters, "converged": bool(st.converged), "rho0": st.rho0, "rho": st.rho,
            "ax_norm": st.ax_norm, "resid_norm2": st.resid_norm2, "rc": rc}


def solve_opts(method="spcg", seed=1, a=3, T=100, tol=5e-7, m0=0, m_max=0, r=0, growth=2,
               qr_passes=0, check_every=1, time_phases=False, time_products=False, a_list=None,
               stage_stride=1, schedule="plain", weights=None, schedule_margin=0,
               record_features=False, stage_dtype=0, transform_segment=0, sketch="srht",
               batch_direct=False, batch_tasks_per_cu=0, m_list=None, a_rule="fixed", omega=0.0,
               nested_gradient=True, stage_limit=0, batch_shape=0, batch_one_launch=False):
    """spcg_solve_opts from keyword arguments (``sketch``: "srht" or "cs",
    the CountSketch of SPCG-CS).  schedule='learned' needs
    ``weights``: a float32 device tensor of SPCG_MLP_PARAMS entries (see
    ``schedule.load_weights``)."""
    o = L.SolveOpts()
    ctx_lib = load()
    ctx_lib.spcg_solve_opts_default(ctypes.byref(o))
    o.sketch.seed, o.sketch.m0, o.sketch.m_max, o.sketch.r, o.sketch.growth = seed, m0, m_max, r, growth
    o.sketch.stage_dtype = stage_dtype
    o.sketch.transform_segment = transform_segment
    o.sketch.kind = _sketch_kind(sketch)
    o.batch_direct = int(batch_direct)
    o.batch_tasks_per_cu = batch_tasks_per_cu
    o.batch_shape = batch_shape
    o.batch_one_launch = int(batch_one_launch)
    sizes, n_sizes = _sizes(m_list)
    if sizes is not None:
        o.sketch.m_list = ctypes.cast(sizes, ctypes.POINTER(ctypes.c_int64))
        o.sketch.m_list_len = n_sizes
    if a_rule not in ("fixed", "theory", L.SPCG_A_FIXED, L.SPCG_A_THEORY):
        raise ValueError(f"unknown a_rule {a_rule!r}")
    o.a_rule = L.SPCG_A_THEORY if a_rule in ("theory", L.SPCG_A_THEORY) else L.SPCG_A_FIXED
    o.omega = omega
    o.nested_gradient = int(nested_gradient)
    o.stage_limit = stage_limit
    o.precond.qr_passes = qr_passes
    o.method = SPCG_METHOD_FULL_PCG if method in ("pcg", "full_pcg", SPCG_METHOD_FULL_PCG) else SPCG_METHOD_SPCG
    o.a, o.T, o.tol, o.check_every = a, T, tol, check_every
    o.time_phases, o.time_products = int(time_phases), int(time_products)
    o.stage_stride = stage_stride
    o.schedule = L.SPCG_SCHEDULE_LEARNED if schedule in ("learned", L.SPCG_SCHEDULE_LEARNED) else L.SPCG_SCHEDULE_PLAIN
    if schedule not in ("plain", "learned", 0, 1):
        raise ValueError(f"unknown schedule {schedule!r}")
    if weights is not None:
        if weights.dtype != torch.float32 or not weights.is_cuda or weights.numel() != L.SPCG_MLP_PARAMS:
            raise ValueError("weights must be a float32 device tensor of SPCG_MLP_PARAMS entries")
        o.schedule_weights = weights.data_ptr()
    o.schedule_margin = schedule_margin
    o.record_features = int(record_features)
    keep = [sizes]   # host arrays the options point to, alive until the call returns
    if a_list is not None:
        arr = (ctypes.c_int32 * len(a_list))(*a_list)
        keep.append(arr)
        o.a_list = ctypes.cast(arr, ctypes.POINTER(ctypes.c_int32))
        o.a_list_len = len(a_list)
    return o, keep


def spcg_solve(ctx, X, Y, beta=None, col_scale=None, **kw):
    """Algorithm 1 (or full-data PCG with method='pcg'); returns (beta, stats).

    Y may have k > 1 columns (beta is then d x k)."""
    o, keep = solve_opts(**kw)
    Xm, Ym = mat(X, col_scale), mat(Y)
    if beta is None:
        k = Y.shape[1] if Y.dim() == 2 else 1
        shape = (X.shape[1],) if k == 1 else (X.shape[1], k)
        beta = torch.empty(shape, dtype=torch.float64, device=X.device)
    st = L.SolveStats()
    rc = ctx.check(ctx.lib.spcg_solve(ctx.h, ctypes.byref(Xm), ctypes.byref(Ym), ctypes.byref(o),
                                      ctypes.c_void_p(beta.data_ptr()), ctypes.byref(st)))
    del keep
    stats = _stats_dict(st)
    stats["rc"] = rc
    return beta, stats


def _stats_dict(st):
    out = {}
    for f, _ in L.SolveStats._fields_:
        v = getattr(st, f)
        out[f] = list(v) if isinstance(v, ctypes.Array) else v
    return out


def spcg_solve_batched(ctx, Xs, Ys, betas=None, **kw):
    """Batched / multi-RHS form: independent problems (Xs[p], Ys[p]) solved
    together; returns (betas, stats_list) with betas[p] of shape d x k."""
    n = len(Xs)
    o, keep = solve_opts(**kw)
    xm = (L.SpcgMat * n)(*[mat(x) for x in Xs])
    ym = (L.SpcgMat * n)(*[mat(y) for y in Ys])
    if betas is None:
        betas = [torch.empty(x.shape[1], y.shape[1], dtype=torch.float64, device=x.device)
                 for x, y in zip(Xs, Ys)]
    ptrs = (ctypes.c_void_p * n)(*[b.data_ptr() for b in betas])
    st = (L.SolveStats * n)()
    rc = ctx.check(ctx.lib.spcg_solve_batched(ctx.h, n, xm, ym, ctypes.byref(o), ptrs, st))
    del keep
    stats = []
    for i in range(n):
        d = _stats_dict(st[i])
        d["rc"] = rc
        stats.append(d)
    return betas, stats


def spcg_sketch_tables_host(seed, L_bits, m, r):
    """Sketch randomness from the library's host code (no GPU needed)."""
    lib = load()
    np_ = 1 << L_bits
    slot = np.zeros(max(m, 1), np.int32)
    hat = np.zeros(max(r, 1), np.int32)
    perm = np.zeros(np_, np.int32)
    sign = np.zeros(max(np_ // 8, 1), np.uint8)
    rc = lib.spcg_sketch_tables_host(seed, L_bits, m, r, slot.ctypes.data, hat.ctypes.data,
                                     perm.ctypes.data, sign.ctypes.data)
    if rc != SPCG_OK:
        raise SpcgError(rc, "spcg_sketch_tables_host failed")
    return {"slot_rows": slot[:m], "hat_rows": hat[:r], "input_perm": perm,
            "sign_bits": sign[:np_ // 8]}


# ------------------------------------------------------------ schedule network

def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _check_f32(t, numel, name):
    if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous() or t.numel() != numel:
        raise ValueError(f"{name}: expected a contiguous float32 device tensor of {numel} entries")


def spcg_mlp_forward(ctx, W, feats, out=None):
    """Network outputs (n x 7) for features (n x 8), both float32 on the device."""
    n = feats.shape[0]
    _check_f32(W, L.SPCG_MLP_PARAMS, "W")
    _check_f32(feats, n * L.SPCG_MLP_F, "feats")
    if out is None:
        out = torch.empty(n, L.SPCG_MLP_O, dtype=torch.float32, device=feats.device)
    _check_f32(out, n * L.SPCG_MLP_O, "out")
    ctx.check(ctx.lib.spcg_mlp_forward(ctx.h, _ptr(W), _ptr(feats), n, _ptr(out)))
    return out


def spcg_mlp_loss_grad(ctx, W, feats, a_label, g_label, s_label, w_a, w_s, grad=None, loss=None):
    """(grad, loss) of the mean schedule loss; every argument a device tensor
    (labels int32, the rest float32)."""
    n = feats.shape[0]
    _check_f32(W, L.SPCG_MLP_PARAMS, "W")
    _check_f32(feats, n * L.SPCG_MLP_F, "feats")
    for t, name in ((s_label, "s_label"), (w_a, "w_a"), (w_s, "w_s")):
        _check_f32(t, n, name)
    for t, name in ((a_label, "a_label"), (g_label, "g_label")):
        if t.dtype != torch.int32 or not t.is_cuda or t.numel() != n or not t.is_contiguous():
            raise ValueError(f"{name}: expected a contiguous int32 device tensor of {n} entries")
    if grad is None:
        grad = torch.empty(L.SPCG_MLP_PARAMS, dtype=torch.float32, device=W.device)
    if loss is None:
        loss = torch.empty(1, dtype=torch.float32, device=W.device)
    ctx.check(ctx.lib.spcg_mlp_loss_grad(ctx.h, _ptr(W), _ptr(feats), _ptr(a_label), _ptr(g_label),
                                         _ptr(s_label), _ptr(w_a), _ptr(w_s), n, _ptr(grad), _ptr(loss)))
    return grad, loss


def spcg_mlp_adam(ctx, W, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step on W (in place), moments m and v updated in place."""
    n = W.numel()
    for t, name in ((W, "W"), (grad, "grad"), (m, "m"), (v, "v")):
        _check_f32(t, n, name)
    ctx.check(ctx.lib.spcg_mlp_adam(ctx.h, _ptr(W), _ptr(grad), _ptr(m), _ptr(v), n, step, lr, beta1,
                                    beta2, eps))
