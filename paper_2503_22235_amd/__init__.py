"""Python binding of libwm, the MI355X latent-processor library.

Argument marshalling only: every computation runs in the HIP kernels of
libwm.so (built in-tree by ``paper_2503_22235_amd.build``).  Function names
are those of the C ABI in include/wm.h.  Tensor arguments are torch device
tensors (or raw integer device addresses); streams default to torch's
current stream.  If the library is missing, every call raises: there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import os

__all__ = [
    "WM_F32", "WM_BF16", "WM_FP8_E4M3", "WmError", "wm_grid", "lib",
    "wm_version", "wm_ctx_create", "wm_ctx_destroy", "wm_nat_indices",
    "wm_nat_forward", "wm_layernorm", "wm_linear", "wm_processor_create",
    "wm_processor_destroy", "wm_processor_block", "wm_processor_step", "wm_processor_step_states",
    "wm_processor_set_rope",
    "wm_schedule", "wm_rollout", "wm_forecast_hourly", "wm_relerr_l2", "grid_of", "LIB_PATH",
    "wm_prof_enable", "wm_prof_select", "wm_prof_collect", "PROF_KINDS", "wm_serve_create",
    "wm_serve_submit", "wm_serve_poll", "wm_serve_status", "wm_serve_destroy",
    "wm_quantize_fp8", "wm_linear_fp8", "wm_nat_forward_noalloc", "WM_NAT_NOALLOC_SCRATCH_BYTES",
]

WM_F32, WM_BF16, WM_FP8_E4M3 = 0, 1, 2
WM_NAT_NOALLOC_SCRATCH_BYTES = 4 << 20   # the fixed per-device scratch of wm_nat_forward_noalloc
LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libwm.so")


class WmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libwm error {code}: {msg}")
        self.code = code


class wm_serve_cfg(ctypes.Structure):
    _fields_ = [("max_batch", ctypes.c_int), ("state_bf16", ctypes.c_int),
                ("hbm_budget_bytes", ctypes.c_size_t), ("max_slots", ctypes.c_int), ("graphs", ctypes.c_int)]


class wm_req_stats(ctypes.Structure):
    _fields_ = [("id", ctypes.c_uint64), ("lead_hours", ctypes.c_int), ("steps", ctypes.c_int),
                ("batches", ctypes.c_int), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double),
                ("max_cobatch", ctypes.c_int)]


class wm_grid(ctypes.Structure):
    _fields_ = [("Z", ctypes.c_int), ("Y", ctypes.c_int), ("X", ctypes.c_int),
                ("C", ctypes.c_int), ("heads", ctypes.c_int),
                ("Kz", ctypes.c_int), ("Ky", ctypes.c_int), ("Kx", ctypes.c_int),
                ("periodic_mask", ctypes.c_uint)]


def grid_of(g) -> wm_grid:
    """wm_grid from any object with Z, Y, X, C, heads, Kz, Ky, Kx fields."""
    if isinstance(g, wm_grid):
        return g
    return wm_grid(g.Z, g.Y, g.X, g.C, g.heads, g.Kz, g.Ky, g.Kx,
                   getattr(g, "periodic_mask", 0x4))


_LIB = None
_vp = ctypes.c_void_p
_int = ctypes.c_int

# name -> (restype, argtypes)
_SIGS = {
    "wm_last_error": (ctypes.c_char_p, []),
    "wm_version": (ctypes.c_char_p, []),
    "wm_ctx_create": (_int, [_int, ctypes.POINTER(_vp)]),
    "wm_ctx_destroy": (None, [_vp]),
    "wm_nat_indices": (_int, [ctypes.POINTER(wm_grid), _vp, _vp]),
    "wm_nat_forward": (_int, [_vp, ctypes.POINTER(wm_grid), _int, _int, _vp, _vp, _vp, _vp, _vp, _vp]),
    "wm_nat_forward_noalloc": (_int, [ctypes.POINTER(wm_grid), _int, _int, _vp, _vp, _vp, _vp, _vp, _vp]),
    "wm_layernorm": (_int, [_int, _int, _vp, _vp, _vp, ctypes.c_float, _int, _vp, _vp]),
    "wm_linear": (_int, [_int, _int, _int, _int, _vp, _vp, _vp, _int, _vp, _vp]),
    "wm_processor_create": (_int, [_vp, ctypes.POINTER(wm_grid), _int, _int, _int, _vp, ctypes.POINTER(_vp)]),
    "wm_processor_destroy": (None, [_vp]),
    "wm_processor_blocks": (_int, [_vp]),
    "wm_processor_set_rope": (_int, [_vp, _int]),
    "wm_processor_block": (_int, [_vp, _vp, _int, _int, _vp, _vp]),
    "wm_processor_step": (_int, [_vp, _vp, _int, _vp, _vp]),
    "wm_processor_step_states": (_int, [_vp, _vp, _int, _vp, _vp]),
    "wm_schedule": (_int, [_int, ctypes.POINTER(_int), _int]),
    "wm_rollout": (_int, [_vp, _vp, _vp, _int, _vp, _int, _vp]),
    "wm_forecast_hourly": (_int, [_vp, _vp, _vp, _vp, _int, _vp, _int, _vp]),
    "wm_relerr_l2": (ctypes.c_double, [_vp, _vp, _vp, ctypes.c_size_t, _vp]),
    "wm_prof_enable": (_int, [_vp, _int]),
    "wm_prof_select": (_int, [_vp, ctypes.c_uint]),
    "wm_serve_create": (_int, [_vp, _vp, _vp, ctypes.POINTER(wm_serve_cfg), ctypes.POINTER(_vp)]),
    "wm_serve_submit": (_int, [_vp, _vp, _int, ctypes.POINTER(ctypes.c_uint64)]),
    "wm_serve_poll": (_int, [_vp, ctypes.c_uint64, _vp, ctypes.POINTER(wm_req_stats)]),
    "wm_serve_status": (_int, [_vp, ctypes.POINTER(_int), ctypes.POINTER(_int), ctypes.POINTER(_int),
                               ctypes.POINTER(_int)]),
    "wm_serve_destroy": (None, [_vp]),
    "wm_quantize_fp8": (_int, [ctypes.c_size_t, _vp, ctypes.c_float, _vp, _vp]),
    "wm_linear_fp8": (_int, [_int, _int, _int, _vp, ctypes.c_float, _vp, ctypes.c_float, _vp, _int, _vp, _vp]),
    "wm_prof_collect": (_int, [_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_longlong), _int]),
}

PROF_KINDS = ("ln1", "qkv", "nat", "proj", "ln2", "mlp1", "mlp2")


def lib():
    """The loaded libwm.so (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with paper_2503_22235_amd.build.build() "
                "(no CPU fallback exists)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = L
    return _LIB


def _check(rc):
    if rc < 0:
        raise WmError(rc, lib().wm_last_error().decode())
    return rc


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream(s):
    if s is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(s, int):
        return s
    return s.cuda_stream


def wm_version() -> str:
    return lib().wm_version().decode()


class Ctx:
    def __init__(self, handle):
        self.handle = handle

    def close(self):
        if self.handle:
            lib().wm_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Processor:
    def __init__(self, handle, grid, n_blocks, prec):
        self.handle = handle
        self.grid = grid
        self.n_blocks = n_blocks
        self.prec = prec

    def close(self):
        if self.handle:
            lib().wm_processor_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def wm_ctx_create(device: int = 0) -> Ctx:
    h = _vp()
    _check(lib().wm_ctx_create(device, ctypes.byref(h)))
    return Ctx(h.value)


def wm_ctx_destroy(ctx: Ctx):
    ctx.close()


def wm_nat_indices(grid, out, stream=None):
    g = grid_of(grid)
    return _check(lib().wm_nat_indices(ctypes.byref(g), _ptr(out), _stream(stream)))


def wm_nat_forward(ctx, grid, B, prec, q, k, v, rpb, out, stream=None):
    g = grid_of(grid)
    return _check(lib().wm_nat_forward(ctx.handle, ctypes.byref(g), B, prec, _ptr(q), _ptr(k),
                                       _ptr(v), _ptr(rpb), _ptr(out), _stream(stream)))


def wm_nat_forward_noalloc(grid, B, prec, q, k, v, rpb, out, stream=None):
    g = grid_of(grid)
    return _check(lib().wm_nat_forward_noalloc(ctypes.byref(g), B, prec, _ptr(q), _ptr(k), _ptr(v),
                                               _ptr(rpb), _ptr(out), _stream(stream)))


def wm_layernorm(M, C, x, gamma, beta, eps, out_prec, out, stream=None):
    return _check(lib().wm_layernorm(M, C, _ptr(x), _ptr(gamma), _ptr(beta), eps, out_prec,
                                     _ptr(out), _stream(stream)))


def wm_linear(M, N, K, prec, a, w, bias, epilogue, out, stream=None):
    return _check(lib().wm_linear(M, N, K, prec, _ptr(a), _ptr(w), _ptr(bias), epilogue,
                                  _ptr(out), _stream(stream)))


def wm_processor_create(ctx, grid, n_blocks, mlp_ratio, prec, host_params) -> Processor:
    """host_params: numpy float32 array in the canonical parameter order."""
    import numpy as np
    hp = np.ascontiguousarray(host_params, dtype=np.float32)
    g = grid_of(grid)
    h = _vp()
    _check(lib().wm_processor_create(ctx.handle, ctypes.byref(g), n_blocks, mlp_ratio, prec,
                                     hp.ctypes.data, ctypes.byref(h)))
    return Processor(h.value, g, n_blocks, prec)


def wm_processor_destroy(p: Processor):
    p.close()


def wm_processor_set_rope(p, on=True):
    return _check(lib().wm_processor_set_rope(p.handle, 1 if on else 0))


def wm_processor_block(ctx, p, block, B, x, stream=None):
    return _check(lib().wm_processor_block(ctx.handle, p.handle, block, B, _ptr(x), _stream(stream)))


def wm_processor_step(ctx, p, B, x, stream=None):
    return _check(lib().wm_processor_step(ctx.handle, p.handle, B, _ptr(x), _stream(stream)))


def wm_processor_step_states(ctx, p, B, dev_states, stream=None):
    """dev_states: a device tensor (int64) holding B state addresses."""
    return _check(lib().wm_processor_step_states(ctx.handle, p.handle, B, _ptr(dev_states), _stream(stream)))


def wm_schedule(lead_hours: int):
    n = _check(lib().wm_schedule(lead_hours, None, 0))
    buf = (_int * max(n, 1))()
    _check(lib().wm_schedule(lead_hours, buf, n))
    return [buf[i] for i in range(n)]


def wm_rollout(ctx, p6, p1, B, x, lead_hours, stream=None):
    return _check(lib().wm_rollout(ctx.handle, p6.handle, p1.handle, B, _ptr(x), lead_hours,
                                   _stream(stream)))


def wm_forecast_hourly(ctx, p6, p1, x, hours, outs=None, batch=8, stream=None):
    """outs: None or a sequence of `hours` device tensors / None entries
    (outs[L-1] receives the state at lead L)."""
    arr = None
    if outs is not None:
        if len(outs) != hours:
            raise ValueError("outs must have one entry per hour")
        arr = (ctypes.c_void_p * hours)(*[(_ptr(o) if o is not None else None) for o in outs])
    return _check(lib().wm_forecast_hourly(ctx.handle, p6.handle, p1.handle, _ptr(x), hours, arr, batch,
                                           _stream(stream)))


def wm_quantize_fp8(x, mul, out, stream=None):
    return _check(lib().wm_quantize_fp8(x.numel(), _ptr(x), mul, _ptr(out), _stream(stream)))


def wm_linear_fp8(M, N, K, a8, a_dequant, w8, w_dequant, bias, epilogue, out, stream=None):
    return _check(lib().wm_linear_fp8(M, N, K, _ptr(a8), a_dequant, _ptr(w8), w_dequant, _ptr(bias),
                                      epilogue, _ptr(out), _stream(stream)))


def wm_prof_enable(ctx, on=True):
    return _check(lib().wm_prof_enable(ctx.handle, 1 if on else 0))


def wm_prof_select(ctx, kinds):
    """Time only the given kinds (names from PROF_KINDS)."""
    mask = 0
    for k in kinds:
        mask |= 1 << PROF_KINDS.index(k)
    return _check(lib().wm_prof_select(ctx.handle, mask))


def wm_prof_collect(ctx):
    """{kind: (total_ms, launches)} of the kernels recorded since the last collect."""
    n = len(PROF_KINDS)
    ms = (ctypes.c_double * n)()
    cnt = (ctypes.c_longlong * n)()
    _check(lib().wm_prof_collect(ctx.handle, ms, cnt, n))
    return {k: (ms[i], cnt[i]) for i, k in enumerate(PROF_KINDS)}


def wm_relerr_l2(ctx, y, y_ref, n=None, stream=None) -> float:
    if n is None:
        n = y.numel()
    r = lib().wm_relerr_l2(ctx.handle, _ptr(y), _ptr(y_ref), n, _stream(stream))
    if r < 0:
        raise WmError(int(r), lib().wm_last_error().decode())
    return r


class Server:
    def __init__(self, handle, elems):
        self.handle = handle
        self.elems = elems

    def close(self):
        if self.handle:
            lib().wm_serve_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def wm_serve_create(ctx, p6, p1, max_batch=8, state_bf16=True, hbm_budget_bytes=0, max_slots=0, graphs=False):
    cfg = wm_serve_cfg(max_batch, 1 if state_bf16 else 0, hbm_budget_bytes, max_slots, 1 if graphs else 0)
    h = _vp()
    _check(lib().wm_serve_create(ctx.handle, p6.handle, p1.handle, ctypes.byref(cfg), ctypes.byref(h)))
    g = p6.grid
    return Server(h.value, g.Z * g.Y * g.X * g.C)


def wm_serve_submit(server, x0, lead_hours) -> int:
    """x0: host float32 array of one state [Z, Y, X, C] (copied before return)."""
    import numpy as np
    a = np.ascontiguousarray(x0, dtype=np.float32)
    if a.size != server.elems:
        raise ValueError(f"state has {a.size} values, server expects {server.elems}")
    rid = ctypes.c_uint64()
    _check(lib().wm_serve_submit(server.handle, a.ctypes.data, lead_hours, ctypes.byref(rid)))
    return rid.value


def wm_serve_poll(server, rid, out=None):
    """(done, stats): done is False while pending; out (float32 numpy) receives the state."""
    st = wm_req_stats()
    ptr = out.ctypes.data if out is not None else None
    rc = lib().wm_serve_poll(server.handle, rid, ptr, ctypes.byref(st))
    if rc == -3:
        return False, None
    _check(rc)
    return True, {f: getattr(st, f) for f, _ in wm_req_stats._fields_}


def wm_serve_status(server):
    q, r, d, s = _int(), _int(), _int(), _int()
    _check(lib().wm_serve_status(server.handle, ctypes.byref(q), ctypes.byref(r), ctypes.byref(d),
                                 ctypes.byref(s)))
    return {"queued": q.value, "running": r.value, "done": d.value, "slots": s.value}


def wm_serve_destroy(server):
    server.close()
