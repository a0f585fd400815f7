"""ctypes binding of libbpdc.so: argument marshalling only.

Every array handed to a decode entry point is a torch tensor on the current
HIP device; its data pointer goes to the C ABI, together with the current
torch stream.  Nothing here computes any part of the decoder.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libbpdc.so")

KERNEL_AUTO, KERNEL_PLAIN, KERNEL_LANE, KERNEL_GROUP = 0, 1, 2, 3
PRIOR_CHANNEL, PRIOR_POSTERIOR = 0, 1
TIE_HASH, TIE_LOWEST_INDEX = 0, 1
RULE_MIN_SUM, RULE_PRODUCT_SUM = 0, 1
FLAG_BAD_CODE = 0x80  # multi-code shot whose code index is out of range (skipped)

EXPORTS = [
    "bpdc_code_create", "bpdc_code_destroy", "bpdc_code_info", "bpdc_plan_create",
    "bpdc_plan_destroy", "bpdc_plan_info", "bpdc_workspace_size", "bpdc_decode",
    "bpdc_decode_multi", "bpdc_graph_capture_multi", "bpdc_graph_launch",
    "bpdc_wms_ckpt_size", "bpdc_wms_forward", "bpdc_wms_backward", "bpdc_lane_precompile",
    "bpdc_plan_set_dc_stats", "bpdc_decode_noalloc", "bpdc_plan_describe", "bpdc_eval_phi",
    "bpdc_status_string", "bpdc_last_error", "bpdc_version",
]


class BpdcError(RuntimeError):
    pass


class _Csr(C.Structure):
    _fields_ = [("rows", C.c_int32), ("cols", C.c_int32),
                ("row_ptr", C.POINTER(C.c_int32)), ("col_idx", C.POINTER(C.c_int32))]


class _Params(C.Structure):
    _fields_ = [("max_iter", C.c_int32 * 2), ("alpha", C.c_float), ("second_pass_prior", C.c_int32),
                ("stop_on_converge", C.c_int32), ("llr_sat", C.c_float), ("tie_eps", C.c_float),
                ("tie_break", C.c_int32), ("seed", C.c_uint64), ("rule", C.c_int32),
                ("soft_period", C.c_int32), ("soft_shift", C.c_float)]


_lib = None


def lib_path() -> str:
    return LIB


def lib():
    """Load libbpdc.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise BpdcError(f"{LIB} not found: build it with paper_2510_08695_amd/build.py")
        L = C.CDLL(LIB)
        P, I32, I64, U64 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64
        sig = {
            "bpdc_code_create": [C.POINTER(_Csr), C.POINTER(_Csr), P, C.POINTER(P)],
            "bpdc_code_destroy": [P],
            "bpdc_code_info": [P, P, P, P, P],
            "bpdc_plan_create": [P, I32, C.POINTER(_Params), I32, C.POINTER(P)],
            "bpdc_plan_destroy": [P],
            "bpdc_plan_info": [P, I32, P, P, P],
            "bpdc_workspace_size": [P, I32, I64, C.POINTER(C.c_size_t)],
            "bpdc_decode": [P, I32, P, I64, I64, P, P, P, P, P, P, C.c_size_t, P],
            "bpdc_decode_multi": [P, P, P, P, P, P, P, P, I64, I64, P, C.c_size_t, P],
            "bpdc_graph_capture_multi": [P, P, P, P, P, P, P, P, I64, I64, P, C.c_size_t, P],
            "bpdc_graph_launch": [P, P],
            "bpdc_wms_ckpt_size": [P, I32, I64, I32, C.POINTER(C.c_size_t)],
            "bpdc_wms_forward": [P, I32, P, P, I64, I64, I32, P, P, P, P, C.c_size_t, P],
            "bpdc_wms_backward": [P, I32, P, P, I64, I32, P, P, P, P, C.c_size_t, P, P],
            "bpdc_lane_precompile": [C.POINTER(_Csr), C.POINTER(_Csr), I32, I32, I32, I32],
            "bpdc_plan_set_dc_stats": [P, P, I64],
            "bpdc_decode_noalloc": [P, I32, P, I64, I64, P, P, P, P, P, P],
            "bpdc_plan_describe": [P, I32, C.c_char_p, C.c_size_t, C.POINTER(C.c_size_t)],
            "bpdc_eval_phi": [P, I64, P, P],
        }
        for name, args in sig.items():
            if not hasattr(L, name):
                continue
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int32
        for name in ("bpdc_status_string",):
            getattr(L, name).restype = C.c_char_p
            getattr(L, name).argtypes = [C.c_int32]
        for name in ("bpdc_last_error", "bpdc_version"):
            getattr(L, name).restype = C.c_char_p
            getattr(L, name).argtypes = []
        _lib = L
    return _lib


def _check(status: int):
    if status != 0:
        L = lib()
        raise BpdcError(f"{L.bpdc_status_string(status).decode()}: {L.bpdc_last_error().decode()}")


def _csr(M):
    rp = np.ascontiguousarray(M.row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(M.col_idx, dtype=np.int32)
    if ci.size == 0:
        ci = np.zeros(1, np.int32)
    s = _Csr(int(M.rows), int(M.cols), rp.ctypes.data_as(C.POINTER(C.c_int32)),
             ci.ctypes.data_as(C.POINTER(C.c_int32)))
    return s, (rp, ci)


@dataclass
class Params:
    max_iter: Sequence[int] = (100, 100)
    alpha: float = 0.625
    second_pass_prior: int = PRIOR_CHANNEL
    stop_on_converge: bool = True
    llr_sat: float = 64.0
    tie_eps: float = 1e-3
    tie_break: int = TIE_HASH
    seed: int = 0
    rule: int = RULE_MIN_SUM
    soft_period: int = 0      # intermittent soft DC every soft_period first-pass iterations (0: off)
    soft_shift: float = 0.0   # prior-LLR increase of each soft nominee

    def to_c(self) -> _Params:
        p = _Params()
        p.max_iter[0], p.max_iter[1] = int(self.max_iter[0]), int(self.max_iter[1])
        p.alpha = self.alpha
        p.second_pass_prior = int(self.second_pass_prior)
        p.stop_on_converge = 1 if self.stop_on_converge else 0
        p.llr_sat = self.llr_sat
        p.tie_eps = self.tie_eps
        p.tie_break = int(self.tie_break)
        p.seed = int(self.seed) & 0xFFFFFFFFFFFFFFFF
        p.rule = int(self.rule)
        p.soft_period = int(self.soft_period)
        p.soft_shift = float(self.soft_shift)
        return p


def lane_precompile(H, D, posterior: bool = False, uniform_prior: bool = True, rule: int = RULE_MIN_SUM,
                    soft: bool = False) -> None:
    """Compile the code-specialised lane kernel into the on-disk cache (no GPU needed)."""
    h, keep_h = _csr(H)
    d, keep_d = _csr(D)
    _check(lib().bpdc_lane_precompile(C.byref(h), C.byref(d), 1 if posterior else 0,
                                      1 if uniform_prior else 0, int(rule), 1 if soft else 0))


class Code:
    """A decoding problem resident on the current device (H, D, priors)."""

    def __init__(self, H, D, priors):
        h, keep_h = _csr(H)
        d, keep_d = _csr(D)
        pri = np.ascontiguousarray(priors, dtype=np.float64)
        handle = C.c_void_p()
        _check(lib().bpdc_code_create(C.byref(h), C.byref(d), pri.ctypes.data_as(C.c_void_p),
                                      C.byref(handle)))
        self.handle = handle
        n, m, md, e = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib().bpdc_code_info(handle, C.byref(n), C.byref(m), C.byref(md), C.byref(e)))
        self.n, self.m, self.md, self.edges = n.value, m.value, md.value, e.value

    @classmethod
    def from_problem(cls, code) -> "Code":
        return cls(code.H, code.D, code.priors)

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib().bpdc_code_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Plan:
    """Launch plan for one or more codes (kernel family chosen per code)."""

    def __init__(self, codes: Sequence[Code], params: Params, kernel: int = KERNEL_AUTO):
        self.codes = list(codes)
        self.params = params
        arr = (C.c_void_p * len(self.codes))(*[c.handle for c in self.codes])
        handle = C.c_void_p()
        p = params.to_c()
        _check(lib().bpdc_plan_create(arr, len(self.codes), C.byref(p), int(kernel), C.byref(handle)))
        self.handle = handle
        self._ws = {}

    def info(self, code: int = 0):
        k, s, t = C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib().bpdc_plan_info(self.handle, code, C.byref(k), C.byref(s), C.byref(t)))
        return {"kernel": k.value, "shots_per_wg": s.value, "threads": t.value}

    def describe(self, code: int = 0) -> dict:
        """The autotuner's record for `code` (-1: the multi-code launch): the tile kept and
        every candidate timed (bpdc_plan_describe)."""
        import json
        need = C.c_size_t()
        _check(lib().bpdc_plan_describe(self.handle, code, None, 0, C.byref(need)))
        buf = C.create_string_buffer(need.value)
        _check(lib().bpdc_plan_describe(self.handle, code, buf, need.value, None))
        return json.loads(buf.value.decode())

    def set_dc_stats(self, stats=None):
        """Accumulate DC diagnostics of later decodes into `stats` (int64 tensor of at least
        103 + n words on the GPU, zeroed by the caller), or stop (None).  Layout: [0, 101)
        histogram of floor(100 * spread) of the first-pass posterior error probabilities over
        each row of D on shots that ran DC, [101] number of such shots, [102, 103 + n) cut sizes."""
        if stats is None:
            _check(lib().bpdc_plan_set_dc_stats(self.handle, None, 0))
            self._dc_stats = None
            return
        assert stats.is_cuda and stats.dtype.itemsize == 8 and stats.is_contiguous()
        self._dc_stats = stats  # keep it alive while the plan writes to it
        _check(lib().bpdc_plan_set_dc_stats(self.handle, _ptr(stats), stats.numel()))

    def workspace_size(self, code: int, B: int) -> int:
        n = C.c_size_t()
        _check(lib().bpdc_workspace_size(self.handle, code, B, C.byref(n)))
        return n.value

    def workspace(self, code: int, B: int):
        import torch
        need = max(256, self.workspace_size(code, B))
        ws = self._ws.get(code)
        if ws is None or ws.numel() < need:
            ws = torch.empty(need, dtype=torch.uint8, device="cuda")
            self._ws[code] = ws
        return ws

    def decode(self, syn, code: int = 0, shot_offset: int = 0, want_post: bool = False,
               want_cut: bool = False, want_iters: bool = False, out: Optional[dict] = None) -> dict:
        """Decode packed syndromes `syn` (int64 tensor [B, ceil(m/64)] on the GPU)."""
        import torch
        c = self.codes[code]
        B = syn.shape[0]
        nw = (c.n + 63) // 64
        assert syn.dtype == torch.int64 and syn.is_cuda and syn.shape[1] == (c.m + 63) // 64
        assert syn.is_contiguous()
        dev = syn.device
        if out is None:
            out = {"corr": torch.empty((B, nw), dtype=torch.int64, device=dev),
                   "flags": torch.empty(B, dtype=torch.uint8, device=dev)}
            if want_post:
                out["post"] = torch.empty((B, c.n), dtype=torch.float32, device=dev)
            if want_cut:
                out["cut"] = torch.empty((B, nw), dtype=torch.int64, device=dev)
            if want_iters:
                out["iters"] = torch.empty((B, 2), dtype=torch.int16, device=dev)
        ws = self.workspace(code, B)
        _check(lib().bpdc_decode(self.handle, code, _ptr(syn), B, shot_offset, _ptr(out["corr"]),
                                 _ptr(out["flags"]), _ptr(out.get("post")), _ptr(out.get("cut")),
                                 _ptr(out.get("iters")), _ptr(ws), ws.numel(), _stream()))
        return out

    def decode_noalloc(self, syn, code: int = 0, shot_offset: int = 0, want_post: bool = False,
                       want_cut: bool = False, want_iters: bool = False, out: Optional[dict] = None) -> dict:
        """decode() through bpdc_decode_noalloc: no workspace, the library's static scratch.
        With `out` given (all buffers preallocated) the call allocates nothing."""
        import torch
        c = self.codes[code]
        B = syn.shape[0]
        nw = (c.n + 63) // 64
        assert syn.dtype == torch.int64 and syn.is_cuda and syn.shape[1] == (c.m + 63) // 64
        assert syn.is_contiguous()
        if out is None:
            dev = syn.device
            out = {"corr": torch.empty((B, nw), dtype=torch.int64, device=dev),
                   "flags": torch.empty(B, dtype=torch.uint8, device=dev)}
            if want_post:
                out["post"] = torch.empty((B, c.n), dtype=torch.float32, device=dev)
            if want_cut:
                out["cut"] = torch.empty((B, nw), dtype=torch.int64, device=dev)
            if want_iters:
                out["iters"] = torch.empty((B, 2), dtype=torch.int16, device=dev)
        _check(lib().bpdc_decode_noalloc(self.handle, code, _ptr(syn), B, shot_offset, _ptr(out["corr"]),
                                         _ptr(out["flags"]), _ptr(out.get("post")), _ptr(out.get("cut")),
                                         _ptr(out.get("iters")), _stream()))
        return out

    # ---- multi-code batch -------------------------------------------------------------
    def multi_buffers(self, code_of_shot, B=None):
        """Offsets for a mixed batch: returns (syn_off, corr_off, syn_words, corr_words) as int64
        tensors/ints, packing each shot's words consecutively in batch order."""
        import torch
        cos = code_of_shot.cpu().numpy().astype(np.int64)
        sw = np.array([(c.m + 63) // 64 for c in self.codes], np.int64)[cos]
        nw = np.array([(c.n + 63) // 64 for c in self.codes], np.int64)[cos]
        syn_off = np.concatenate([[0], np.cumsum(sw)[:-1]]) if len(cos) else np.zeros(0, np.int64)
        corr_off = np.concatenate([[0], np.cumsum(nw)[:-1]]) if len(cos) else np.zeros(0, np.int64)
        return (torch.from_numpy(syn_off).cuda(), torch.from_numpy(corr_off).cuda(),
                int(sw.sum()), int(nw.sum()))

    def multi_workspace(self, B: int):
        import torch
        n = C.c_size_t()
        _check(lib().bpdc_workspace_size(self.handle, -1, B, C.byref(n)))
        ws = self._ws.get(-1)
        if ws is None or ws.numel() < n.value:
            ws = torch.empty(max(256, n.value), dtype=torch.uint8, device="cuda")
            self._ws[-1] = ws
        return ws

    def decode_multi(self, code_of_shot, syn, syn_off, corr, corr_off, flags, iters=None,
                     shot_offset: int = 0):
        """One persistent launch over a mixed batch (all tensors on the GPU)."""
        B = code_of_shot.shape[0]
        ws = self.multi_workspace(B)
        _check(lib().bpdc_decode_multi(self.handle, _ptr(code_of_shot), _ptr(syn), _ptr(syn_off), _ptr(corr),
                                       _ptr(corr_off), _ptr(flags), _ptr(iters), B, shot_offset, _ptr(ws),
                                       ws.numel(), _stream()))

    def capture_multi(self, code_of_shot, syn, syn_off, corr, corr_off, flags, iters=None,
                      shot_offset: int = 0):
        """Capture decode_multi on these buffers into a HIP graph held by the plan."""
        B = code_of_shot.shape[0]
        ws = self.multi_workspace(B)
        self._graph_keep = (code_of_shot, syn, syn_off, corr, corr_off, flags, iters, ws)
        _check(lib().bpdc_graph_capture_multi(self.handle, _ptr(code_of_shot), _ptr(syn), _ptr(syn_off),
                                              _ptr(corr), _ptr(corr_off), _ptr(flags), _ptr(iters), B,
                                              shot_offset, _ptr(ws), ws.numel(), _stream()))

    def graph_launch(self):
        _check(lib().bpdc_graph_launch(self.handle, _stream()))

    # ---- weighted min-sum ----------------------------------------------------------------
    def wms_ckpt_size(self, code: int, B: int, ckpt_every: int) -> int:
        n = C.c_size_t()
        _check(lib().bpdc_wms_ckpt_size(self.handle, code, B, ckpt_every, C.byref(n)))
        return n.value

    def wms_forward(self, w, syn, code: int = 0, shot_offset: int = 0, ckpt_every: int = 1):
        """Weighted forward: returns dict(post [2,B,n], cut [B,nw], flags [B], ckpt)."""
        import torch
        c = self.codes[code]
        B = syn.shape[0]
        nw = (c.n + 63) // 64
        post = torch.empty((2, B, c.n), dtype=torch.float32, device="cuda")
        cut = torch.empty((B, nw), dtype=torch.int64, device="cuda")
        flags = torch.empty(B, dtype=torch.uint8, device="cuda")
        ck = torch.empty(max(4, self.wms_ckpt_size(code, B, ckpt_every)), dtype=torch.uint8, device="cuda")
        assert w.dtype == torch.float32 and w.is_contiguous() and w.numel() == 2 * c.edges
        _check(lib().bpdc_wms_forward(self.handle, code, _ptr(w), _ptr(syn), B, shot_offset, ckpt_every,
                                      _ptr(post), _ptr(cut), _ptr(flags), _ptr(ck), ck.numel(), _stream()))
        return {"post": post, "cut": cut, "flags": flags, "ckpt": ck, "ckpt_every": ckpt_every}

    def wms_backward(self, w, syn, fwd: dict, grad_post, code: int = 0):
        """Adjoint of wms_forward: dLoss/dw [2, E] for dLoss/dpost [2, B, n]."""
        import torch
        c = self.codes[code]
        B = syn.shape[0]
        gw = torch.zeros(2 * c.edges, dtype=torch.float32, device="cuda")
        gp = grad_post.contiguous().float()
        _check(lib().bpdc_wms_backward(self.handle, code, _ptr(w), _ptr(syn), B, fwd["ckpt_every"], _ptr(gp),
                                       _ptr(fwd["cut"]), _ptr(fwd["flags"]), _ptr(fwd["ckpt"]),
                                       fwd["ckpt"].numel(), _ptr(gw), _stream()))
        return gw

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib().bpdc_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def eval_phi(x):
    """The library's float32 phi(x) = -ln tanh(x/2) (product-sum) on a float32 CUDA tensor."""
    import torch
    assert x.dtype == torch.float32 and x.is_cuda and x.is_contiguous()
    out = torch.empty_like(x)
    _check(lib().bpdc_eval_phi(_ptr(x), x.numel(), _ptr(out), _stream()))
    return out


def weighted_bpdc(plan: "Plan", code: int = 0, ckpt_every: int = 1):
    """torch.autograd.Function over the weighted min-sum BP+DC decoder.

    Returns a callable f(w, syn) -> (post [2, B, n], cut, flags): w is the
    [2 * E] float32 weight tensor (pass 1, pass 2), syn the packed syndromes.
    The backward runs the library's adjoint kernel with the cut held fixed.
    """
    import torch

    class _WeightedBPDC(torch.autograd.Function):
        @staticmethod
        def forward(ctx, w, syn):
            out = plan.wms_forward(w.detach().contiguous(), syn, code=code, ckpt_every=ckpt_every)
            ctx.save_for_backward(w, syn)
            ctx.fwd = out
            ctx.mark_non_differentiable(out["cut"], out["flags"])
            return out["post"], out["cut"], out["flags"]

        @staticmethod
        def backward(ctx, g_post, g_cut, g_flags):
            w, syn = ctx.saved_tensors
            if g_post is None:
                return None, None
            gw = plan.wms_backward(w.detach().contiguous(), syn, ctx.fwd, g_post, code=code)
            return gw, None

    return _WeightedBPDC.apply
