"""Thin ctypes binding of libcssar.so (include/cssar.h).

Argument marshalling only: every step of G, G^H and the iterative
thresholding runs in the library's HIP kernels.  Torch supplies device
memory (complex64 CUDA/HIP tensors) and the current stream.  The library
must have been built (``__graft_entry__.build()`` or
``python paper_1302_3120_amd/build.py``); there is no fallback path.
"""

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcssar.so")

OK, EINVAL, EUNSUPPORTED, EHIP, ENONFINITE, ENOMEM = 0, -1, -2, -3, -4, -5
_ERRORS = {EINVAL: "EINVAL", EUNSUPPORTED: "EUNSUPPORTED", EHIP: "EHIP",
           ENONFINITE: "ENONFINITE", ENOMEM: "ENOMEM"}

SYMBOLS = (
    "cssar_make_operator", "cssar_destroy_operator", "cssar_workspace_size",
    "cssar_apply_G", "cssar_apply_GH", "cssar_pack_mask", "cssar_ita_solve",
    "cssar_sync_status", "cssar_last_error", "cssar_supported_length",
    "cssar_plan_info", "cssar_profile_enable", "cssar_profile_read",
    "cssar_make_batch", "cssar_destroy_batch", "cssar_batch_workspace_size",
    "cssar_batch_set_graph", "cssar_batch_autotune", "cssar_batch_describe",
    "cssar_ita_solve_batched", "cssar_checkpoint_size", "cssar_grad_workspace_size",
    "cssar_ita_forward", "cssar_ita_backward", "cssar_ita_solve_adaptive",
    "cssar_make_operator_rda", "cssar_operator_chain", "cssar_ita_solve_safeguarded",
    "cssar_azimuth_fm_rate", "cssar_params_with_rates", "cssar_batch_sync_status",
    "cssar_ita_solve_ex",
)

PROFILE_KINDS = ("row_M", "row_G", "col_fwd", "col_inv", "col_update_threshold",
                 "col_residual", "col_threshold_adjoint", "col_data_adjoint",
                 "col_iterate_adjoint", "col_restricted_step", "col_step_norm",
                 "col_value", "col_threshold_selected", "row_adjoint_M", "row_adjoint_G",
                 "select_kth", "col_update_sparse")
NK = len(PROFILE_KINDS)


class CssarError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_ERRORS.get(code, code)}: {msg}")
        self.code = code


class SolveOpts(ctypes.Structure):
    """cssar_solve_opts (device pointers; NULL = unused)."""
    _fields_ = [("x0", ctypes.c_void_p), ("resid_hist", ctypes.c_void_p),
                ("l1_hist", ctypes.c_void_p), ("nnz_hist", ctypes.c_void_p)]


class Params(ctypes.Structure):
    _fields_ = [("fc", ctypes.c_double), ("Kr", ctypes.c_double),
                ("Tp", ctypes.c_double), ("fs", ctypes.c_double),
                ("prf", ctypes.c_double), ("v", ctypes.c_double),
                ("r_ref", ctypes.c_double), ("ba", ctypes.c_double),
                ("f_dc", ctypes.c_double), ("src", ctypes.c_int)]

    @classmethod
    def from_dict(cls, d):
        return cls(float(d["fc"]), float(d["Kr"]), float(d.get("Tp", 0.0)),
                   float(d["fs"]), float(d["prf"]), float(d["v"]),
                   float(d["r_ref"]), float(d.get("ba", 0.0)),
                   float(d.get("f_dc", 0.0)), int(d.get("src", 1)))


_lib = None


def lib():
    """Load libcssar.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, i, f = ctypes.c_void_p, ctypes.c_int, ctypes.c_float
        L.cssar_make_operator.argtypes = [ctypes.POINTER(Params), i, i, ctypes.POINTER(vp)]
        L.cssar_azimuth_fm_rate.argtypes = [ctypes.POINTER(Params)]
        L.cssar_azimuth_fm_rate.restype = ctypes.c_double
        L.cssar_params_with_rates.argtypes = [ctypes.POINTER(Params), ctypes.c_double, ctypes.c_double,
                                              ctypes.POINTER(Params)]
        L.cssar_params_with_rates.restype = ctypes.c_int
        L.cssar_make_operator_rda.argtypes = [ctypes.POINTER(Params), i, i, i, ctypes.POINTER(vp)]
        L.cssar_make_operator_rda.restype = ctypes.c_int
        L.cssar_operator_chain.argtypes = [vp]
        L.cssar_operator_chain.restype = ctypes.c_int
        L.cssar_destroy_operator.argtypes = [vp]
        L.cssar_workspace_size.argtypes = [vp, i]
        L.cssar_workspace_size.restype = ctypes.c_size_t
        L.cssar_apply_G.argtypes = [vp, vp, vp, vp, vp]
        L.cssar_apply_GH.argtypes = [vp, vp, vp, vp, vp]
        L.cssar_pack_mask.argtypes = [vp, vp, vp, vp]
        L.cssar_ita_solve.argtypes = [vp, vp, vp, f, i, vp, vp, vp, vp]
        L.cssar_ita_solve_ex.argtypes = [vp, vp, vp, f, i, ctypes.POINTER(SolveOpts), vp, vp, vp]
        L.cssar_sync_status.argtypes = [vp, vp]
        L.cssar_last_error.restype = ctypes.c_char_p
        L.cssar_supported_length.argtypes = [i]
        L.cssar_plan_info.argtypes = [i, ctypes.POINTER(i), ctypes.POINTER(i),
                                      ctypes.POINTER(i * 8)]
        L.cssar_profile_enable.argtypes = [vp, i]
        L.cssar_profile_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double * NK),
                                         ctypes.POINTER(ctypes.c_long * NK)]
        pp = ctypes.POINTER(vp)
        L.cssar_make_batch.argtypes = [pp, i, pp]
        L.cssar_destroy_batch.argtypes = [vp]
        L.cssar_batch_workspace_size.argtypes = [vp]
        L.cssar_batch_workspace_size.restype = ctypes.c_size_t
        L.cssar_batch_set_graph.argtypes = [vp, i]
        L.cssar_batch_autotune.argtypes = [vp, vp, ctypes.c_char_p, vp]
        L.cssar_batch_describe.argtypes = [vp, ctypes.c_char_p, i]
        L.cssar_ita_solve_batched.argtypes = [vp, pp, pp, ctypes.POINTER(f), i, pp, vp, vp]
        L.cssar_batch_sync_status.argtypes = [vp, vp, ctypes.POINTER(i)]
        L.cssar_checkpoint_size.argtypes = [vp, i, i]
        L.cssar_checkpoint_size.restype = ctypes.c_size_t
        L.cssar_grad_workspace_size.argtypes = [vp, i]
        L.cssar_grad_workspace_size.restype = ctypes.c_size_t
        L.cssar_ita_forward.argtypes = [vp, vp, vp, f, i, i, vp, vp, vp, vp]
        L.cssar_ita_backward.argtypes = [vp, vp, vp, f, i, i, vp, vp, vp, vp, vp, vp]
        L.cssar_ita_solve_adaptive.argtypes = [vp, vp, vp, ctypes.c_long, i, vp, vp, vp, vp, vp, vp]
        L.cssar_ita_solve_adaptive.restype = ctypes.c_int
        L.cssar_ita_solve_safeguarded.argtypes = [vp, vp, vp, ctypes.c_long, i, ctypes.c_double,
                                                  ctypes.c_double, i, vp, vp, vp, vp, vp, vp, vp]
        L.cssar_ita_solve_safeguarded.restype = ctypes.c_int
        L.cssar_ita_forward.restype = ctypes.c_int
        L.cssar_ita_backward.restype = ctypes.c_int
        for name in ("cssar_make_operator", "cssar_destroy_operator", "cssar_apply_G",
                     "cssar_apply_GH", "cssar_pack_mask", "cssar_ita_solve",
                     "cssar_sync_status", "cssar_supported_length", "cssar_plan_info",
                     "cssar_profile_enable", "cssar_profile_read", "cssar_make_batch",
                     "cssar_destroy_batch", "cssar_batch_set_graph", "cssar_batch_autotune",
                     "cssar_batch_describe", "cssar_ita_solve_batched", "cssar_batch_sync_status",
                     "cssar_ita_solve_ex"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(rc):
    if rc != OK:
        raise CssarError(rc, lib().cssar_last_error().decode())
    return rc


def supported_length(n):
    return bool(lib().cssar_supported_length(int(n)))


def plan_info(n):
    """(elements per thread, radices) of the FFT plan of a length."""
    e, p = ctypes.c_int(), ctypes.c_int()
    r = (ctypes.c_int * 8)()
    _check(lib().cssar_plan_info(int(n), ctypes.byref(e), ctypes.byref(p), ctypes.byref(r)))
    return e.value, [r[i] for i in range(p.value)]


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


CHAINS = ("csa", "rda")


class Operator:
    """Approximated observation G and its adjoint G^H = M on an
    N_a x N_r grid (the handle of cssar_make_operator, or of
    cssar_make_operator_rda with chain="rda" and a truncated-sinc length taps)."""

    def __init__(self, params, shape, chain="csa", taps=8):
        if chain not in CHAINS:
            raise ValueError(f"chain must be one of {CHAINS}")
        self.shape = (int(shape[0]), int(shape[1]))
        self.params = dict(params)
        self.chain = chain
        self._p = Params.from_dict(params)
        h = ctypes.c_void_p()
        if chain == "csa":
            _check(lib().cssar_make_operator(ctypes.byref(self._p), self.shape[0],
                                             self.shape[1], ctypes.byref(h)))
        else:
            _check(lib().cssar_make_operator_rda(ctypes.byref(self._p), self.shape[0],
                                                 self.shape[1], int(taps), ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().cssar_destroy_operator(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def workspace_size(self, mode):
        return int(lib().cssar_workspace_size(self._h, int(mode)))

    def _arr(self, t, name):
        if not isinstance(t, torch.Tensor) or t.dtype != torch.complex64:
            raise TypeError(f"{name} must be a complex64 tensor")
        if not t.is_cuda:
            raise ValueError(f"{name} must be on the GPU")
        if tuple(t.shape) != self.shape or not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous with shape {self.shape}")
        return t

    def _ws(self, ws, mode, device):
        if ws is None:
            return self.workspace(mode, device)
        if ws.numel() * ws.element_size() < self.workspace_size(mode) or not ws.is_cuda:
            raise ValueError("workspace too small")
        return ws

    def apply_G(self, x, out=None, ws=None):
        """y = G x."""
        x = self._arr(x, "x")
        out = torch.empty_like(x) if out is None else self._arr(out, "out")
        ws = self._ws(ws, 0, x.device)
        _check(lib().cssar_apply_G(self._h, _ptr(x), _ptr(out), _ptr(ws), _stream()))
        return out

    def apply_GH(self, y, out=None, ws=None):
        """x = G^H y = M y (the focusing chain)."""
        y = self._arr(y, "y")
        out = torch.empty_like(y) if out is None else self._arr(out, "out")
        ws = self._ws(ws, 0, y.device)
        _check(lib().cssar_apply_GH(self._h, _ptr(y), _ptr(out), _ptr(ws), _stream()))
        return out

    def pack_mask(self, mask):
        """Pack a bool/uint8 N_a x N_r mask into the solver's bit layout."""
        if mask.dtype not in (torch.bool, torch.uint8) or not mask.is_cuda:
            raise TypeError("mask must be a bool or uint8 GPU tensor")
        if tuple(mask.shape) != self.shape or not mask.is_contiguous():
            raise ValueError(f"mask must be contiguous with shape {self.shape}")
        n = self.shape[0] * self.shape[1]
        bits = torch.empty((n + 31) // 32, dtype=torch.int32, device=mask.device)
        _check(lib().cssar_pack_mask(self._h, _ptr(mask), _ptr(bits), _stream()))
        return bits

    def workspace(self, mode, device=None):
        """A fresh workspace tensor for cssar_workspace_size(mode) bytes
        (torch's allocator returns 256-byte aligned blocks)."""
        nbytes = self.workspace_size(mode)
        return torch.empty(max(nbytes, 8), dtype=torch.uint8, device=device or "cuda")

    def ita_solve(self, y, mask_bits, lam, iters, out=None, ws=None, resid=False):
        """Iterative thresholding (eq. (th2d) / Algorithm 1), X^(0) = 0.
        Returns X^(iters), and the residual norms ||R^(t)||^2 if resid."""
        y = self._arr(y, "y")
        if mask_bits.dtype != torch.int32 or not mask_bits.is_cuda:
            raise TypeError("mask_bits must come from pack_mask")
        out = torch.empty_like(y) if out is None else self._arr(out, "out")
        ws = self._ws(ws, 1, y.device)
        hist = torch.empty(int(iters), dtype=torch.float32, device=y.device) if resid else None
        _check(lib().cssar_ita_solve(self._h, _ptr(y), _ptr(mask_bits), float(lam),
                                     int(iters), _ptr(out),
                                     _ptr(hist) if hist is not None else None,
                                     _ptr(ws), _stream()))
        return (out, hist) if resid else out

    def ita_solve_ex(self, y, mask_bits, lam, iters, x0=None, out=None, ws=None):
        """cssar_ita_solve_ex: iterative thresholding from X^(0) = x0 (None:
        0), returning (X^(iters), ||R^(t)||^2, ||X^(t+1)||_1, nonzero count
        of X^(t+1)), the last three as device tensors of iters entries."""
        y = self._arr(y, "y")
        if mask_bits.dtype != torch.int32 or not mask_bits.is_cuda:
            raise TypeError("mask_bits must come from pack_mask")
        out = torch.empty_like(y) if out is None else self._arr(out, "out")
        x0 = None if x0 is None else self._arr(x0, "x0")
        ws = self._ws(ws, 1, y.device)
        n = int(iters)
        hist = torch.empty(max(n, 1), dtype=torch.float32, device=y.device)
        l1 = torch.empty(max(n, 1), dtype=torch.float32, device=y.device)
        nnz = torch.empty(max(n, 1), dtype=torch.int32, device=y.device)
        o = SolveOpts(x0.data_ptr() if x0 is not None else None, hist.data_ptr(), l1.data_ptr(),
                      nnz.data_ptr())
        _check(lib().cssar_ita_solve_ex(self._h, _ptr(y), _ptr(mask_bits), float(lam), n,
                                        ctypes.byref(o), _ptr(out), _ptr(ws), _stream()))
        return out, hist[:n], l1[:n], nnz[:n]

    def ita_solve_adaptive(self, y, mask_bits, k, iters, out=None, ws=None):
        """Iterative thresholding with the step and threshold of Section IV.B
        set per iteration from the sparsity k (cssar_ita_solve_adaptive).
        Returns (X^(iters), mu_t, lambda_t, ||R^(t)||^2), the last three as
        float32 device tensors of iters entries."""
        y = self._arr(y, "y")
        if mask_bits.dtype != torch.int32 or not mask_bits.is_cuda:
            raise TypeError("mask_bits must come from pack_mask")
        out = torch.empty_like(y) if out is None else self._arr(out, "out")
        ws = self._ws(ws, 2, y.device)
        hists = [torch.empty(int(iters), dtype=torch.float32, device=y.device) for _ in range(3)]
        _check(lib().cssar_ita_solve_adaptive(self._h, _ptr(y), _ptr(mask_bits), int(k), int(iters),
                                              _ptr(out), *(_ptr(h) for h in hists), _ptr(ws),
                                              _stream()))
        return (out, *hists)

    def ita_solve_safeguarded(self, y, mask_bits, k, iters, c=0.01, kappa=2.0, max_shrinks=2,
                              out=None, ws=None):
        """ita_solve_adaptive with the support-change safeguard of the step
        (cssar_ita_solve_safeguarded).  Returns (X^(iters), mu_t, lambda_t,
        ||R^(t)||^2, shrinks_t), the last four as device tensors of iters
        entries (float32; int32 for the shrinks)."""
        y = self._arr(y, "y")
        if mask_bits.dtype != torch.int32 or not mask_bits.is_cuda:
            raise TypeError("mask_bits must come from pack_mask")
        out = torch.empty_like(y) if out is None else self._arr(out, "out")
        ws = self._ws(ws, 3, y.device)
        hists = [torch.empty(int(iters), dtype=torch.float32, device=y.device) for _ in range(3)]
        shrinks = torch.empty(int(iters), dtype=torch.int32, device=y.device)
        _check(lib().cssar_ita_solve_safeguarded(self._h, _ptr(y), _ptr(mask_bits), int(k), int(iters),
                                                 float(c), float(kappa), int(max_shrinks), _ptr(out),
                                                 *(_ptr(h) for h in hists), _ptr(shrinks), _ptr(ws),
                                                 _stream()))
        return (out, *hists, shrinks)

    def ita_forward(self, y, mask_bits, lam, iters, every, out=None):
        """cssar_ita_forward: X^(iters) and the checkpoint buffer for the
        reverse pass."""
        y = self._arr(y, "y")
        if mask_bits.dtype != torch.int32 or not mask_bits.is_cuda:
            raise TypeError("mask_bits must come from pack_mask")
        out = torch.empty_like(y) if out is None else self._arr(out, "out")
        nck = int(lib().cssar_checkpoint_size(self._h, int(iters), int(every)))
        ckpt = torch.empty(max(nck, 8), dtype=torch.uint8, device=y.device)
        ws = self.workspace(1, y.device)
        _check(lib().cssar_ita_forward(self._h, _ptr(y), _ptr(mask_bits), float(lam), int(iters),
                                       int(every), _ptr(out), _ptr(ckpt) if nck else None,
                                       _ptr(ws), _stream()))
        return out, ckpt

    def ita_backward(self, y, mask_bits, lam, iters, every, ckpt, grad_x):
        """cssar_ita_backward: (dL/dy, tensor([dL/dlambda, dL/dK_a, dL/dK_r]))
        given dL/dX^(iters)."""
        y = self._arr(y, "y")
        grad_x = self._arr(grad_x.contiguous(), "grad_x")
        gy = torch.empty_like(y)
        gs = torch.empty(3, dtype=torch.float64, device=y.device)
        nws = int(lib().cssar_grad_workspace_size(self._h, int(every)))
        ws = torch.empty(max(nws, 8), dtype=torch.uint8, device=y.device)
        _check(lib().cssar_ita_backward(self._h, _ptr(y), _ptr(mask_bits), float(lam), int(iters),
                                        int(every), _ptr(ckpt), _ptr(grad_x), _ptr(gy),
                                        ctypes.c_void_p(gs.data_ptr()), _ptr(ws), _stream()))
        return gy, gs

    def sync_status(self):
        _check(lib().cssar_sync_status(self._h, _stream()))

    def profile(self, on):
        """Enable/disable per-launch HIP event timing of the pass kernels."""
        _check(lib().cssar_profile_enable(self._h, 1 if on else 0))

    def profile_read(self):
        """{kind: (total ms, launches)} since the last read (waits for the events)."""
        ms = (ctypes.c_double * NK)()
        cnt = (ctypes.c_long * NK)()
        _check(lib().cssar_profile_read(self._h, ctypes.byref(ms), ctypes.byref(cnt)))
        return {PROFILE_KINDS[k]: (ms[k], cnt[k]) for k in range(NK) if cnt[k]}


def make_operator(params, shape, chain="csa", taps=8):
    return Operator(params, shape, chain, taps)


def _ptrs(ts):
    return (ctypes.c_void_p * len(ts))(*[t.data_ptr() for t in ts])


class Batch:
    """Many scenes solved together (cssar_make_batch): grouped pass kernels
    per line length, optional HIP-graph replay, measuring autotuner.  Keeps
    references to its operators (they must outlive it)."""

    def __init__(self, ops):
        self.ops = list(ops)
        if not self.ops:
            raise ValueError("need at least one operator")
        arr = (ctypes.c_void_p * len(self.ops))(*[op.handle.value for op in self.ops])
        h = ctypes.c_void_p()
        _check(lib().cssar_make_batch(arr, len(self.ops), ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().cssar_destroy_batch(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace_size(self):
        return int(lib().cssar_batch_workspace_size(self._h))

    def workspace(self, device=None):
        return torch.empty(max(self.workspace_size(), 8), dtype=torch.uint8,
                           device=device or "cuda")

    def set_graph(self, on):
        _check(lib().cssar_batch_set_graph(self._h, 1 if on else 0))

    def autotune(self, ws=None, cache_path=None):
        ws = self.workspace() if ws is None else ws
        if ws.numel() * ws.element_size() < self.workspace_size() or not ws.is_cuda:
            raise ValueError("workspace too small")
        cp = cache_path.encode() if cache_path else None
        _check(lib().cssar_batch_autotune(self._h, _ptr(ws), cp, _stream()))

    def describe(self):
        n = lib().cssar_batch_describe(self._h, None, 0)
        buf = ctypes.create_string_buffer(max(n, 0) + 1)
        lib().cssar_batch_describe(self._h, buf, len(buf))
        return buf.value.decode()

    def sync_status(self):
        """Wait for the stream; raise CssarError (CSSAR_ENONFINITE, naming the
        first scene) if a call left NaN or Inf in some X^(iters)."""
        sc = ctypes.c_int(-1)
        _check(lib().cssar_batch_sync_status(self._h, _stream(), ctypes.byref(sc)))

    def ita_solve(self, ys, mask_bits, lams, iters, outs=None, ws=None):
        """Iterative thresholding of every scene; returns the list of X^(iters)."""
        if not (len(ys) == len(mask_bits) == len(lams) == len(self.ops)):
            raise ValueError("one y, mask and lambda per scene")
        ys = [op._arr(y, "y") for op, y in zip(self.ops, ys)]
        for m in mask_bits:
            if m.dtype != torch.int32 or not m.is_cuda:
                raise TypeError("mask_bits must come from pack_mask")
        outs = [torch.empty_like(y) for y in ys] if outs is None else \
            [op._arr(o, "out") for op, o in zip(self.ops, outs)]
        if ws is None:
            ws = self.workspace(ys[0].device)
        elif ws.numel() * ws.element_size() < self.workspace_size() or not ws.is_cuda:
            raise ValueError("workspace too small")
        lam = (ctypes.c_float * len(lams))(*[float(v) for v in lams])
        _check(lib().cssar_ita_solve_batched(self._h, _ptrs(ys), _ptrs(mask_bits), lam,
                                             int(iters), _ptrs(outs), _ptr(ws), _stream()))
        return outs


def make_batch(ops):
    return Batch(ops)


_PARAM_KEYS = ("fc", "Kr", "Tp", "fs", "prf", "v", "r_ref", "ba", "f_dc", "src")


def ka_of(params):
    """Azimuth FM rate at the reference range (cssar_azimuth_fm_rate)."""
    p = Params.from_dict(params)
    return float(lib().cssar_azimuth_fm_rate(ctypes.byref(p)))


def params_with_theta(params, Ka, Kr):
    """params with the azimuth FM rate Ka and the range chirp rate Kr
    (cssar_params_with_rates)."""
    src = Params.from_dict(params)
    out = Params()
    _check(lib().cssar_params_with_rates(ctypes.byref(src), float(Ka), float(Kr), ctypes.byref(out)))
    p = dict(params)
    p.update({k: getattr(out, k) for k in _PARAM_KEYS})
    return p


# The operator of the last ITAUnrolled call, reused while the parameters,
# rates, shape and device stay the same.
_unrolled_op = {"key": None, "op": None}


def _unrolled_operator(params, Ka, Kr, shape, device):
    key = (tuple(sorted((k, float(v)) for k, v in params.items() if k in _PARAM_KEYS)),
           float(Ka), float(Kr), tuple(shape), str(device))
    if _unrolled_op["key"] != key:
        _unrolled_op["op"] = Operator(params_with_theta(params, float(Ka), float(Kr)), tuple(shape))
        _unrolled_op["key"] = key
    return _unrolled_op["op"]


class ITAUnrolled(torch.autograd.Function):
    """X^(K) of K unrolled iterations as a differentiable function of the
    raw data y (complex64), lambda, K_a and K_r (0-dim float64 tensors).
    Forward: cssar_ita_forward with a checkpoint every ``every`` iterations;
    backward: cssar_ita_backward.  The operator is built from (K_a, K_r) and
    reused while they (and the other parameters) do not change."""

    @staticmethod
    def forward(ctx, y, lam, Ka, Kr, mask, iters, every, params):
        op = _unrolled_operator(params, Ka, Kr, y.shape, y.device)
        bits = op.pack_mask(mask)
        x, ckpt = op.ita_forward(y.contiguous(), bits, float(lam), int(iters), int(every))
        ctx.op, ctx.bits, ctx.ckpt = op, bits, ckpt
        ctx.args = (float(lam), int(iters), int(every))
        ctx.meta = [(t.device, t.dtype) if isinstance(t, torch.Tensor) else None for t in (lam, Ka, Kr)]
        ctx.save_for_backward(y)
        return x

    @staticmethod
    def backward(ctx, gx):
        (y,) = ctx.saved_tensors
        lam, iters, every = ctx.args
        gy, gs = ctx.op.ita_backward(y.contiguous(), ctx.bits, lam, iters, every, ctx.ckpt, gx)
        scal = [gs[i].to(device=m[0], dtype=m[1]) if m is not None else None
                for i, m in enumerate(ctx.meta)]
        return (gy, *scal, None, None, None, None)
