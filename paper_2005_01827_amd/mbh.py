"""Thin Python binding of libmbh (include/mbh.h).

Argument marshalling only: every step of the likelihood runs in the HIP
kernels of ``libmbh.so``.  PyTorch provides device memory and the stream.
There is no CPU fallback; if the library or a GPU is missing, the calls raise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmbh.so")

MBH_OK, MBH_EINVAL, MBH_ENOMEM, MBH_EHIP, MBH_EBATCH = 0, -1, -2, -3, -4
MBH_FP64, MBH_FP32C = 0, 1
STATUS_NAMES = {0: "MBH_OK", -1: "MBH_EINVAL", -2: "MBH_ENOMEM", -3: "MBH_EHIP", -4: "MBH_EBATCH"}

# Every entry point declared in include/mbh.h.
EXPORTED = ("mbh_ctx_create", "mbh_ctx_destroy", "mbh_last_error", "mbh_waveform_gen", "mbh_response",
            "mbh_interp_and_inner", "mbh_loglike_batch", "mbh_loglike_batch_noalloc", "mbh_template", "mbh_get_sparse", "mbh_set_sparse",
            "mbh_set_timing", "mbh_get_timing", "mbh_set_schedule", "mbh_get_schedule", "mbh_autotune",
            "mbh_flow_create", "mbh_flow_destroy", "mbh_flow_last_error",
            "mbh_flow_num_params", "mbh_flow_get_layout", "mbh_flow_get_params", "mbh_flow_set_params",
            "mbh_flow_forward", "mbh_flow_inverse", "mbh_flow_loss_grad", "mbh_flow_adam", "mbh_version")


class MbhError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class CtxDesc(ctypes.Structure):
    _fields_ = [("df", ctypes.c_double), ("k0", ctypes.c_int64), ("n", ctypes.c_int64),
                ("data", ctypes.POINTER(ctypes.c_double)), ("psd", ctypes.POINTER(ctypes.c_double)),
                ("n_modes", ctypes.c_int), ("modes", (ctypes.c_int * 2) * 6), ("n_sparse", ctypes.c_int),
                ("t0", ctypes.c_double), ("precision", ctypes.c_int), ("max_batch", ctypes.c_int)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libmbh.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libmbh.so not found at {path}: build it with paper_2005_01827_amd/build.py")
    L = ctypes.CDLL(path)
    vp, dp, i64p = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)
    L.mbh_ctx_create.argtypes = [ctypes.POINTER(CtxDesc), ctypes.POINTER(vp)]
    L.mbh_ctx_create.restype = ctypes.c_int
    L.mbh_ctx_destroy.argtypes = [vp]
    L.mbh_ctx_destroy.restype = None
    L.mbh_last_error.argtypes = [vp]
    L.mbh_last_error.restype = ctypes.c_char_p
    L.mbh_waveform_gen.argtypes = [vp, vp, ctypes.c_int, vp]
    L.mbh_response.argtypes = [vp, ctypes.c_int, vp]
    L.mbh_interp_and_inner.argtypes = [vp, ctypes.c_int, vp, vp]
    L.mbh_loglike_batch.argtypes = [vp, vp, ctypes.c_int, vp, vp]
    L.mbh_loglike_batch_noalloc.argtypes = [vp, vp, ctypes.c_int, vp, vp]
    L.mbh_template.argtypes = [vp, vp, vp, vp]
    L.mbh_get_sparse.argtypes = [vp, ctypes.c_int, i64p, dp, dp, dp, dp, vp]
    L.mbh_set_sparse.argtypes = [vp, ctypes.c_int, i64p, dp, dp, dp, vp]
    for name in ("mbh_waveform_gen", "mbh_response", "mbh_interp_and_inner", "mbh_loglike_batch",
                 "mbh_loglike_batch_noalloc", "mbh_template",
                 "mbh_get_sparse", "mbh_set_sparse"):
        getattr(L, name).restype = ctypes.c_int
    L.mbh_set_timing.argtypes = [vp, ctypes.c_int]
    L.mbh_set_timing.restype = ctypes.c_int
    L.mbh_get_timing.argtypes = [vp, dp, i64p]
    L.mbh_get_timing.restype = ctypes.c_int
    ip, fp = ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_float)
    L.mbh_set_schedule.argtypes = [vp, ctypes.c_int, ctypes.c_int]
    L.mbh_get_schedule.argtypes = [vp, ip, ip]
    L.mbh_autotune.argtypes = [vp, vp, ctypes.c_int, ctypes.c_int, ip, dp, vp]
    for name in ("mbh_set_schedule", "mbh_get_schedule", "mbh_autotune"):
        getattr(L, name).restype = ctypes.c_int
    L.mbh_flow_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ip, ctypes.c_uint64,
                                  ctypes.POINTER(vp)]
    L.mbh_flow_destroy.argtypes = [vp]
    L.mbh_flow_destroy.restype = None
    L.mbh_flow_last_error.argtypes = [vp]
    L.mbh_flow_last_error.restype = ctypes.c_char_p
    L.mbh_flow_num_params.argtypes = [vp]
    L.mbh_flow_num_params.restype = ctypes.c_int64
    L.mbh_flow_get_layout.argtypes = [vp, ip, ip]
    L.mbh_flow_get_params.argtypes = [vp, fp]
    L.mbh_flow_set_params.argtypes = [vp, fp]
    L.mbh_flow_forward.argtypes = [vp, vp, ctypes.c_int, vp, vp, vp]
    L.mbh_flow_inverse.argtypes = [vp, vp, ctypes.c_int, vp, vp, vp]
    L.mbh_flow_loss_grad.argtypes = [vp, vp, ctypes.c_int, dp, fp, vp]
    L.mbh_flow_adam.argtypes = [vp, ctypes.c_float, vp]
    for name in ("mbh_flow_create", "mbh_flow_get_layout", "mbh_flow_get_params", "mbh_flow_set_params",
                 "mbh_flow_forward", "mbh_flow_inverse", "mbh_flow_loss_grad", "mbh_flow_adam"):
        getattr(L, name).restype = ctypes.c_int
    L.mbh_version.restype = ctypes.c_int
    _lib = L
    return L


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("libmbh needs a ROCm GPU: torch.cuda.is_available() is False")
    return torch


def _ptr(a):
    return ctypes.cast(a.ctypes.data, ctypes.POINTER(ctypes.c_double)) if a is not None else None


class Likelihood:
    """A libmbh context: data and PSD resident on the GPU, batched ln L.

    data: complex [3][n] (A, E, T) on the grid f_k = k df, k = k0..k0+n-1;
    psd: [3][n] one-sided PSD.  Parameters are physical (see include/mbh.h).
    """

    def __init__(self, grid, data, psd, modes, n_sparse=256, t0=0.0, precision=MBH_FP64, max_batch=1024):
        self._torch = _torch()
        self.lib = load_library()
        self.grid = grid
        self.modes = tuple(tuple(m) for m in modes)
        self.n_sparse = n_sparse
        self.max_batch = max_batch
        self.precision = precision
        d = np.ascontiguousarray(np.stack([np.asarray(data).real, np.asarray(data).imag], axis=-1), dtype=np.float64)
        S = np.ascontiguousarray(psd, dtype=np.float64)
        if d.shape != (3, grid.n, 2) or S.shape != (3, grid.n):
            raise ValueError("data must be [3][n] complex and psd [3][n]")
        desc = CtxDesc()
        desc.df, desc.k0, desc.n = grid.df, grid.k0, grid.n
        desc.data, desc.psd = _ptr(d), _ptr(S)
        desc.n_modes = len(self.modes)
        for i, (l, m) in enumerate(self.modes):
            desc.modes[i][0], desc.modes[i][1] = l, m
        desc.n_sparse, desc.t0, desc.precision, desc.max_batch = n_sparse, t0, precision, max_batch
        self._torch.cuda.init()
        h = ctypes.c_void_p()
        st = self.lib.mbh_ctx_create(ctypes.byref(desc), ctypes.byref(h))
        if st != MBH_OK:
            raise MbhError(st, "mbh_ctx_create rejected the descriptor or failed to allocate")
        self.ctx = h

    # -- helpers --------------------------------------------------------
    def _check(self, st, what):
        if st != MBH_OK:
            msg = self.lib.mbh_last_error(self.ctx)
            raise MbhError(st, f"{what}: {msg.decode() if msg else ''}")

    def _stream(self, stream=None):
        s = stream if stream is not None else self._torch.cuda.current_stream()
        return ctypes.c_void_p(s.cuda_stream)

    def _params(self, params):
        t = self._torch
        p = params if isinstance(params, t.Tensor) else t.as_tensor(np.asarray(params, dtype=np.float64))
        p = p.to(device="cuda", dtype=t.float64).contiguous()
        if p.dim() == 1:
            p = p.unsqueeze(0)
        if p.dim() != 2 or p.shape[1] != 11:
            raise ValueError("params must be [B][11]")
        return p

    # -- entry points ----------------------------------------------------
    def waveform_gen(self, params, stream=None):
        p = self._params(params)
        self._check(self.lib.mbh_waveform_gen(self.ctx, ctypes.c_void_p(p.data_ptr()), p.shape[0],
                                              self._stream(stream)), "mbh_waveform_gen")
        self._keep = p
        return p.shape[0]

    def response(self, B, stream=None):
        self._check(self.lib.mbh_response(self.ctx, B, self._stream(stream)), "mbh_response")

    def interp_and_inner(self, B, out7=None, stream=None):
        t = self._torch
        if out7 is None:
            out7 = t.empty((B, 7), dtype=t.float64, device="cuda")
        self._check(self.lib.mbh_interp_and_inner(self.ctx, B, ctypes.c_void_p(out7.data_ptr()),
                                                  self._stream(stream)), "mbh_interp_and_inner")
        return out7

    def stages(self, params, stream=None):
        """waveform_gen -> response -> interp_and_inner; returns out7 [B][7] (device)."""
        B = self.waveform_gen(params, stream)
        self.response(B, stream)
        return self.interp_and_inner(B, stream=stream)

    def loglike(self, params, out=None, stream=None):
        """ln L [B] (device tensor) through the graph-launched entry point."""
        t = self._torch
        p = self._params(params)
        B = p.shape[0]
        if out is None:
            out = t.empty(B, dtype=t.float64, device="cuda")
        self._check(self.lib.mbh_loglike_batch(self.ctx, ctypes.c_void_p(p.data_ptr()), B,
                                               ctypes.c_void_p(out.data_ptr()), self._stream(stream)),
                    "mbh_loglike_batch")
        self._keep = p
        return out

    def loglike_noalloc(self, params, out, stream=None):
        """ln L [B] into the caller's device tensor 'out' through the entry
        point that allocates nothing (fixed per-GPU workspace); params must
        already be a contiguous float64 [B][11] device tensor."""
        t = self._torch
        if not (isinstance(params, t.Tensor) and params.is_cuda and params.dtype == t.float64 and
                params.dim() == 2 and params.shape[1] == 11 and params.is_contiguous()):
            raise ValueError("params must be a contiguous float64 [B][11] device tensor")
        B = params.shape[0]
        if not (isinstance(out, t.Tensor) and out.is_cuda and out.dtype == t.float64 and out.numel() >= B):
            raise ValueError("out must be a float64 device tensor of at least B entries")
        self._check(self.lib.mbh_loglike_batch_noalloc(self.ctx, ctypes.c_void_p(params.data_ptr()), B,
                                                       ctypes.c_void_p(out.data_ptr()), self._stream(stream)),
                    "mbh_loglike_batch_noalloc")
        return out

    def template(self, params, stream=None):
        """Dense template h[3][n] (complex128 device tensor) of one walker."""
        t = self._torch
        p = self._params(params)[:1].contiguous()
        h = t.empty((3, self.grid.n, 2), dtype=t.float64, device="cuda")
        self._check(self.lib.mbh_template(self.ctx, ctypes.c_void_p(p.data_ptr()), ctypes.c_void_p(h.data_ptr()),
                                          self._stream(stream)), "mbh_template")
        self._keep = p
        return t.view_as_complex(h)

    def get_sparse(self, w, stream=None):
        nm, ns = len(self.modes), self.n_sparse
        band = np.zeros((nm, 4), dtype=np.int64)
        fband = np.zeros((nm, 2))
        f = np.zeros((nm, ns))
        fn = np.zeros((nm, 8, ns))
        cf = np.zeros((nm, 8, ns - 1, 4))
        self._check(self.lib.mbh_get_sparse(self.ctx, w, band.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                            _ptr(fband), _ptr(f), _ptr(fn), _ptr(cf), self._stream(stream)),
                    "mbh_get_sparse")
        return dict(band=band, fband=fband, f=f, fn=fn, cf=cf)

    def set_sparse(self, band, fband, f, fn, stream=None):
        band = np.ascontiguousarray(band, dtype=np.int64)
        fband, f, fn = (np.ascontiguousarray(x, dtype=np.float64) for x in (fband, f, fn))
        B = band.shape[0]
        self._check(self.lib.mbh_set_sparse(self.ctx, B, band.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                            _ptr(fband), _ptr(f), _ptr(fn), self._stream(stream)), "mbh_set_sparse")
        return B

    def set_timing(self, on: bool):
        self._check(self.lib.mbh_set_timing(self.ctx, 1 if on else 0), "mbh_set_timing")

    def get_timing(self):
        """(summed dense-kernel milliseconds, number of timed launches)."""
        ms = ctypes.c_double()
        cnt = ctypes.c_int64()
        self._check(self.lib.mbh_get_timing(self.ctx, ctypes.byref(ms), ctypes.byref(cnt)), "mbh_get_timing")
        return ms.value, cnt.value

    def set_schedule(self, blocks_per_cu=8, one_per_walker=False):
        self._check(self.lib.mbh_set_schedule(self.ctx, int(blocks_per_cu), 1 if one_per_walker else 0),
                    "mbh_set_schedule")

    def get_schedule(self):
        b, o = ctypes.c_int(), ctypes.c_int()
        self._check(self.lib.mbh_get_schedule(self.ctx, ctypes.byref(b), ctypes.byref(o)), "mbh_get_schedule")
        return b.value, bool(o.value)

    def autotune(self, params, reps=5, cache=None, key=None, stream=None):
        """Pick the dense launch shape for this batch (see mbh_autotune).

        With a cache path, results are stored as JSON under 'key' (default:
        grid size, batch, modes, precision and the GPU name) and reused.
        Returns (blocks_per_cu, median dense ms or None if from the cache)."""
        import json
        t = self._torch
        p = self._params(params)
        if key is None:
            key = (f"{t.cuda.get_device_name()}|n={self.grid.n}|B={p.shape[0]}|modes={len(self.modes)}|"
                   f"ns={self.n_sparse}|prec={self.precision}")
        table = {}
        if cache and os.path.exists(cache):
            with open(cache) as fh:
                table = json.load(fh)
        if key in table:
            self.set_schedule(table[key]["blocks_per_cu"], False)
            return table[key]["blocks_per_cu"], None
        b, ms = ctypes.c_int(), ctypes.c_double()
        self._check(self.lib.mbh_autotune(self.ctx, ctypes.c_void_p(p.data_ptr()), p.shape[0], reps,
                                          ctypes.byref(b), ctypes.byref(ms), self._stream(stream)), "mbh_autotune")
        if cache:
            table[key] = {"blocks_per_cu": b.value, "dense_ms": ms.value}
            os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
            tmp = cache + ".tmp"
            with open(tmp, "w") as fh:
                json.dump(table, fh, indent=1, sort_keys=True)
            os.replace(tmp, cache)
        return b.value, ms.value

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.mbh_ctx_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Flow:
    """The affine-coupling flow of include/mbh.h (FP32, on the GPU).

    Rows are float32 [n][dim] torch CUDA tensors (numpy arrays are copied to
    the device).  perm: optional [L][dim] int permutations.
    """

    def __init__(self, dim, n_layers=8, hidden=128, max_batch=65536, perm=None, seed=0):
        self._torch = _torch()
        self.lib = load_library()
        self.dim, self.n_layers, self.hidden, self.max_batch = dim, n_layers, hidden, max_batch
        self._torch.cuda.init()
        pp = None
        if perm is not None:
            self._perm_in = np.ascontiguousarray(perm, dtype=np.int32)
            if self._perm_in.shape != (n_layers, dim):
                raise ValueError("perm must be [n_layers][dim]")
            pp = self._perm_in.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
        h = ctypes.c_void_p()
        st = self.lib.mbh_flow_create(dim, n_layers, hidden, max_batch, pp, seed, ctypes.byref(h))
        if st != MBH_OK:
            raise MbhError(st, "mbh_flow_create rejected the arguments or failed to allocate")
        self.flow = h
        self.n_params = int(self.lib.mbh_flow_num_params(h))

    def _check(self, st, what):
        if st != MBH_OK:
            msg = self.lib.mbh_flow_last_error(self.flow)
            raise MbhError(st, f"{what}: {msg.decode() if msg else ''}")

    def _stream(self, stream=None):
        s = stream if stream is not None else self._torch.cuda.current_stream()
        return ctypes.c_void_p(s.cuda_stream)

    def _rows(self, x):
        t = self._torch
        r = x if isinstance(x, t.Tensor) else t.as_tensor(np.asarray(x, dtype=np.float32))
        r = r.to(device="cuda", dtype=t.float32).contiguous()
        if r.dim() != 2 or r.shape[1] != self.dim:
            raise ValueError(f"rows must be [n][{self.dim}]")
        return r

    def layout(self):
        perm = np.zeros((self.n_layers, self.dim), dtype=np.int32)
        nc = np.zeros(self.n_layers, dtype=np.int32)
        ip = ctypes.POINTER(ctypes.c_int)
        self._check(self.lib.mbh_flow_get_layout(self.flow, perm.ctypes.data_as(ip), nc.ctypes.data_as(ip)),
                    "mbh_flow_get_layout")
        return perm, nc

    def get_params(self):
        p = np.empty(self.n_params, dtype=np.float32)
        self._check(self.lib.mbh_flow_get_params(self.flow, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float))),
                    "mbh_flow_get_params")
        return p

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        if p.shape != (self.n_params,):
            raise ValueError(f"expected {self.n_params} parameters")
        self._check(self.lib.mbh_flow_set_params(self.flow, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float))),
                    "mbh_flow_set_params")

    def _outs(self, n, out):
        if out is not None:
            a, lq = out
            if a.shape != (n, self.dim) or lq.shape != (n,) or not (a.is_contiguous() and lq.is_contiguous()):
                raise ValueError("out must be contiguous ([n][dim], [n]) float32 CUDA tensors")
            return a, lq
        t = self._torch
        return t.empty((n, self.dim), dtype=t.float32, device="cuda"), t.empty(n, dtype=t.float32, device="cuda")

    def forward(self, u, stream=None, out=None):
        """(z, log q(u)) as CUDA tensors (written into out=(z, lq) if given)."""
        u = self._rows(u)
        n = u.shape[0]
        z, lq = self._outs(n, out)
        self._check(self.lib.mbh_flow_forward(self.flow, ctypes.c_void_p(u.data_ptr()), n,
                                              ctypes.c_void_p(z.data_ptr()), ctypes.c_void_p(lq.data_ptr()),
                                              self._stream(stream)), "mbh_flow_forward")
        return z, lq

    def inverse(self, z, stream=None, out=None):
        """(u = f^-1(z), log q(u)) as CUDA tensors (written into out=(u, lq) if given)."""
        z = self._rows(z)
        n = z.shape[0]
        u, lq = self._outs(n, out)
        self._check(self.lib.mbh_flow_inverse(self.flow, ctypes.c_void_p(z.data_ptr()), n,
                                              ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(lq.data_ptr()),
                                              self._stream(stream)), "mbh_flow_inverse")
        return u, lq

    def loss_grad(self, u, want_grad=True, stream=None):
        """(loss, gradient as a float32 numpy array or None)."""
        u = self._rows(u)
        loss = ctypes.c_double()
        g = np.empty(self.n_params, dtype=np.float32) if want_grad else None
        gp = g.ctypes.data_as(ctypes.POINTER(ctypes.c_float)) if want_grad else None
        self._check(self.lib.mbh_flow_loss_grad(self.flow, ctypes.c_void_p(u.data_ptr()), u.shape[0],
                                                ctypes.byref(loss), gp, self._stream(stream)), "mbh_flow_loss_grad")
        return loss.value, g

    def adam(self, lr, stream=None):
        self._check(self.lib.mbh_flow_adam(self.flow, float(lr), self._stream(stream)), "mbh_flow_adam")

    def close(self):
        if getattr(self, "flow", None):
            self.lib.mbh_flow_destroy(self.flow)
            self.flow = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
