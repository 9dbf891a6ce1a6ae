"""MI355X widefield measurement operator: Phi, Phi^dag and Phi^dag Phi under hybrid
w-stacking / w-projection (Dabbech & Wiaux), behind the C ABI of include/wf.h.

This module only marshals arguments: every step of the operator runs in the HIP
library libwf.so.  Importing it fails loudly when the library has not been built.
Device buffers are torch tensors on the current HIP device; calls are asynchronous
on torch's current stream unless another stream is given.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import (WfImageShape, WfOptions, WfPlanInfo, WfTuneInfo, check, APPLY, OTF_FORM,
                   STORE, STRATEGY)

_lib.load()

__all__ = ["Operator", "Graph", "Network", "default_options", "briggs_weights", "plan"]


def default_options(**kw) -> WfOptions:
    o = WfOptions()
    _lib.load().wf_default_options(ctypes.byref(o))
    for k, v in kw.items():
        if k == "store":
            v = STORE[v] if isinstance(v, str) else int(v)
        elif k == "strategy":
            v = STRATEGY[v] if isinstance(v, str) else int(v)
        elif k == "otf_form":
            v = OTF_FORM[v] if isinstance(v, str) else int(v)
        elif k == "surrogate":
            v = None if v is None else (v._h.value if isinstance(v, Network) else int(v))
        elif k in ("weights", "flags"):
            raise TypeError(f"{k} is an argument of Operator, not an option")
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


def briggs_weights(uvw_m, freqs_hz, nx, ny, cell_rad, robust, chan_rows=None, natural=None,
                   flags=None, stream=None):
    """Briggs robust operator weights sqrt(w'_k) (include/wf.h, wf_briggs_weights),
    float32 [total rows], computed on the device."""
    lib = _lib.load()
    uvw = np.ascontiguousarray(uvw_m, dtype=np.float64)
    fr = np.ascontiguousarray(np.atleast_1d(freqs_hz), dtype=np.float64)
    cr = None if chan_rows is None else np.ascontiguousarray(chan_rows, dtype=np.int64)
    n = int(cr.sum()) if cr is not None else int(uvw.shape[0]) * int(fr.size)
    nat = None if natural is None else np.ascontiguousarray(natural, dtype=np.float32)
    fl = None if flags is None else np.ascontiguousarray(flags, dtype=np.uint8)
    for a, name in ((nat, "natural"), (fl, "flags")):
        if a is not None and a.shape != (n,):
            raise ValueError(f"{name} must have shape ({n},)")
    out = np.empty(n, dtype=np.float32)
    ptr = lambda a: None if a is None else a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
    check(lib.wf_briggs_weights(ptr(uvw), ctypes.c_int64(uvw.shape[0]), ptr(cr), ptr(fr),
                                ctypes.c_int32(fr.size), WfImageShape(int(nx), int(ny),
                                                                      float(cell_rad)),
                                float(robust), ptr(nat), ptr(fl), ptr(out),
                                _stream_handle(stream)), "wf_briggs_weights")
    return out


def plan(uvw_m, freq_hz, nx, ny, cell_rad, memory_budget=288e9, **opts):
    """The planner alone on the host (include/wf.h, wf_plan): (plan dict, centroids)."""
    lib = _lib.load()
    uvw = np.ascontiguousarray(uvw_m, dtype=np.float64)
    o = default_options(**opts)
    info = WfPlanInfo()
    cent = np.zeros(256, dtype=np.float64)
    check(lib.wf_plan(uvw.ctypes.data_as(ctypes.c_void_p), ctypes.c_int64(uvw.shape[0]),
                      float(freq_hz), WfImageShape(int(nx), int(ny), float(cell_rad)),
                      ctypes.c_uint64(int(memory_budget)), ctypes.byref(o), ctypes.byref(info),
                      cent.ctypes.data_as(ctypes.c_void_p), cent.size), "wf_plan")
    d = {k: getattr(info, k) for k, _ in WfPlanInfo._fields_}
    return d, cent[:d["nbins"]].copy()


def _layout(t, name, dtype, shape):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name}: expected a torch.Tensor, got {type(t).__name__}")
    if t.dtype != dtype:
        raise TypeError(f"{name}: dtype {t.dtype}, expected {dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: shape {tuple(t.shape)}, expected {tuple(shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: tensor is not contiguous")


def _device_tensors(*specs):
    """Check device buffers against what the C ABI will read or write through their
    pointers (the ABI sees no sizes).  Each spec is (tensor, name, dtype, shape, device):
    a torch tensor of that dtype and exact shape, contiguous, on the operator's device
    (device None: any HIP device).  Layouts are checked first, then devices; anything
    wrong raises before a call is made.  Returns the pointers."""
    for t, name, dtype, shape, _ in specs:
        _layout(t, name, dtype, shape)
    for t, name, _, _, device in specs:
        if t.device.type != "cuda" or (device is not None and t.device.index != device):
            raise ValueError(f"{name}: tensor on {t.device}, expected cuda:{device}")
    return [ctypes.c_void_p(t.data_ptr()) for t, *_ in specs]


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Operator:
    """Widefield operator for nchan channels sharing one image geometry.

    uvw_m      (nrows, 3) float64 metres (host array).
    freqs_hz   channel frequencies.
    chan_rows  optional per-channel row counts (channel c uses its own block of rows).
    weights    optional float32 [total rows] data weights (row k of Phi scaled by them).
    flags      optional bool / uint8 [total rows]; True discards the measurement.
    Options: see include/wf.h (J, beta, alpha, smax, eps_w, nbins, strategy, store, ...).
    """

    def __init__(self, uvw_m, freqs_hz, nx, ny, cell_rad, memory_budget=288e9,
                 chan_rows=None, stream=None, weights=None, flags=None, **opts):
        self._lib = _lib.load()
        self._h = ctypes.c_void_p()
        uvw = np.ascontiguousarray(uvw_m, dtype=np.float64)
        fr = np.ascontiguousarray(np.atleast_1d(freqs_hz), dtype=np.float64)
        cr = None
        if chan_rows is not None:
            cr = np.ascontiguousarray(chan_rows, dtype=np.int64)
        self.nchan = int(fr.size)
        self.nx, self.ny = int(nx), int(ny)
        self.nrows_total = int(cr.sum()) if cr is not None else int(uvw.shape[0]) * self.nchan
        self.opts = default_options(**opts)
        wts = fl = None
        if weights is not None:
            wts = np.ascontiguousarray(weights, dtype=np.float32)
            if wts.shape != (self.nrows_total,):
                raise ValueError(f"weights must have shape ({self.nrows_total},)")
            self.opts.weights = wts.ctypes.data
        if flags is not None:
            fl = np.ascontiguousarray(flags, dtype=np.uint8)
            if fl.shape != (self.nrows_total,):
                raise ValueError(f"flags must have shape ({self.nrows_total},)")
            self.opts.flags = fl.ctypes.data
        shape = WfImageShape(self.nx, self.ny, float(cell_rad))
        import torch
        self.device = torch.cuda.current_device()
        st = self._lib.wf_build_operator(
            uvw.ctypes.data_as(ctypes.c_void_p), ctypes.c_int64(uvw.shape[0]),
            cr.ctypes.data_as(ctypes.c_void_p) if cr is not None else None,
            fr.ctypes.data_as(ctypes.c_void_p), ctypes.c_int32(self.nchan), shape,
            ctypes.c_uint64(int(memory_budget)), ctypes.byref(self.opts),
            _stream_handle(stream), ctypes.byref(self._h))
        self.opts.weights = None
        self.opts.flags = None
        check(st, "wf_build_operator")

    # ------------------------------------------------------------------ applies
    def _img_shape(self):
        return (self.nchan, self.ny, self.nx)

    def _out(self, out, shape, dtype):
        import torch
        if out is None:
            out = torch.empty(shape, dtype=dtype, device=f"cuda:{self.device}")
        return out

    def _call(self, name, a, a_spec, b, b_spec, stream):
        pa, pb = _device_tensors((a, f"{name} input", *a_spec, self.device),
                                 (b, f"{name} output", *b_spec, self.device))
        check(getattr(self._lib, name)(self._h, pa, pb, _stream_handle(stream)), name)

    def forward(self, img, out=None, stream=None):
        """y = Phi x; img float32 [nchan, ny, nx] -> complex64 [total rows]."""
        import torch
        out = self._out(out, (self.nrows_total,), torch.complex64)
        self._call("wf_forward", img, (torch.float32, self._img_shape()), out,
                   (torch.complex64, (self.nrows_total,)), stream)
        return out

    def adjoint(self, vis, out=None, stream=None):
        """Phi^dag y; vis complex64 [total rows] -> complex64 [nchan, ny, nx]."""
        import torch
        out = self._out(out, self._img_shape(), torch.complex64)
        self._call("wf_adjoint", vis, (torch.complex64, (self.nrows_total,)), out,
                   (torch.complex64, self._img_shape()), stream)
        return out

    def psf_apply(self, img, out=None, stream=None):
        """Phi^dag Phi x; img float32 [nchan, ny, nx] -> complex64 [nchan, ny, nx]."""
        import torch
        out = self._out(out, self._img_shape(), torch.complex64)
        self._call("wf_psf_apply", img, (torch.float32, self._img_shape()), out,
                   (torch.complex64, self._img_shape()), stream)
        return out

    def psf_apply_re(self, img, out=None, stream=None):
        """Re{Phi^dag Phi x}; img float32 -> float32 [nchan, ny, nx]."""
        import torch
        out = self._out(out, self._img_shape(), torch.float32)
        self._call("wf_psf_apply_re", img, (torch.float32, self._img_shape()), out,
                   (torch.float32, self._img_shape()), stream)
        return out

    # ------------------------------------------------------------------ introspection
    def plan(self, chan=0) -> dict:
        info = WfPlanInfo()
        check(self._lib.wf_get_plan(self._h, chan, ctypes.byref(info)), "wf_get_plan")
        return {k: getattr(info, k) for k, _ in WfPlanInfo._fields_}

    def centroids(self, chan=0):
        P = self.plan(chan)["nbins"]
        out = np.zeros(P, dtype=np.float64)
        check(self._lib.wf_get_centroids(self._h, chan, out.ctypes.data_as(ctypes.c_void_p), P),
              "wf_get_centroids")
        return out

    def bin_rows(self, chan=0):
        P = self.plan(chan)["nbins"]
        out = np.zeros(P, dtype=np.int64)
        check(self._lib.wf_get_bin_rows(self._h, chan, out.ctypes.data_as(ctypes.c_void_p), P),
              "wf_get_bin_rows")
        return out

    def get_row(self, row, chan=0):
        """(T, qu0, qv0, bin, values complex64 [T, T]) of one stored row of G."""
        T, qu, qv, b = (ctypes.c_int32() for _ in range(4))
        buf = np.zeros(2 * 64 * 64, dtype=np.float32)
        check(self._lib.wf_get_row(self._h, chan, ctypes.c_int64(row), ctypes.byref(T),
                                   ctypes.byref(qu), ctypes.byref(qv), ctypes.byref(b),
                                   buf.ctypes.data_as(ctypes.c_void_p), 64 * 64), "wf_get_row")
        t = T.value
        vals = buf[:2 * t * t].view(np.complex64).reshape(t, t).copy()
        return t, qu.value, qv.value, b.value, vals

    def layer_grid(self, chan, bin_, img, out=None, stream=None):
        """X_p = F Z_p x as complex64 [Ky, Kx] (rows = v)."""
        import torch
        gshape = (2 * self.ny, 2 * self.nx)
        out = self._out(out, gshape, torch.complex64)
        pi, po = _device_tensors(
            (img, "wf_layer_grid input", torch.float32, self._img_shape(), self.device),
            (out, "wf_layer_grid output", torch.complex64, gshape, self.device))
        check(self._lib.wf_layer_grid(self._h, chan, bin_, pi, po, _stream_handle(stream)),
              "wf_layer_grid")
        return out

    def profile_enable(self, kernel_id, enable=True):
        check(self._lib.wf_profile_enable(self._h, kernel_id, int(enable)), "wf_profile_enable")

    def profile_read(self, kernel_id):
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        check(self._lib.wf_profile_read(self._h, kernel_id, ctypes.byref(n), ctypes.byref(ms)),
              "wf_profile_read")
        return n.value, ms.value

    # ------------------------------------------------------------------ forward-backward
    def dirty_image(self, vis, out=None, stream=None):
        """Re{Phi^dag y} as float32 [nchan, ny, nx]."""
        import torch
        out = self._out(out, self._img_shape(), torch.float32)
        self._call("wf_dirty_image", vis, (torch.complex64, (self.nrows_total,)), out,
                   (torch.float32, self._img_shape()), stream)
        return out

    def op_norm(self, iters=50, stream=None):
        """Largest eigenvalue of Re{Phi^dag Phi} by power iteration."""
        v = ctypes.c_double()
        check(self._lib.wf_op_norm(self._h, int(iters), ctypes.byref(v),
                                   _stream_handle(stream)), "wf_op_norm")
        return v.value

    def fb_iterate(self, dirty, x, iters, gamma, lam, stream=None):
        """iters forward-backward iterations (eq. 4) on x in place."""
        import torch
        pd, px = _device_tensors(
            (dirty, "wf_fb_iterate dirty", torch.float32, self._img_shape(), self.device),
            (x, "wf_fb_iterate x", torch.float32, self._img_shape(), self.device))
        check(self._lib.wf_fb_iterate(self._h, pd, px, int(iters), float(gamma), float(lam),
                                      _stream_handle(stream)), "wf_fb_iterate")
        return x

    # ------------------------------------------------------------------ batched form
    def set_branches(self, n):
        """Run applies on n concurrent branches (streams with their own work grids)."""
        check(self._lib.wf_set_branches(self._h, int(n)), "wf_set_branches")

    def set_sweep(self, enable=True, lanes=1):
        """Layer-batched applies: one launch per stage over every (channel, bin) layer,
        on `lanes` streams of contiguous channel ranges (include/wf.h, wf_set_sweep)."""
        n = int(lanes) if enable else 0
        check(self._lib.wf_set_sweep(self._h, n), "wf_set_sweep")

    def capture(self, kind, inp, out, stream):
        """Capture one apply ('forward', 'adjoint', 'psf', 'psf_re') with fixed buffers
        into a HIP graph; stream must be a created torch.cuda.Stream."""
        import torch
        img = (torch.float32, self._img_shape())
        vis = (torch.complex64, (self.nrows_total,))
        cimg = (torch.complex64, self._img_shape())
        spec = {"forward": (img, vis), "adjoint": (vis, cimg), "psf": (img, cimg),
                "psf_re": (img, img)}[kind]
        pi, po = _device_tensors((inp, "wf_graph_capture input", *spec[0], self.device),
                                 (out, "wf_graph_capture output", *spec[1], self.device))
        g = ctypes.c_void_p()
        check(self._lib.wf_graph_capture(self._h, APPLY[kind], pi, po, _stream_handle(stream),
                                         ctypes.byref(g)), "wf_graph_capture")
        return Graph(self, g)

    def latency_enable(self, enable=True):
        check(self._lib.wf_latency_enable(self._h, int(enable)), "wf_latency_enable")

    def read_latency(self):
        """ms from the start of the last apply to each channel's completion."""
        out = np.zeros(self.nchan, dtype=np.float64)
        check(self._lib.wf_read_latency(self._h, out.ctypes.data_as(ctypes.c_void_p),
                                        self.nchan), "wf_read_latency")
        return out

    def bin_tiles(self, chan=0):
        """Work-item tile side of every bin of a channel (include/wf.h, wf_get_bin_tiles)."""
        P = self.plan(chan)["nbins"]
        out = np.zeros(P, dtype=np.int32)
        check(self._lib.wf_get_bin_tiles(self._h, chan, out.ctypes.data_as(ctypes.c_void_p),
                                         P), "wf_get_bin_tiles")
        return out

    def set_bin_tiles(self, tiles, chan=0):
        t = np.ascontiguousarray(tiles, dtype=np.int32)
        check(self._lib.wf_set_bin_tiles(self._h, chan, t.ctypes.data_as(ctypes.c_void_p),
                                         t.size), "wf_set_bin_tiles")

    def autotune(self, img, out, reps=3, stream=None) -> dict:
        import torch
        pi, po = _device_tensors(
            (img, "wf_autotune input", torch.float32, self._img_shape(), self.device),
            (out, "wf_autotune output", torch.float32, self._img_shape(), self.device))
        info = WfTuneInfo()
        check(self._lib.wf_autotune(self._h, pi, po, _stream_handle(stream), int(reps),
                                    ctypes.byref(info)), "wf_autotune")
        return {k: getattr(info, k) for k, _ in WfTuneInfo._fields_}

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self._lib.wf_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Graph:
    """An apply captured into a HIP graph (see wf_graph_capture in include/wf.h)."""

    def __init__(self, op, handle):
        self._op = op          # keeps the operator alive while the graph exists
        self._lib = op._lib
        self._g = handle

    def launch(self, stream=None):
        check(self._lib.wf_graph_launch(self._g, _stream_handle(stream)), "wf_graph_launch")

    def nodes(self):
        """(kernel launches, all nodes) of the captured apply."""
        k, n = ctypes.c_int64(), ctypes.c_int64()
        check(self._lib.wf_graph_nodes(self._g, ctypes.byref(k), ctypes.byref(n)),
              "wf_graph_nodes")
        return int(k.value), int(n.value)

    def close(self):
        if getattr(self, "_g", None) and self._g.value:
            self._lib.wf_graph_destroy(self._g)
            self._g = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Network:
    """Residual-kernel network (include/wf.h, learned kernels): FP32 training and BF16
    inference on the GPU.  Tensors are torch tensors on the current HIP device."""

    NIN, NOUT = 5, 451

    def __init__(self, seed=5):
        self._lib = _lib.load()
        self._h = ctypes.c_void_p()
        check(self._lib.wf_mlp_create(ctypes.c_uint64(seed), ctypes.byref(self._h)),
              "wf_mlp_create")

    @staticmethod
    def num_params():
        return int(_lib.load().wf_mlp_num_params())

    def get_params(self):
        out = np.zeros(self.num_params(), dtype=np.float32)
        check(self._lib.wf_mlp_get_params(self._h, out.ctypes.data_as(ctypes.c_void_p),
                                          out.size), "wf_mlp_get_params")
        return out

    def set_params(self, theta):
        theta = np.ascontiguousarray(theta, dtype=np.float32)
        check(self._lib.wf_mlp_set_params(self._h, theta.ctypes.data_as(ctypes.c_void_p),
                                          theta.size), "wf_mlp_set_params")

    @staticmethod
    def inputs(w, L, fu, fv, stream=None, **opts):
        """Network inputs [n, 5] and uncapped kernel sides [n] from float64 tensors."""
        import torch
        n = w.numel()
        dev = w.device.index
        ptrs = _device_tensors(*((t, f"wf_mlp_inputs {nm}", torch.float64, (n,), dev)
                                 for t, nm in ((w, "w"), (L, "L"), (fu, "fu"), (fv, "fv"))))
        x = torch.empty((n, 5), dtype=torch.float32, device=w.device)
        nk = torch.empty(n, dtype=torch.int32, device=w.device)
        o = default_options(**opts)
        check(_lib.load().wf_mlp_inputs(*ptrs, n, ctypes.byref(o), ctypes.c_void_p(x.data_ptr()),
                                        ctypes.c_void_p(nk.data_ptr()), _stream_handle(stream)),
              "wf_mlp_inputs")
        return x, nk

    @staticmethod
    def targets(w, L, stream=None, **opts):
        """Exact thresholded kernels [n, 450] (zeros where the side exceeds 15)."""
        import torch
        n = w.numel()
        dev = w.device.index
        pw, pL = _device_tensors((w, "wf_mlp_targets w", torch.float64, (n,), dev),
                                 (L, "wf_mlp_targets L", torch.float64, (n,), dev))
        t = torch.empty((n, 450), dtype=torch.float32, device=w.device)
        o = default_options(**opts)
        check(_lib.load().wf_mlp_targets(pw, pL, n, ctypes.byref(o), ctypes.c_void_p(t.data_ptr()),
                                         _stream_handle(stream)), "wf_mlp_targets")
        return t

    @staticmethod
    def _xt(x, t, name):
        import torch
        n = x.shape[0] if hasattr(x, "shape") and len(x.shape) else 0
        dev = x.device.index if hasattr(x, "device") else None
        return _device_tensors((x, f"{name} x", torch.float32, (n, Network.NIN), dev),
                               (t, f"{name} t", torch.float32, (n, Network.NOUT - 1), dev))

    def loss_grad(self, x, t, stream=None):
        import torch
        px, pt = self._xt(x, t, "wf_mlp_loss_grad")
        g = torch.empty(self.num_params(), dtype=torch.float32, device=x.device)
        loss = torch.empty(2, dtype=torch.float32, device=x.device)
        check(self._lib.wf_mlp_loss_grad(self._h, px, pt, x.shape[0],
                                         ctypes.c_void_p(g.data_ptr()),
                                         ctypes.c_void_p(loss.data_ptr()),
                                         _stream_handle(stream)), "wf_mlp_loss_grad")
        return loss, g

    def adam_step(self, lr, stream=None):
        check(self._lib.wf_mlp_adam_step(self._h, ctypes.c_float(lr), _stream_handle(stream)),
              "wf_mlp_adam_step")

    def train(self, x, t, batch=4096, epochs=10, lr0=1e-3, lr_end=1e-5, seed=5, stream=None):
        """Returns the per-epoch mean (kernel loss, error-output loss)."""
        import torch
        px, pt = self._xt(x, t, "wf_mlp_train")
        hist = torch.zeros((max(epochs, 1), 2), dtype=torch.float32, device=x.device)
        check(self._lib.wf_mlp_train(self._h, px, pt, x.shape[0], batch, epochs,
                                     lr0, lr_end, ctypes.c_uint64(seed),
                                     ctypes.c_void_p(hist.data_ptr()), _stream_handle(stream)),
              "wf_mlp_train")
        return hist[:epochs].cpu().numpy() / max(x.shape[0] // batch, 1)

    def infer(self, x, bf16=2, out=None, stream=None):
        """bf16: 0 FP32 kernels, 1 plain BF16, 2 split BF16 (the build's form)."""
        import torch
        n = x.shape[0] if hasattr(x, "shape") and len(x.shape) else 0
        dev = x.device.index if hasattr(x, "device") else None
        _layout(x, "wf_mlp_infer x", torch.float32, (n, self.NIN))
        if out is None:
            out = torch.empty((n, self.NOUT), dtype=torch.float32, device=x.device)
        px, po = _device_tensors((x, "wf_mlp_infer x", torch.float32, (n, self.NIN), dev),
                                 (out, "wf_mlp_infer out", torch.float32, (n, self.NOUT), dev))
        check(self._lib.wf_mlp_infer(self._h, px, n, int(bf16), po,
                                     _stream_handle(stream)), "wf_mlp_infer")
        return out

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self._lib.wf_mlp_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
