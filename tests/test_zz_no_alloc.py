"""Allocation-free Briggs weighting (wf_briggs_weights_noalloc, include/wf.h) against the
allocating entry point wf_briggs_weights, through the C ABI, on two calls in a row --
the second smaller, so that the shared static scratch must be cleared between calls."""
import ctypes

import numpy as np
import pytest

import wfsynth as ws

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _host_weights(lib, obs, uvw, nat, flags, robust):
    from paper_2605_26347_amd._lib import WfImageShape, check
    M = uvw.shape[0]
    out = np.empty(M, dtype=np.float32)
    fr = np.array([obs.freqs_hz[0]], dtype=np.float64)
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
    check(lib.wf_briggs_weights(p(uvw), ctypes.c_int64(M), None, p(fr), 1,
                                WfImageShape(obs.nx, obs.ny, obs.cell_rad), float(robust),
                                p(nat), p(flags), p(out), None), "wf_briggs_weights")
    return out


def _device_weights(lib, obs, uvw, nat, flags, robust, stream):
    from paper_2605_26347_amd._lib import WfImageShape, check
    M = uvw.shape[0]
    du = torch.from_numpy(uvw).to("cuda:0")
    dn = torch.from_numpy(nat).to("cuda:0")
    df = torch.from_numpy(flags).to("cuda:0")
    out = torch.full((M,), float("nan"), dtype=torch.float32, device="cuda:0")
    torch.cuda.synchronize()
    check(lib.wf_briggs_weights_noalloc(ctypes.c_void_p(du.data_ptr()), ctypes.c_int64(M),
                                        float(obs.freqs_hz[0]),
                                        WfImageShape(obs.nx, obs.ny, obs.cell_rad),
                                        float(robust), ctypes.c_void_p(dn.data_ptr()),
                                        ctypes.c_void_p(df.data_ptr()),
                                        ctypes.c_void_p(out.data_ptr()),
                                        ctypes.c_void_p(stream.cuda_stream)),
          "wf_briggs_weights_noalloc")
    stream.synchronize()
    return out.cpu().numpy()


def test_noalloc_briggs_matches_allocating_entry_point():
    from paper_2605_26347_amd import _lib
    lib = _lib.load()
    stream = torch.cuda.Stream()
    # first call on 1024^2 / 60k rows, then a smaller one on 256^2 / 15k rows
    for n, nvis, R in ((1024, 60_000, 0.5), (256, 15_000, -1.0)):
        obs = ws.widefield(n=n, nvis=nvis, fov_deg=2.0, sky=False)
        uvw = np.ascontiguousarray(obs.uvw_m, dtype=np.float64)
        M = uvw.shape[0]
        nat = (1.0 / ws.noise_sigma(M).astype(np.float64) ** 2).astype(np.float32)
        flags = ws.flag_runs(M, 0.05).astype(np.uint8)
        ref = _host_weights(lib, obs, uvw, nat, flags, R)
        got = _device_weights(lib, obs, uvw, nat, flags, R, stream)
        assert np.all(np.isfinite(got))
        assert np.all(got[flags.astype(bool)] == 0)
        err = float(np.max(np.abs(got - ref)) / np.max(ref))
        print(f"[gpu] noalloc Briggs {n}^2 / {M} rows: max error {err:.2e} of the largest weight",
              flush=True)
        assert err <= 1e-6


def test_noalloc_rejects_oversized_grid():
    from paper_2605_26347_amd import _lib
    from paper_2605_26347_amd._lib import WfImageShape, WF_EINVAL
    lib = _lib.load()
    st = lib.wf_briggs_weights_noalloc(None, ctypes.c_int64(0), 1.0e9,
                                       WfImageShape(4096, 2048, 1e-5), 0.0, None, None, None,
                                       None)
    assert st == WF_EINVAL
