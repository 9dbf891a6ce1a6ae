"""Drive the host-side entry points of the AddressSanitizer build of the library (run by
tests/test_host_asan.py in a child process with the sanitizer runtime preloaded; no GPU
and no torch).  Exercises the planner (Sect. 3.4: k-means over the planning subset,
K(P), eq. 5/9/10, the decision tree of Fig. 2) on seeded inputs at budgets that reach
each branch, and every argument check that runs before a device is touched.  Prints
'asan driver ok' at the end; any sanitizer report aborts the process first."""
import ctypes
import importlib.util
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import wfsynth as ws  # noqa: E402

spec = importlib.util.spec_from_file_location(
    "wf_lib_decls", os.path.join(ROOT, "paper_2605_26347_amd", "_lib.py"))
L = importlib.util.module_from_spec(spec)
spec.loader.exec_module(L)

lib = L.bind(ctypes.CDLL(sys.argv[1]))
ptr = lambda a: None if a is None else a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731


def options(**kw):
    o = L.WfOptions()
    lib.wf_default_options(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def plan(uvw, f, n, cell, budget, **kw):
    o = options(**kw)
    info = L.WfPlanInfo()
    cent = np.zeros(256)
    st = lib.wf_plan(ptr(uvw), ctypes.c_int64(uvw.shape[0]), f, L.WfImageShape(n, n, cell),
                     ctypes.c_uint64(int(budget)), ctypes.byref(o), ctypes.byref(info),
                     ptr(cent), cent.size)
    return st, info, cent


def build(uvw, freqs, n=64, cell=1e-4, chan_rows=None, **kw):
    o = options(**kw)
    h = ctypes.c_void_p()
    fr = np.ascontiguousarray(freqs, dtype=np.float64)
    st = lib.wf_build_operator(ptr(uvw), uvw.shape[0], ptr(chan_rows), ptr(fr), fr.size,
                               L.WfImageShape(n, n, cell), 1 << 30, ctypes.byref(o), None,
                               ctypes.byref(h))
    return st, h


# planner on a widefield sample: generous, tight and too-small budgets, both storages,
# forced P, and a tiny input
obs = ws.widefield(n=1024, nvis=200_000, fov_deg=2.0, sky=False)
uvw = np.ascontiguousarray(obs.uvw_m)
f = float(obs.freqs_hz[0])
seen = set()
for budget in (288e9, 2e9, 4e8, 1e8, 1e6):
    for store in (0, 1, 2):
        st, info, cent = plan(uvw, f, 1024, obs.cell_rad, budget, store=store)
        assert st in (L.WF_OK, L.WF_EBUDGET), (st, lib.wf_last_error())
        if st == L.WF_OK:
            seen.add(info.strategy)
            P = info.nbins
            assert 1 <= P <= 256 and np.all(np.diff(cent[:P]) > 0)
st, info, _ = plan(uvw, f, 1024, obs.cell_rad, 288e9, nbins=8)
assert st == L.WF_OK and info.nbins == 8
for strategy in (1, 2, 3):
    st, info, _ = plan(uvw, f, 1024, obs.cell_rad, 4e8, strategy=strategy)
    assert st in (L.WF_OK, L.WF_EBUDGET), (strategy, st, lib.wf_last_error())
    if st == L.WF_OK:
        seen.add(info.strategy)
small = np.ascontiguousarray(uvw[:3])
st, info, _ = plan(small, f, 64, 1e-4, 1e9)
assert st == L.WF_OK, lib.wf_last_error()
print("planner strategies reached:", sorted(seen), flush=True)

# argument checks before any device use
UVW = np.ascontiguousarray(np.random.default_rng(0).normal(0, 100, (50, 3)))
for kw in (dict(n=48), dict(n=4), dict(cell=0.0), dict(cell=0.02), dict(J=6), dict(smax=33),
           dict(J=9, smax=31), dict(nbins=300), dict(oversample=3), dict(tile=48),
           dict(branches=17)):
    st, h = build(UVW, [1e9], **kw)
    assert st == L.WF_EINVAL and not h.value, (kw, st)
st, h = build(UVW, [1e9, 1.2e9], chan_rows=np.array([20, 20], dtype=np.int64))
assert st == L.WF_EINVAL
bad = UVW.copy()
bad[3, 1] = np.nan
assert build(bad, [1e9])[0] == L.WF_EINVAL
w = np.ones(UVW.shape[0], dtype=np.float32)
w[7] = np.inf
assert build(UVW, [1e9], weights=w.ctypes.data)[0] == L.WF_EINVAL
st, info, cent = plan(UVW, 1e9, 64, 1e-4, 1e9, nbins=300)
assert st == L.WF_EINVAL
assert lib.wf_plan(None, 0, 1e9, L.WfImageShape(64, 64, 1e-4), 1 << 30, None, None, None,
                   0) == L.WF_EINVAL
for call in (lambda: lib.wf_psf_apply(None, None, None, None),
             lambda: lib.wf_destroy(None),
             lambda: lib.wf_set_branches(None, 2),
             lambda: lib.wf_set_sweep(None, 1),
             lambda: lib.wf_graph_launch(None, None),
             lambda: lib.wf_graph_destroy(None),
             lambda: lib.wf_latency_enable(None, 1),
             lambda: lib.wf_read_latency(None, None, 0),
             lambda: lib.wf_autotune(None, None, None, None, 1, None),
             lambda: lib.wf_mlp_destroy(None),
             lambda: lib.wf_mlp_get_params(None, None, 0)):
    assert call() == L.WF_EINVAL
    assert len(lib.wf_last_error()) > 0
nat = -np.ones(UVW.shape[0], dtype=np.float32)
out = np.zeros(UVW.shape[0], dtype=np.float32)
fr = np.array([1e9])
assert lib.wf_briggs_weights(ptr(UVW), UVW.shape[0], None, ptr(fr), 1,
                             L.WfImageShape(64, 64, 1e-4), 0.0, ptr(nat), None, ptr(out),
                             None) == L.WF_EINVAL
print("asan driver ok", flush=True)
