"""Host-side checks of the C ABI (no GPU): the library loads, exports every function
that include/wf.h declares, and rejects invalid arguments before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2605_26347_amd import _lib, default_options
from paper_2605_26347_amd._lib import WfImageShape, WfOptions

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "wf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(wf_[a-z_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    lib = _lib.load()
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
        assert n in _lib.SIGNATURES, n


def test_default_options():
    o = default_options()
    assert (o.J, o.oversample, o.smax, o.nbins, o.store) == (7, 2, 31, 0, 0)
    assert abs(o.beta - 2.34 * 7) < 1e-12 and o.eps_w == 1e-6
    assert o.plan_fraction == 0.01 and o.budget_fraction == 0.65
    assert o.branches == 0 and o.max_rows_per_item == 0 and o.otf_form == 0


def _build(uvw, freqs, nx=64, ny=64, cell=1e-4, chan_rows=None, **kw):
    lib = _lib.load()
    h = ctypes.c_void_p()
    o = default_options(**kw)
    uvw = np.ascontiguousarray(uvw, dtype=np.float64)
    fr = np.ascontiguousarray(freqs, dtype=np.float64)
    cr = None if chan_rows is None else np.ascontiguousarray(chan_rows, dtype=np.int64)
    st = lib.wf_build_operator(uvw.ctypes.data_as(ctypes.c_void_p), uvw.shape[0],
                               None if cr is None else cr.ctypes.data_as(ctypes.c_void_p),
                               fr.ctypes.data_as(ctypes.c_void_p), fr.size,
                               WfImageShape(nx, ny, cell), 1 << 30, ctypes.byref(o), None,
                               ctypes.byref(h))
    return st, lib.wf_last_error().decode(), h


UVW = np.random.default_rng(0).normal(0, 100, (50, 3))


@pytest.mark.parametrize("kw,frag", [
    (dict(nx=48), "powers of two"),
    (dict(nx=4, ny=4), "powers of two"),
    (dict(cell=0.0), "cell"),
    (dict(cell=0.02), "too wide"),
    (dict(J=6), "J must be odd"),
    (dict(smax=33), "smax"),
    (dict(J=9, smax=31), "patch side"),
    (dict(nbins=300), "nbins"),
    (dict(oversample=3), "oversample"),
    (dict(tile=48), "tile"),
    (dict(branches=17), "branches"),
    (dict(otf_form=3), "otf_form"),
    (dict(otf_form=-1), "otf_form"),
])
def test_invalid_arguments(kw, frag):
    st, msg, h = _build(UVW, [1e9], **kw)
    assert st == _lib.WF_EINVAL and frag in msg and not h.value


def test_invalid_rows_and_freqs():
    st, msg, _ = _build(UVW, [1e9, 1.2e9], chan_rows=[20, 20])
    assert st == _lib.WF_EINVAL and "sum" in msg
    st, msg, _ = _build(UVW, [-1e9])
    assert st == _lib.WF_EINVAL and "frequencies" in msg
    bad = UVW.copy()
    bad[3, 1] = np.nan
    st, msg, _ = _build(bad, [1e9])
    assert st == _lib.WF_EINVAL and "non-finite" in msg


def test_null_handle_calls():
    lib = _lib.load()
    assert lib.wf_psf_apply(None, None, None, None) == _lib.WF_EINVAL
    assert lib.wf_destroy(None) == _lib.WF_EINVAL
    assert b"null" in lib.wf_last_error()


def test_null_handle_batched_calls():
    lib = _lib.load()
    g = ctypes.c_void_p()
    assert lib.wf_set_branches(None, 2) == _lib.WF_EINVAL
    assert lib.wf_graph_capture(None, 3, None, None, None, ctypes.byref(g)) == _lib.WF_EINVAL
    assert not g.value
    assert lib.wf_graph_launch(None, None) == _lib.WF_EINVAL
    assert lib.wf_graph_destroy(None) == _lib.WF_EINVAL
    k, n = ctypes.c_int64(-1), ctypes.c_int64(-1)
    assert lib.wf_graph_nodes(None, ctypes.byref(k), ctypes.byref(n)) == _lib.WF_EINVAL
    assert lib.wf_set_sweep(None, 1) == _lib.WF_EINVAL
    assert lib.wf_latency_enable(None, 1) == _lib.WF_EINVAL
    assert lib.wf_read_latency(None, None, 0) == _lib.WF_EINVAL
    assert lib.wf_autotune(None, None, None, None, 1, None) == _lib.WF_EINVAL


def test_network_host_calls():
    lib = _lib.load()
    assert lib.wf_mlp_num_params() == 5 * 256 + 256 + 3 * (256 * 256 + 256) + 256 * 451 + 451
    assert lib.wf_mlp_destroy(None) == _lib.WF_EINVAL
    assert lib.wf_mlp_get_params(None, None, 0) == _lib.WF_EINVAL
    assert lib.wf_mlp_infer(None, None, 0, 1, None, None) == _lib.WF_EINVAL
    assert lib.wf_mlp_train(None, None, None, 0, 1, 1, 1e-3, 1e-5, 0, None, None) == _lib.WF_EINVAL
    o = default_options()
    assert o.surrogate is None and o.surrogate_tol == 1e-3


def test_weight_and_briggs_host_checks():
    lib = _lib.load()
    h = ctypes.c_void_p()
    o = default_options()
    w = np.ones(UVW.shape[0], dtype=np.float32)
    w[7] = np.inf
    o.weights = w.ctypes.data
    uvw = np.ascontiguousarray(UVW)
    fr = np.array([1e9])
    st = lib.wf_build_operator(uvw.ctypes.data_as(ctypes.c_void_p), uvw.shape[0], None,
                               fr.ctypes.data_as(ctypes.c_void_p), 1, WfImageShape(64, 64, 1e-4),
                               1 << 30, ctypes.byref(o), None, ctypes.byref(h))
    assert st == _lib.WF_EINVAL and b"weight" in lib.wf_last_error() and not h.value
    with pytest.raises(TypeError):
        default_options(weights=None)
    out = np.zeros(uvw.shape[0], dtype=np.float32)
    ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
    nat = -np.ones(uvw.shape[0], dtype=np.float32)
    assert lib.wf_briggs_weights(ptr(uvw), uvw.shape[0], None, ptr(fr), 1,
                                 WfImageShape(64, 64, 1e-4), 0.0, ptr(nat), None, ptr(out),
                                 None) == _lib.WF_EINVAL
    assert b"natural" in lib.wf_last_error()
    assert lib.wf_briggs_weights(ptr(uvw), uvw.shape[0], None, ptr(fr), 1,
                                 WfImageShape(64, 64, 1e-4), float("nan"), None, None,
                                 ptr(out), None) == _lib.WF_EINVAL
    assert lib.wf_briggs_weights(ptr(uvw), uvw.shape[0], None, ptr(fr), 1,
                                 WfImageShape(0, 64, 1e-4), 0.0, None, None, ptr(out),
                                 None) == _lib.WF_EINVAL
    # no rows: nothing to do, no device work
    assert lib.wf_briggs_weights(None, 0, None, ptr(fr), 1, WfImageShape(64, 64, 1e-4), 0.0,
                                 None, None, ptr(out), None) == _lib.WF_OK


def _declarations():
    """name -> number of parameters of every function include/wf.h declares."""
    src = open(os.path.join(ROOT, "include", "wf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    out = {}
    for m in re.finditer(r"\b(wf_[a-z_0-9]+)\s*\(([^;{]*?)\)\s*;", src, flags=re.S):
        params = m.group(2).strip()
        out[m.group(1)] = 0 if params in ("", "void") else params.count(",") + 1
    return out


def test_binding_argument_counts_match_header():
    decl = _declarations()
    assert len(decl) >= 30
    for name, (_, args) in _lib.SIGNATURES.items():
        assert name in decl, name
        assert len(args) == decl[name], (name, len(args), decl[name])


def test_binding_struct_layouts_match_header(tmp_path):
    """The ctypes mirrors of the ABI's structs have the C compiler's size and offsets."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"wf_image_shape": _lib.WfImageShape, "wf_options": _lib.WfOptions,
               "wf_plan_info": _lib.WfPlanInfo, "wf_tune_info": _lib.WfTuneInfo}
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "wf.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "probe"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True, capture_output=True)
    got = {}
    for ln in subprocess.run([str(exe)], check=True, capture_output=True,
                             text=True).stdout.splitlines():
        cname, field, val = ln.split()
        got[(cname, field)] = int(val)
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)
