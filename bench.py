#!/usr/bin/env python3
"""Benchmark of the widefield Phi^dag Phi apply on one MI355X.

Workload: 4096^2 image over a 3 degree field, 50M visibilities of the 64-antenna
array over 16 h at 1.28 GHz, w-bin count chosen by the planner (eq. 10) under 288 GB.
One step = one Re{Phi^dag Phi x} apply over all w-bins (the operator the
forward-backward iteration of eq. 4 consumes), inputs resident in HBM.

Two forms are built and timed: G stored as complex FP16 with FP32 accumulation and
FP32 FFTs (the mixed form, reported as `value`) and G stored as complex FP32.
Printed: one JSON line with applies/s, Gvis/s, the mixed/FP32 speedup, the roofline
of the dominant kernel (fused G^dag G, HIP events on its stream during the timed
region) and the FP64 oracle's throughput on a bounded CPU sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Φ†Φ applies/s, Gvis/s (4096², 50M vis): mixed vs FP32 at ≤1e-3 rel err"
HBM_PEAK_GBS = 8000.0
# arithmetic type of the path per value storage of G (phases and coordinates in FP64)
DTYPE = {"f32": "f32", "f16": "f16-stored/f32-compute", "bf16": "bf16-stored/f32-compute"}
FP64_VECTOR_PEAK_TFS = 78.6


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--nvis", type=int, default=50_000_000)
    ap.add_argument("--fov", type=float, default=3.0)
    ap.add_argument("--budget", type=float, default=288e9)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--forms", default="f16,f32")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--workload", default="precision",
                    choices=["precision", "batched", "learned", "holographic", "counters",
                             "onthefly", "weighted", "cpu"],
                    help="precision: one channel 4096^2 / 50M rows (default); batched: "
                         "16 channels 2048^2 / 48M rows, autotuned, one graph per sweep; "
                         "learned: G of 20M rows on 4096^2 / 16 bins built with the "
                         "residual-kernel network vs the exact construction; onthefly: "
                         "the precision form with G rebuilt at every apply (strategy (c)); "
                         "weighted: the precision form with Briggs weights and 10%% flags; "
                         "cpu: the oracle's timing protocol on the host cores")
    ap.add_argument("--train-examples", type=int, default=1_000_000)
    ap.add_argument("--epochs", type=int, default=100)
    ap.add_argument("--store", default="f16", help="value storage of the batched form")
    return ap.parse_args()


KSRC = os.path.join(ROOT, "paper_2605_26347_amd", "csrc", "k_grid.hip")
TRAFFIC = os.path.join(ROOT, "profiles", "gtg_traffic_4096sq_50M.json")


def kernel_hash():
    import hashlib
    return hashlib.sha256(open(KSRC, "rb").read()).hexdigest()[:16]


def measured_traffic(store):
    """HBM bytes per launch of the fused kernel from the committed counter summary, or
    None when it is missing or was taken on a different kernel source."""
    if not os.path.exists(TRAFFIC):
        return None
    d = json.load(open(TRAFFIC))
    if d.get("kernel_sha256_16") != kernel_hash():
        return None
    f = d.get("forms", {}).get(store)
    return None if f is None else f.get("bytes_per_launch")


def gtg_bytes(info, store):
    """Algorithmic bytes of the fused G^dag G kernel over one apply: every stored value
    of G once (b_v per tap), the per-row metadata (patch origin word + value offset) and
    the work-item records.  Grid reads and writes are not counted (lower bound)."""
    bv = 8 if store == "f32" else 4
    return bv * info["ntaps"] + 8 * info["nrows"] + 32 * info["nwork"]


def time_form(obs, store, args, torch):
    from paper_2605_26347_amd import Operator
    t0 = time.time()
    op = Operator(obs.uvw_m, obs.freqs_hz, obs.nx, obs.ny, obs.cell_rad,
                  memory_budget=args.budget, store=store)
    tb = time.time() - t0
    info = op.plan(0)
    log(f"{store}: built in {tb:.1f} s: P={info['nbins']} (P*={info['p_star']}, "
        f"P_WSClean={info['p_wsclean']}), taps={info['ntaps']:.3e}, "
        f"G={info['mem_g_bytes'] / 1e9:.1f} GB, work items={info['nwork']}, "
        f"capped={info['capped_fraction']:.4f}")
    x = torch.from_numpy(obs.sky.astype(np.float32)[None]).to("cuda:0")
    out = torch.empty_like(x)
    stream = torch.cuda.current_stream()
    # the library's autotuner picks the rows per work item and the number of concurrent
    # branches (w-bins of the channel spread over streams) by timing applies
    tune = op.autotune(x, out, reps=2)
    info = op.plan(0)
    log(f"{store}: autotune {tune}, rows per item {info['max_rows_per_item']}")
    for i in range(args.warmup):
        op.psf_apply_re(x, out)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    start.record(stream)
    for i in range(args.steps):
        op.psf_apply_re(x, out)
    end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    ms = start.elapsed_time(end) / args.steps
    # the fused kernel on its own (one branch, so that no other kernel shares the GPU
    # while its launches are timed), HIP events on its stream
    op.set_branches(1)
    for i in range(args.warmup):
        op.psf_apply_re(x, out)
    op.profile_enable(0, True)
    for i in range(args.steps):
        op.psf_apply_re(x, out)
    nl, kms = op.profile_read(0)
    op.profile_enable(0, False)
    log(f"{store}: {ms:.3f} ms/apply (wall {1e3 * wall / args.steps:.3f}) on "
        f"{tune['branches']} branches; G^dag G alone {kms / max(nl, 1):.3f} ms/launch over "
        f"{nl} launches")
    # Phi (de-gridding) and Phi^dag (gridding) applies on their own, tuned branches
    op.set_branches(tune["branches"])
    y = op.forward(x)
    img_c = op.adjoint(y)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for i in range(args.steps):
        op.forward(x, out=y)
    e1.record(stream)
    torch.cuda.synchronize()
    fwd_ms = e0.elapsed_time(e1) / args.steps
    e0.record(stream)
    for i in range(args.steps):
        op.adjoint(y, out=img_c)
    e1.record(stream)
    torch.cuda.synchronize()
    adj_ms = e0.elapsed_time(e1) / args.steps
    log(f"{store}: Phi {fwd_ms:.3f} ms, Phi^dag {adj_ms:.3f} ms per apply")
    del y, img_c
    res = dict(ms=ms, info=info, build_s=tb, gtg_launches=nl, gtg_ms_total=kms,
               out=out.clone(), store=store, tune=tune, fwd_ms=fwd_ms, adj_ms=adj_ms)
    if store == args.forms.split(",")[0]:
        # forward-backward iterations (eq. 4) on the same operator, tuned branches
        op.set_branches(tune["branches"])
        y = op.forward(x)
        dirty = op.dirty_image(y)
        L = op.op_norm(10)
        xk = torch.zeros_like(x)
        op.fb_iterate(dirty, xk, 1, 1.0 / L, 0.0)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        op.fb_iterate(dirty, xk, 5, 1.0 / L, 0.0)
        e1.record(stream)
        torch.cuda.synchronize()
        res["fb_ms"] = e0.elapsed_time(e1) / 5
        log(f"{store}: forward-backward iteration {res['fb_ms']:.3f} ms")
    op.close()
    del op
    torch.cuda.empty_cache()
    return res


def accuracy_vs_oracle(forms, torch):
    """Relative L2 error of Phi^dag Phi x against the FP64 oracle on the stored samples
    (tests/golden/fullsize_*.npz, written by a script that calls only the oracle): all 50M
    rows on the central 512^2 crop, and the 4096^2 image with a seeded 300k-row subset,
    P = 22 w-bins as in the benchmark's plan, each value storage of G."""
    import wfsynth as ws
    from paper_2605_26347_amd import Operator
    res = {}
    for case in ("crop512", "sub4096"):
        fx = np.load(os.path.join(ROOT, "tests", "golden", f"fullsize_{case}.npz"))
        uvw, f, n, cell = ws.fullsize_case(case)
        pix, _ = ws.fullsize_samples(n, uvw.shape[0])
        x = torch.from_numpy(ws.gauss_image(n, 4).astype(np.float32)[None]).to("cuda:0")
        pixd = torch.from_numpy(pix).to("cuda:0")
        ref = fx["psf"]
        for store in forms:
            op = Operator(uvw, [f], n, n, cell, nbins=ws.FULLSIZE_P, store=store)
            got = op.psf_apply(x)[0].flatten()[pixd].cpu().numpy()
            op.close()
            del op
            torch.cuda.empty_cache()
            e = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
            res[f"{store}_{case}"] = e
            log(f"accuracy {case} {store}: Phi^dag Phi rel L2 vs FP64 oracle {e:.2e}")
    return res


def _warm_median(fn, reps=3):
    """One untimed warm-up call, then the median wall time of `reps` calls (seconds)."""
    fn()
    ts = []
    for _ in range(reps):
        t = time.perf_counter()
        fn()
        ts.append(time.perf_counter() - t)
    return float(np.median(ts))


def _host_threads():
    import threadpoolctl
    blas = max([i.get("num_threads", 1) for i in threadpoolctl.threadpool_info()] + [1])
    return {"os_cpu_count": os.cpu_count(), "fft_workers": os.cpu_count(),
            "blas_threads": int(blas), "sparse_products": "one thread (numpy)"}


def oracle_full(obs, nbins, smax, cache_bytes=2 << 30):
    """Seconds per oracle Phi^dag Phi apply of a whole configuration (G's patches cached
    by the warm-up call when they fit `cache_bytes`, as G is stored on the GPU)."""
    from oracle import OracleOperator, OperatorParams
    prm = OperatorParams(obs.nx, obs.ny, obs.cell_rad, smax=smax)
    orc = OracleOperator(obs.uvw_m, obs.freqs_hz[0], prm, nbins=nbins,
                         cache_bytes=cache_bytes)
    return _warm_median(lambda: orc.psf(obs.sky))


def oracle_sampled(uvw, f, n, cell, centroids, nsamp, M_total, x):
    """Seconds per oracle apply extrapolated from a bounded sample: every layer's FFT pair
    and modulation at full size is timed on the most populated layer, the G^dag G products
    on `nsamp` seeded rows of that layer; t = P t_layer + M t_row."""
    from oracle import OracleOperator, OperatorParams, wbins
    from oracle.operator import C_LIGHT
    P = len(centroids)
    b = wbins.assign_bins(uvw[:, 2] * (f / C_LIGHT), centroids)
    pbig = int(np.argmax(np.bincount(b, minlength=P)))
    cand = np.nonzero(b == pbig)[0]
    rng = np.random.default_rng(11)
    rows = np.sort(rng.choice(cand, min(nsamp, cand.size), replace=False))
    orc = OracleOperator(uvw[rows], f, OperatorParams(n, n, cell), centroids=centroids)
    p = int(np.argmax([r.size for r in orc.bin_rows]))
    z = orc.zp(p)
    X = orc.fwd_fft(z * x)
    t_fft = _warm_median(lambda: np.conj(z) * orc.inv_fft_crop(orc.fwd_fft(orc.zp(p) * x)))
    t_rows = _warm_median(lambda: orc.gtg(p, X))
    t_row = t_rows / orc.bin_rows[p].size
    return P * t_fft + M_total * t_row, t_fft, t_row, int(orc.bin_rows[p].size)


def cpu_baseline(obs, P_gpu):
    """FP64 oracle on the host cores (1 warm-up, median of 3 for every timed part): the
    headline apply extrapolated from a bounded sample, and the tiny configuration timed
    in full.  The full protocol (the 1024^2 configuration in full, the 512^2 crop) is the
    'cpu' workload, too long for the default run."""
    import wfsynth as ws
    from oracle import wbins
    from oracle.operator import C_LIGHT
    t0 = time.perf_counter()
    f = float(obs.freqs_hz[0])
    w_all = obs.uvw_m[:, 2] * (f / C_LIGHT)
    mask = wbins.plan_subset_mask(w_all.size, 0.01, 0)
    cents = wbins.kmeans_1d(w_all[mask], P_gpu)
    M = obs.uvw_m.shape[0]
    t_apply, t_fft, t_row, nrow = oracle_sampled(obs.uvw_m, f, obs.nx, obs.cell_rad, cents,
                                                 80_000, M, obs.sky)
    t_tiny = oracle_full(ws.tiny(), 1, 1)
    log(f"cpu oracle: layer FFT pair + modulation {t_fft:.2f} s, {1e6 * t_row:.2f} us/row "
        f"({nrow} rows) -> {t_apply:.0f} s per full apply (extrapolated); tiny "
        f"configuration {1e3 * t_tiny:.1f} ms per apply")
    return {"value": 1.0 / t_apply, "unit": "applies/s", "cores": os.cpu_count(),
            "kind": "oracle", "extrapolated": True,
            "sample": (f"one full-size w-layer (4096^2 image, 8192^2 FFTs) plus the G^dag G "
                       f"products of {nrow} seeded rows of that (most populated) layer, "
                       f"scaled to P={P_gpu} layers and {M} rows: P*t_layer + M*t_row; "
                       f"1 warm-up, median of 3"),
            "threads": _host_threads(),
            "tiny_full_apply_s": t_tiny,
            "seconds": time.perf_counter() - t0}


def bench_cpu(args):
    """The oracle's timing protocol on the host cores, no GPU: the tiny configuration and
    the 1024^2 / 2M-row configuration in full (8 bins, residual kernels up to 15), the
    512^2 crop of the precision form (all 50M rows, P = 22) extrapolated from 1M seeded
    rows, and the 4096^2 precision form extrapolated as in the bench line."""
    import wfsynth as ws
    res = {"threads": _host_threads()}
    o = ws.tiny()
    res["tiny_64sq_19200"] = {"s_per_apply": oracle_full(o, 1, 1), "kind": "full"}
    log(f"tiny: {res['tiny_64sq_19200']}")
    o = ws.widefield()
    res["widefield_1024sq_2M_8bins"] = {"s_per_apply": oracle_full(o, 8, 15, 96 << 30),
                                        "kind": "full"}
    log(f"widefield: {res['widefield_1024sq_2M_8bins']}")
    fx = np.load(os.path.join(ROOT, "tests", "golden", "fullsize_crop512.npz"))
    uvw, f, n, cell = ws.fullsize_case("crop512")
    x = ws.gauss_image(n, 4)
    t, t_fft, t_row, nrow = oracle_sampled(uvw, f, n, cell, fx["centroids"], 1_000_000,
                                           uvw.shape[0], x)
    res["crop512_50M_22bins"] = {"s_per_apply": t, "kind": "extrapolated",
                                 "t_layer_s": t_fft, "t_row_us": 1e6 * t_row, "rows": nrow}
    log(f"crop512: {res['crop512_50M_22bins']}")
    del uvw
    obs = ws.precision_form()
    res["precision_4096sq_50M_22bins"] = cpu_baseline(obs, ws.FULLSIZE_P)
    print(json.dumps({"workload": "oracle timing protocol", "results": res}), flush=True)


def fft_bytes_per_bin(nx, ny):
    """Algorithmic HBM bytes of the four FFT passes of one w-layer on the full grid:
    image read, A written and read twice, X written, Y read, output read and written."""
    K2 = 4 * nx * ny
    return 4 * nx * ny + 4 * (8 * ny * 2 * nx) + 8 * K2 + 8 * K2 + 2 * 8 * nx * ny


def bench_batched(args, torch):
    """Batched form: 16 channels 0.9-1.67 GHz, 2048^2 each, 48M rows in total with
    uneven per-channel counts; per-channel P from the planner; autotuned work items and
    branch count; one HIP graph per sweep of all channels and bins."""
    import wfsynth as ws
    from paper_2605_26347_amd import Operator
    t0 = time.time()
    obs = ws.batched()
    nchan = obs.freqs_hz.size
    M = int(obs.chan_rows.sum())
    log(f"inputs: {nchan} channels, {M} rows ({obs.chan_rows.min()}..{obs.chan_rows.max()} "
        f"per channel), {obs.nx}^2 images, {time.time() - t0:.1f} s")
    t0 = time.time()
    op = Operator(obs.uvw_m, obs.freqs_hz, obs.nx, obs.ny, obs.cell_rad,
                  memory_budget=args.budget, chan_rows=obs.chan_rows, store=args.store)
    tb = time.time() - t0
    plans = [op.plan(c) for c in range(nchan)]
    log(f"built in {tb:.1f} s; P per channel {[p['nbins'] for p in plans]}")
    imgs = np.stack([ws.gauss_image(obs.nx, 100 + c) for c in range(nchan)]).astype(np.float32)
    x = torch.from_numpy(imgs).to("cuda:0")
    out = torch.empty_like(x)
    stream = torch.cuda.Stream()

    def timed(fn, n):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(n):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n

    for _ in range(args.warmup):
        op.psf_apply_re(x, out, stream=stream)
    eager_before = timed(lambda: op.psf_apply_re(x, out, stream=stream), max(2, args.steps // 4))
    op.set_branches(1)
    for _ in range(args.warmup):
        op.psf_apply_re(x, out, stream=stream)
    serial = timed(lambda: op.psf_apply_re(x, out, stream=stream), max(2, args.steps // 4))
    ref = out.clone()
    tune = op.autotune(x, out, reps=2, stream=stream)
    log(f"eager {eager_before:.2f} ms (default branches), {serial:.2f} ms (one branch); "
        f"autotune {tune}")
    op.latency_enable(True)

    def graph_run(label):
        g = op.capture("psf_re", x, out, stream)
        kern, nodes = g.nodes()
        for _ in range(args.warmup):
            g.launch(stream)
        ms = timed(lambda: g.launch(stream), args.steps)
        d = float((out - ref).norm() / ref.norm())
        lat = []
        for _ in range(max(5, args.steps // 2)):
            g.launch(stream)
            stream.synchronize()
            lat.append(op.read_latency())
        lat = np.concatenate(lat)
        g.close()
        log(f"{label}: graph sweep {ms:.2f} ms ({1e3 / ms:.2f} sweeps/s), {kern} kernel "
            f"nodes ({nodes} nodes), vs one-branch eager rel {d:.2e}, latency p50 "
            f"{np.percentile(lat, 50):.2f} p99 {np.percentile(lat, 99):.2f}")
        return dict(ms=ms, rel=d, kernels=kern, nodes=nodes,
                    latency_ms={"p50": float(np.percentile(lat, 50)),
                                "p99": float(np.percentile(lat, 99)),
                                "max": float(lat.max())})

    br = graph_run(f"branches ({tune['branches']})")
    # the persistent form: every layer's grids resident, one launch per FFT stage over all
    # layers and one persistent launch per patch class draining all (channel, bin) items
    t0 = time.time()
    op.set_sweep(True)
    t_sw = time.time() - t0
    # the autotuner in sweep mode: rows per item and item tiles again, then the lane count
    # (channel ranges on streams of their own)
    tune_sw = op.autotune(x, out, reps=2, stream=stream)
    log(f"sweep autotune {tune_sw}")
    for _ in range(args.warmup):
        op.psf_apply_re(x, out, stream=stream)
    eager_sweep = timed(lambda: op.psf_apply_re(x, out, stream=stream), max(2, args.steps // 4))
    sw = graph_run(f"persistent sweep ({tune_sw['branches']} lanes)")
    ms = sw["ms"]
    plans = [op.plan(c) for c in range(nchan)]
    bv = 8 if args.store == "f32" else 4
    nbins_active = sum(int((op.bin_rows(c) > 0).sum()) for c in range(nchan))
    gbytes = sum(bv * p["ntaps"] + 8 * p["nrows"] + 32 * p["nwork"] for p in plans)
    fbytes = nbins_active * fft_bytes_per_bin(obs.nx, obs.ny)
    achieved = (gbytes + fbytes) / (ms * 1e-3) / 1e9
    line = {
        "metric": "\u03a6\u2020\u03a6 sweeps/s and p50/p99 per-channel latency "
                  "(16 \u00d7 2048\u00b2, 48M vis)",
        "value": 1e3 / ms, "unit": "sweeps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": DTYPE[args.store],
        "data": "synthetic",
        "config": {"workload": f"Re{{Phi^dag Phi x}} sweep over {nchan} channels "
                               f"0.9-1.67 GHz, {obs.nx}^2 image each, {M} visibilities "
                               f"(uneven per channel), 3 deg field",
                   "store": args.store, "nchan": nchan, "nvis": M,
                   "nbins": [p["nbins"] for p in plans]},
        "latency_ms": sw["latency_ms"],
        "graph": {"kernel_nodes": sw["kernels"], "nodes": sw["nodes"],
                  "lanes": tune_sw["branches"]},
        "sweep_autotune": tune_sw,
        "gvis_per_s": 1e3 / ms * M / 1e9,
        "sweep_build_s": t_sw, "eager_ms_sweep": eager_sweep,
        "branch_graph": {"ms": br["ms"], "kernel_nodes": br["kernels"], "nodes": br["nodes"],
                         "latency_ms": br["latency_ms"], "branches": tune["branches"]},
        "eager_ms_default_branches": eager_before, "eager_ms_one_branch": serial,
        "speedup_vs_branch_graph": br["ms"] / ms,
        "autotune": tune, "graph_vs_eager_rel": sw["rel"], "build_s": tb,
        "roofline": {"bound": "hbm", "kernel": "whole sweep (all kernels)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "bytes_per_sweep": gbytes + fbytes},
    }
    print(json.dumps(line), flush=True)


def counters_run(args, torch):
    """Counter-collection run (under rocprofv3 --pmc): a plain 1 GiB device copy for
    calibrating the byte counters, then exactly one Re{Phi^dag Phi} apply of the precision
    form per storage form (one branch, default work items), so that the fused kernel's
    counters summed over the run and divided by P are the bytes of one launch per bin."""
    import wfsynth as ws
    from paper_2605_26347_amd import Operator
    a = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    torch.cuda.empty_cache()
    obs = ws.precision_form(n=args.n, nvis=args.nvis, fov_deg=args.fov)
    x = torch.from_numpy(obs.sky.astype(np.float32)[None]).to("cuda:0")
    for f in args.forms.split(","):
        op = Operator(obs.uvw_m, obs.freqs_hz, obs.nx, obs.ny, obs.cell_rad,
                      memory_budget=args.budget, store=f)
        out = op.psf_apply_re(x)
        torch.cuda.synchronize()
        log(f"counters: {f} P={op.plan(0)['nbins']} one apply done")
        op.close()
        del op, out
        torch.cuda.empty_cache()


def bench_holographic(args, torch):
    """Holographic strategy where it pays: the central 512^2 of the precision form
    (same cell, 0.375 degree field) with all 50M visibilities, ~48 per grid cell.
    Phi^dag Phi with the stencils of H_p = G_p^dag G_p against the fused G^dag G."""
    import wfsynth as ws
    from paper_2605_26347_amd import Operator
    full = ws.precision_form(n=4096, nvis=args.nvis, fov_deg=args.fov, sky=False)
    n = 512
    cell = full.cell_rad
    M = full.uvw_m.shape[0]
    x = torch.from_numpy(ws.gauss_image(n, 4).astype(np.float32)[None]).to("cuda:0")
    res = {}
    for strat in ("G", "H"):
        t0 = time.time()
        op = Operator(full.uvw_m, full.freqs_hz, n, n, cell, memory_budget=args.budget,
                      store=args.store, strategy=strat)
        torch.cuda.synchronize()
        tb = time.time() - t0
        info = op.plan(0)
        out = torch.empty_like(x)
        for _ in range(args.warmup):
            op.psf_apply_re(x, out)
        op.profile_enable(0, True)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(args.steps):
            op.psf_apply_re(x, out)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        nl, kms = op.profile_read(0)
        op.profile_enable(0, False)
        byts = info["mem_h_bytes"] if strat == "H" else info["mem_g_bytes"]
        res[strat] = dict(ms=ms, build_s=tb, nbins=info["nbins"], bytes=byts,
                          kernel_ms=kms / max(args.steps, 1), out=out.clone())
        log(f"{strat}: P={info['nbins']} built {tb:.1f} s, {byts / 1e9:.2f} GB, "
            f"{ms:.3f} ms/apply (G^dag G or H part {kms / max(args.steps, 1):.3f} ms)")
        op.close()
        del op
        torch.cuda.empty_cache()
    d = float((res["H"]["out"] - res["G"]["out"]).norm() / res["G"]["out"].norm())
    kh = res["H"]["kernel_ms"]
    line = {
        "metric": "Φ†Φ applies/s with the holographic H vs the fused G†G (512² crop of the "
                  "4096² / 3° field, 50M vis)",
        "value": 1e3 / res["H"]["ms"], "unit": "applies/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": res["H"]["ms"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"Re{{Phi^dag Phi x}}, {n}^2 image at the 4096^2 / 3 deg cell, "
                               f"{M} visibilities", "store": args.store,
                   "nbins": res["H"]["nbins"]},
        "G": {k: v for k, v in res["G"].items() if k != "out"},
        "H": {k: v for k, v in res["H"].items() if k != "out"},
        "speedup_H_vs_G": res["G"]["ms"] / res["H"]["ms"],
        "H_vs_G_rel": d,
        "roofline": {"bound": "hbm", "kernel": "k_happly (H stencils)",
                     "achieved": res["H"]["bytes"] / (kh * 1e-3) / 1e9 if kh > 0 else None,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": (res["H"]["bytes"] / (kh * 1e-3) / 1e9 / HBM_PEAK_GBS)
                     if kh > 0 else None, "traffic": None},
    }
    print(json.dumps(line), flush=True)


def _timed_applies(op, x, out, n, torch):
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(n):
        op.psf_apply_re(x, out)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / n


def bench_onthefly(args, torch):
    """Strategy (c) on the precision form: no G is stored.  Factorised form (the value):
    the build stores each row's thresholded residual kernel and every apply convolves it
    with the row's Kaiser-Bessel taps, chunk by chunk, before the fused kernel applies
    the chunk.  Rebuilt form: every apply repeats the FP64 value pass of the build.  Both
    compared with the stored-G operator (same P) for time and result."""
    import wfsynth as ws
    from paper_2605_26347_amd import Operator
    obs = ws.precision_form(n=args.n, nvis=args.nvis, fov_deg=args.fov)
    M = obs.uvw_m.shape[0]
    x = torch.from_numpy(obs.sky.astype(np.float32)[None]).to("cuda:0")
    steps, warm = max(1, min(args.steps, 5)), max(1, min(args.warmup, 2))
    b_v = 8 if args.store == "f32" else 4

    def run(form, nsteps):
        t0 = time.time()
        op = Operator(obs.uvw_m, obs.freqs_hz, obs.nx, obs.ny, obs.cell_rad,
                      memory_budget=args.budget, store=args.store, strategy="otf",
                      otf_form=form)
        tb = time.time() - t0
        info = op.plan(0)
        log(f"on the fly, {form}: built in {tb:.1f} s, P={info['nbins']}, row data "
            f"{info['mem_g_bytes'] / 1e9:.2f} GB (kernels {info['mem_khat_bytes'] / 1e9:.2f} "
            f"GB), transient {info['mem_transient_bytes'] / 1e9:.2f} GB per branch, value "
            f"pass {info['value_pass_flops'] / 1e12:.3f} TFLOP per apply")
        out = torch.empty_like(x)
        # the autotuner picks rows per item and the branch count (each branch has its own
        # transient buffer: one bin's expansion overlaps another's fused kernel and FFTs)
        tune = op.autotune(x, out, reps=1)
        log(f"on the fly, {form}: autotune {tune}")
        for _ in range(warm):
            op.psf_apply_re(x, out)
        ms = _timed_applies(op, x, out, nsteps, torch)
        op.set_branches(1)
        op.profile_enable(5, True)
        op.profile_enable(0, True)
        op.psf_apply_re(x, out)
        n5, ms5 = op.profile_read(5)
        n0, ms0 = op.profile_read(0)
        op.profile_enable(5, False)
        op.profile_enable(0, False)
        log(f"on the fly, {form}: {ms:.1f} ms/apply on {tune['branches']} branches; value pass "
            f"{ms5:.1f} ms in {n5} launches, G^dag G {ms0:.1f} ms in {n0} launches (one branch)")
        res = out.clone()
        op.close()
        del op
        torch.cuda.empty_cache()
        return dict(build_s=tb, ms=ms, value_pass_ms=ms5, value_pass_launches=n5,
                    gtg_ms=ms0, branches=tune["branches"], info=info), res

    fac, fout = run("factorised", steps)
    reb, rout = run("rebuilt", 1)
    info = fac["info"]
    g = Operator(obs.uvw_m, obs.freqs_hz, obs.nx, obs.ny, obs.cell_rad,
                 memory_budget=args.budget, store=args.store, nbins=info["nbins"])
    gout = torch.empty_like(x)
    for _ in range(warm):
        g.psf_apply_re(x, gout)
    gms = _timed_applies(g, x, gout, steps, torch)
    gbytes = g.plan(0)["mem_g_bytes"]
    df = float((fout - gout).norm() / gout.norm())
    dr = float((rout - gout).norm() / gout.norm())
    log(f"stored G ({gbytes / 1e9:.1f} GB): {gms:.1f} ms/apply; vs stored: factorised "
        f"{df:.2e}, rebuilt {dr:.2e}; factorised {reb['ms'] / fac['ms']:.1f}x faster than "
        f"rebuilt")
    g.close()
    # expansion traffic per apply: the kernels read (b_v n'^2 per row), G written
    # (b_v T^2 per row), and per row its 2J FP32 taps (56 B at J = 7) and five 32-bit
    # words (list entry, patch word, kernel offset, item, value offset)
    J = 7
    kvals = (info["mem_khat_bytes"] - (4.0 + 8.0 * J) * M) / b_v
    xbytes = b_v * (kvals + info["ntaps"]) + (8.0 * J + 20.0) * M
    ach = xbytes / (fac["value_pass_ms"] * 1e-3) / 1e9 if fac["value_pass_ms"] > 0 else None
    ms = fac["ms"]
    strip = lambda d: {k: v for k, v in d.items() if k != "info"}
    line = {
        "metric": "Φ†Φ applies/s with G computed on the fly (strategy (c)), 4096², 50M vis",
        "value": 1e3 / ms, "unit": "applies/s", "n_gpus": 1, "steps": steps, "warmup": warm,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"Re{{Phi^dag Phi x}}, {obs.nx}^2 image, {M} visibilities, "
                               f"3 deg field, G expanded from stored kernels at every apply",
                   "store": args.store, "nbins": info["nbins"],
                   "strategy": "on the fly, factorised"},
        "factorised": strip(fac), "rebuilt": strip(reb),
        "kernel_bytes": info["mem_khat_bytes"], "row_data_bytes": info["mem_g_bytes"],
        "transient_bytes_per_branch": info["mem_transient_bytes"],
        "stored_G": {"ms": gms, "bytes": gbytes},
        "factorised_vs_stored_rel": df, "rebuilt_vs_stored_rel": dr,
        "factorised_speedup_vs_rebuilt": reb["ms"] / ms,
        "roofline": {"bound": "hbm", "kernel": "k_expand (all classes, per apply)",
                     "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": ach / HBM_PEAK_GBS if ach else None, "traffic": None,
                     "bytes_per_apply": xbytes,
                     "bytes": "b_v (n'^2 + T^2) + 8 J + 20 per row: kernel read, G written, "
                              "taps and row words"},
    }
    print(json.dumps(line), flush=True)


def bench_weighted(args, torch):
    """Data weighting and flags in G (Sect. 2) on the precision form: Briggs robust
    weights (R = 0) from log-normal noise levels, 10% of the rows flagged in runs, both
    folded into the stored G; timed like the precision form."""
    import wfsynth as ws
    from paper_2605_26347_amd import Operator, briggs_weights
    obs = ws.precision_form(n=args.n, nvis=args.nvis, fov_deg=args.fov)
    M = obs.uvw_m.shape[0]
    sigma = ws.noise_sigma(M)
    flags = ws.flag_runs(M, 0.1)
    nat = (1.0 / sigma.astype(np.float64) ** 2).astype(np.float32)
    torch.cuda.synchronize()
    t0 = time.time()
    w = briggs_weights(obs.uvw_m, obs.freqs_hz, obs.nx, obs.ny, obs.cell_rad, 0.0,
                       natural=nat, flags=flags)
    tw = time.time() - t0
    w = (w / w.max()).astype(np.float32)
    log(f"Briggs weights of {M} rows in {tw:.2f} s (host arrays in and out)")
    t0 = time.time()
    op = Operator(obs.uvw_m, obs.freqs_hz, obs.nx, obs.ny, obs.cell_rad,
                  memory_budget=args.budget, store=args.store, weights=w, flags=flags)
    tb = time.time() - t0
    info = op.plan(0)
    x = torch.from_numpy(obs.sky.astype(np.float32)[None]).to("cuda:0")
    out = torch.empty_like(x)
    tune = op.autotune(x, out, reps=2)
    for _ in range(args.warmup):
        op.psf_apply_re(x, out)
    ms = _timed_applies(op, x, out, args.steps, torch)
    op.set_branches(1)
    for _ in range(args.warmup):
        op.psf_apply_re(x, out)
    op.profile_enable(0, True)
    for _ in range(args.steps):
        op.psf_apply_re(x, out)
    nl, kms = op.profile_read(0)
    op.profile_enable(0, False)
    kl = kms / max(nl, 1)
    P = info["nbins"]
    per_launch = gtg_bytes(info, args.store) / max(P, 1)
    ach = per_launch / (kl * 1e-3) / 1e9
    log(f"weighted: built {tb:.1f} s, P={P}, {info['nrows']} rows kept, {ms:.3f} ms/apply, "
        f"G^dag G {kl:.3f} ms/launch")
    line = {
        "metric": "Φ†Φ applies/s with Briggs weights and 10% flags in G (4096², 50M vis)",
        "value": 1e3 / ms, "unit": "applies/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"Re{{Phi^dag Phi x}}, {obs.nx}^2 image, {M} visibilities, "
                               f"Briggs R=0, 10% flagged", "store": args.store, "nbins": P},
        "briggs_s": tw, "build_s": tb, "rows_kept": info["nrows"],
        "rows_flagged": info["nflagged"], "autotune": tune,
        "roofline": {"bound": "hbm", "kernel": "fused G^dag G (k_gtg)", "achieved": ach,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                     "traffic": None, "bytes_per_launch": per_launch, "ms_per_launch": kl},
    }
    op.close()
    print(json.dumps(line), flush=True)


def bench_learned(args, torch):
    """Learned form: the residual-kernel network trained on 1M exact kernels (residual w
    of the 64-antenna array binned at 16 bins, fields of 1-4 degrees), then G of 20M rows
    on a 4096^2 / 3 degree image with 16 bins built with the network (exact fallback where
    its predicted error exceeds 1e-3 or the kernel side exceeds 15) and without it."""
    import wfsynth as ws
    from paper_2605_26347_amd import Network, Operator
    t0 = time.time()
    obs = ws.learned_form()
    M = obs.uvw_m.shape[0]
    log(f"inputs: {M} rows, {obs.nx}^2, {time.time() - t0:.1f} s")
    mk = dict(memory_budget=args.budget, nbins=16, store="f32")
    torch.cuda.synchronize()
    t0 = time.time()
    op_e = Operator(obs.uvw_m, obs.freqs_hz, obs.nx, obs.ny, obs.cell_rad, **mk)
    torch.cuda.synchronize()
    t_exact = time.time() - t0
    pe = op_e.plan(0)
    cents = op_e.centroids(0)
    w = obs.uvw_m[:, 2] * (obs.freqs_hz[0] / 299792458.0)
    wp = w - cents[np.searchsorted(0.5 * (cents[1:] + cents[:-1]), w, side="left")]
    w_, L_, fu_, fv_ = ws.kernel_examples(wp, args.train_examples)
    dev = [torch.from_numpy(a).to("cuda:0") for a in (w_, L_, fu_, fv_)]
    t0 = time.time()
    x, nk = Network.inputs(*dev)
    t = Network.targets(dev[0], dev[1])
    keep = (nk <= 15).nonzero().squeeze(1)
    x, t = x[keep].contiguous(), t[keep].contiguous()
    torch.cuda.synchronize()
    t_targets = time.time() - t0
    net = Network(seed=5)
    t0 = time.time()
    hist = net.train(x, t, batch=4096, epochs=args.epochs, lr0=2e-3, lr_end=1e-6, seed=3)
    torch.cuda.synchronize()
    t_train = time.time() - t0
    log(f"training: {x.shape[0]} kernels (of {args.train_examples}) in {t_train:.1f} s "
        f"(targets {t_targets:.2f} s); kernel loss {hist[0, 0]:.2e} -> {hist[-1, 0]:.2e}")
    # held-out accuracy of the network itself
    hv = ws.kernel_examples(wp, 100_000, seed=99)
    hd = [torch.from_numpy(a).to("cuda:0") for a in hv]
    xv, nkv = Network.inputs(*hd)
    tv = Network.targets(hd[0], hd[1])
    kv = (nkv <= 15).nonzero().squeeze(1)
    pv = net.infer(xv[kv].contiguous(), bf16=2)
    ev = ((pv[:, :450] - tv[kv]).norm(dim=1) / tv[kv].norm(dim=1)).cpu().numpy()
    torch.cuda.synchronize()
    t0 = time.time()
    op_s = Operator(obs.uvw_m, obs.freqs_hz, obs.nx, obs.ny, obs.cell_rad, surrogate=net,
                    surrogate_tol=1e-3, **mk)
    torch.cuda.synchronize()
    t_sur = time.time() - t0
    ps = op_s.plan(0)
    xs = torch.from_numpy(obs.sky.astype(np.float32)[None]).to("cuda:0")
    ref = op_e.psf_apply(xs)
    got = op_s.psf_apply(xs)
    err = float((got - ref).norm() / ref.norm())
    # against the FP64 oracle (exact kernels): its Phi^dag Phi of the N(0,1) probe at the
    # stored pixel samples (tests/golden/learned_4096sq_2M.npz, written by a script that
    # calls only the oracle) for a seeded 2M-row subset of these rows, P = 16 and the
    # oracle's centroids
    vs_oracle = None
    fxp = os.path.join(ROOT, "tests", "golden", "learned_4096sq_2M.npz")
    if os.path.exists(fxp):
        fx = np.load(fxp)
        sub = np.ascontiguousarray(obs.uvw_m[ws.seeded_subset(M, 2_000_000, 3)])
        xg = torch.from_numpy(ws.gauss_image(obs.nx, 4).astype(np.float32)[None]).to("cuda:0")
        pix = torch.from_numpy(fx["pix"]).to("cuda:0")
        vs_oracle = {}
        for name, kw in (("network", {"surrogate": net}), ("exact", {})):
            for strat, form in (("G", "auto"), ("otf", "factorised"), ("otf", "rebuilt")):
                o = Operator(sub, obs.freqs_hz, obs.nx, obs.ny, obs.cell_rad, nbins=16,
                             store="f32", strategy=strat, otf_form=form, **kw)
                assert np.allclose(o.centroids(0), fx["centroids"], rtol=1e-12, atol=1e-9)
                v = o.psf_apply(xg)[0].flatten()[pix].cpu().numpy()
                key = f"{name}_{strat}" + ("" if strat == "G" else f"_{form}")
                vs_oracle[key] = float(np.linalg.norm(v - fx["psf"]) / np.linalg.norm(fx["psf"]))
                o.close()
                del o
                torch.cuda.empty_cache()
        log(f"Phi^dag Phi vs FP64 oracle (2M-row subset, 32768 pixels): {vs_oracle}")
    # strategy (c), rebuilt form: kernels rebuilt at every apply, with and without the
    # network (the factorised form stores them, so the network acts at its build only)
    otf = {}
    for name, kw in (("exact", {}), ("network", {"surrogate": net})):
        o = Operator(obs.uvw_m, obs.freqs_hz, obs.nx, obs.ny, obs.cell_rad, strategy="otf",
                     otf_form="rebuilt", **{**mk, "store": "f16"}, **kw)
        out = o.psf_apply_re(xs)
        torch.cuda.synchronize()
        o.profile_enable(5, True)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(3):
            o.psf_apply_re(xs, out)
        e1.record()
        torch.cuda.synchronize()
        _, vp = o.profile_read(5)
        otf[name] = {"apply_ms": e0.elapsed_time(e1) / 3, "value_pass_ms": vp / 3,
                     "network_rows": o.plan(0)["surrogate_fraction"]}
        o.close()
        del o
        torch.cuda.empty_cache()
    log(f"strategy (c): {otf}")
    log(f"build: exact {t_exact:.2f} s (channel {pe['build_seconds']:.2f} s), network "
        f"{t_sur:.2f} s (channel {ps['build_seconds']:.2f} s); network rows "
        f"{ps['surrogate_fraction']:.3f}; Phi^dag Phi rel vs exact {err:.2e}")
    line = {
        "metric": "G build time, 4096² / 20M vis / 16 bins: residual-kernel network + exact "
                  "fallback vs exact",
        "value": ps["build_seconds"], "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": 1e3 * ps["build_seconds"], "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"G of {M} visibilities, {obs.nx}^2 image, 3 deg field, "
                               f"16 w-bins, FP32 values", "nvis": M, "nbins": 16},
        "build_s": {"exact": pe["build_seconds"], "network": ps["build_seconds"],
                    "exact_wall": t_exact, "network_wall": t_sur},
        "network_rows": ps["surrogate_fraction"],
        "fallback_fraction": 1.0 - ps["surrogate_fraction"],
        "psf_rel_vs_exact": err,
        "psf_rel_vs_fp64_oracle": vs_oracle,
        "onthefly": otf,
        "onthefly_value_pass_gain": otf["exact"]["value_pass_ms"] / otf["network"]["value_pass_ms"],
        "train": {"examples": int(x.shape[0]), "epochs": args.epochs, "seconds": t_train,
                  "kernel_loss_first": float(hist[0, 0]), "kernel_loss_last": float(hist[-1, 0])},
        "heldout_rel_err": {"p50": float(np.median(ev)), "p90": float(np.percentile(ev, 90)),
                            "p99": float(np.percentile(ev, 99))},
    }
    print(json.dumps(line), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the operator "
              "shards by w-bin across GPUs only in design", file=sys.stderr)
        sys.exit(2)
    import torch
    import wfsynth as ws
    if args.workload == "cpu":
        bench_cpu(args)
        return
    if args.workload == "batched":
        bench_batched(args, torch)
        return
    if args.workload == "learned":
        bench_learned(args, torch)
        return
    if args.workload == "holographic":
        bench_holographic(args, torch)
        return
    if args.workload == "counters":
        counters_run(args, torch)
        return
    if args.workload == "onthefly":
        bench_onthefly(args, torch)
        return
    if args.workload == "weighted":
        bench_weighted(args, torch)
        return
    t0 = time.time()
    obs = ws.precision_form(n=args.n, nvis=args.nvis, fov_deg=args.fov)
    log(f"inputs: {obs.uvw_m.shape[0]} rows, {obs.nx}^2 image, {time.time() - t0:.1f} s")
    forms = args.forms.split(",")
    if args.calib_copy:
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        bcopy = torch.empty_like(a)
        bcopy.copy_(a)
        torch.cuda.synchronize()
        log("calibration copy: 1 GiB read + 1 GiB written")
        del a, bcopy
        torch.cuda.empty_cache()
    res = {}
    for f in forms:
        res[f] = time_form(obs, f, args, torch)
    head = res[forms[0]]
    M = obs.uvw_m.shape[0]
    aps = 1e3 / head["ms"]
    for r in res.values():
        r.pop("out", None)
    torch.cuda.empty_cache()
    acc = {"vs_fp64_oracle": accuracy_vs_oracle(["f32", "f16", "bf16"], torch),
           "samples": "32768 seeded pixels of Phi^dag Phi x per case"}
    nl = head["gtg_launches"]
    kms = head["gtg_ms_total"] / max(nl, 1)
    bytes_per_apply = gtg_bytes(head["info"], head["store"])
    P = head["info"]["nbins"]
    per_launch = bytes_per_apply / max(P, 1)
    achieved = per_launch / (kms * 1e-3) / 1e9
    traffic = measured_traffic(head["store"])
    line = {
        "metric": METRIC, "value": aps, "unit": "applies/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPE[head["store"]], "data": "synthetic",
        "config": {"workload": f"Re{{Phi^dag Phi x}}, {obs.nx}^2 image, {M} visibilities, "
                               f"3 deg field, 64-antenna array 16 h, 1.28 GHz",
                   "store": head["store"], "nbins": P, "image": obs.nx, "nvis": M},
        "gvis_per_s": aps * M / 1e9,
        "forms": {f: {"ms": r["ms"], "applies_per_s": 1e3 / r["ms"],
                      "gvis_per_s": 1e3 / r["ms"] * M / 1e9, "nbins": r["info"]["nbins"],
                      "ntaps": r["info"]["ntaps"], "build_s": r["build_s"],
                      "g_bytes": r["info"]["mem_g_bytes"], "forward_ms": r["fwd_ms"],
                      "adjoint_ms": r["adj_ms"]} for f, r in res.items()},
        "accuracy": acc,
        "autotune": head["tune"],
        "fb_iteration_ms": head.get("fb_ms"),
        "roofline": {"bound": "hbm", "kernel": "fused G^dag G (k_gtg)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "bytes_per_launch": per_launch, "ms_per_launch": kms,
                     "timed": "one branch, HIP events around each launch on its stream",
                     "share_of_step": kms * P / head["ms"]},
    }
    # whole apply: G's bytes plus the four FFT passes of every layer
    e2e = (bytes_per_apply + P * fft_bytes_per_bin(obs.nx, obs.ny)) / (head["ms"] * 1e-3) / 1e9
    line["end_to_end"] = {"achieved": e2e, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": e2e / HBM_PEAK_GBS,
                          "bytes_per_apply": bytes_per_apply
                          + P * fft_bytes_per_bin(obs.nx, obs.ny)}
    if "f32" in res and forms[0] != "f32":
        line["speedup_mixed_vs_f32"] = res["f32"]["ms"] / head["ms"]
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(obs, P)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
