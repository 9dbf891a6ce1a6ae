"""Shared helpers of the GPU parity tests: build the HIP operator and the FP64 oracle
on the same seeded inputs."""
import numpy as np

from oracle import OracleOperator, OperatorParams

TOL = {"f32": 1e-5, "f16": 1e-3, "bf16": 5e-3}


def rel(a, b):
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def oracle_for(obs, nbins, chan=0, uvw=None, **kw):
    prm = OperatorParams(obs.nx, obs.ny, obs.cell_rad,
                         J=kw.get("J", 7), beta=kw.get("beta", 2.34 * kw.get("J", 7)),
                         alpha=kw.get("alpha", 2.0), smax=kw.get("smax", 31),
                         eps=kw.get("eps_w", 1e-6))
    u = obs.uvw_m if uvw is None else uvw
    return OracleOperator(u, obs.freqs_hz[chan], prm, nbins=nbins, seed=kw.get("seed", 0),
                          plan_fraction=kw.get("plan_fraction", 0.01),
                          weights=kw.get("weights"), flags=kw.get("flags"))


def gpu_operator(obs, nbins, **kw):
    from paper_2605_26347_amd import Operator
    return Operator(obs.uvw_m, obs.freqs_hz, obs.nx, obs.ny, obs.cell_rad, nbins=nbins,
                    chan_rows=obs.chan_rows, **kw)


def to_dev(x, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda:0")
