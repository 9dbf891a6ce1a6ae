"""Pins of the oracle's data weighting and flags (Sect. 2: a weighting scheme injected in
the measurement operator; a flag vector marking measurements to discard) and of its
Briggs robust weights (published definition, Briggs 1995), no GPU."""
import numpy as np
import pytest

import wfsynth as ws
from oracle import OracleOperator, OperatorParams, direct_forward, direct_adjoint
from oracle.operator import C_LIGHT
from oracle import weighting as wt


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


@pytest.fixture(scope="module")
def small():
    obs = ws.tiny(n=24, nant=10, nsteps=30, fov_deg=5.0)
    prm = OperatorParams(24, 24, obs.cell_rad)
    r = np.random.default_rng(41)
    M = obs.uvw_m.shape[0]
    omega = r.uniform(0.2, 3.0, M)
    flags = r.random(M) < 0.2
    return obs, prm, omega, flags


def test_weighted_forward_matches_weighted_direct_sum():
    """One bin, no residual kernel, w replaced by the bin centre: w-stacking is exact
    algebra, so the weighted operator must equal omega times the direct sum."""
    obs = ws.tiny()
    prm = OperatorParams(obs.nx, obs.ny, obs.cell_rad, smax=1)
    M = obs.uvw_m.shape[0]
    omega = np.random.default_rng(42).uniform(0.1, 2.0, M)
    op = OracleOperator(obs.uvw_m, obs.freqs_hz[0], prm, nbins=1, weights=omega)
    uvw = obs.uvw_m * (obs.freqs_hz[0] / C_LIGHT)
    uvw[:, 2] = op.centroids[0]
    x = obs.sky
    assert rel(op.forward(x), omega * direct_forward(x, uvw, obs.cell_rad)) <= 1e-5
    y = np.random.default_rng(43).standard_normal(M) + 0j
    assert rel(op.adjoint(y),
               direct_adjoint(omega * y, uvw, obs.nx, obs.ny, obs.cell_rad)) <= 1e-5


def test_weights_scale_rows(small):
    obs, prm, omega, _ = small
    plain = OracleOperator(obs.uvw_m, obs.freqs_hz[0], prm, nbins=3)
    wop = OracleOperator(obs.uvw_m, obs.freqs_hz[0], prm, nbins=3, weights=omega)
    r = np.random.default_rng(44)
    x = r.standard_normal((24, 24))
    y = r.standard_normal(plain.M) + 1j * r.standard_normal(plain.M)
    assert rel(wop.forward(x), omega * plain.forward(x)) <= 1e-13
    assert rel(wop.adjoint(y), plain.adjoint(omega * y)) <= 1e-13
    assert rel(wop.psf(x), plain.adjoint(omega ** 2 * plain.forward(x))) <= 1e-13
    assert rel(wop.psf_via_H(x), wop.psf(x)) <= 1e-12
    fx = wop.forward(x)
    a = np.vdot(y, fx)
    b = np.vdot(wop.adjoint(y), x)
    assert abs(a - b) <= 1e-12 * np.linalg.norm(fx) * np.linalg.norm(y)


def test_flags_discard_rows_before_planning(small):
    """Flagging a row is the same as never having it: same bins, same values on the kept
    rows, zero forward value on flagged rows, flagged data ignored by the adjoint."""
    obs, prm, omega, flags = small
    keep = ~flags
    fop = OracleOperator(obs.uvw_m, obs.freqs_hz[0], prm, nbins=3, weights=omega,
                         flags=flags, plan_fraction=0.5)
    sub = OracleOperator(obs.uvw_m[keep], obs.freqs_hz[0], prm, nbins=3,
                         weights=omega[keep], plan_fraction=0.5)
    assert np.array_equal(fop.centroids, sub.centroids)
    r = np.random.default_rng(45)
    x = r.standard_normal((24, 24))
    y = fop.forward(x)
    assert y.shape == (obs.uvw_m.shape[0],)
    assert np.all(y[flags] == 0)
    assert np.array_equal(y[keep], sub.forward(x))
    yv = r.standard_normal(y.size) + 1j * r.standard_normal(y.size)
    yz = yv.copy()
    yz[flags] = 1e6
    assert np.array_equal(fop.adjoint(yz), sub.adjoint(yv[keep]))
    assert np.array_equal(fop.psf(x), sub.psf(x))


# ------------------------------------------------------------------ Briggs weights

def test_briggs_hand_example():
    """Three samples on a 4 x 4 Fourier grid with unit cells (cell = 1/4), natural
    weights (1, 2, 1), R = 0.  Cells (with the conjugate of each sample):
    s1 (0.1, 0.2) -> (0, 0), conj -> (0, 0); s2 (1.2, 0) -> (1, 0), conj -> (3, 0);
    s3 (0.9, 0.1) -> (1, 0), conj -> (3, 0).  Densities W(0,0) = 2, W(1,0) = W(3,0) = 3;
    sum w W = 1*2 + 2*3 + 1*3 = 11, sum w = 4, f^2 = 25 * 4 / 11 = 100/11;
    w' = (1 / (1 + 200/11), 2 / (1 + 300/11), 1 / (1 + 300/11)) = (11/211, 22/311, 11/311)."""
    u = np.array([0.1, 1.2, 0.9])
    v = np.array([0.2, 0.0, 0.1])
    got = wt.briggs(u, v, 4, 4, 0.25, 0.0, natural=np.array([1.0, 2.0, 1.0]))
    assert np.allclose(got, [11 / 211, 22 / 311, 11 / 311], rtol=1e-14, atol=0)


def briggs_case(seed=46, M=3000, n=32):
    r = np.random.default_rng(seed)
    cell = 1e-3
    span = 0.5 / cell
    u = r.normal(0, span / 4, M)
    v = r.normal(0, span / 4, M)
    nat = r.uniform(0.5, 2.0, M)
    return u, v, n, cell, nat


def my_cells(u, v, n, cell):
    iu = np.floor(u * n * cell + 0.5).astype(np.int64) % n
    iv = np.floor(v * n * cell + 0.5).astype(np.int64) % n
    return iv * n + iu


def test_briggs_natural_and_uniform_limits():
    u, v, n, cell, nat = briggs_case()
    w_nat = wt.briggs(u, v, n, n, cell, 12.0, natural=nat)
    assert np.allclose(w_nat, nat, rtol=1e-12, atol=0)
    # uniform limit: every occupied cell carries the same total weight (each sample
    # counted at its own cell and at its conjugate's)
    w_uni = wt.briggs(u, v, n, n, cell, -12.0, natural=nat)
    tot = np.zeros(n * n)
    np.add.at(tot, my_cells(u, v, n, cell), w_uni)
    np.add.at(tot, my_cells(-u, -v, n, cell), w_uni)
    occ = tot[tot > 0]
    assert occ.size > 50
    assert np.allclose(occ, occ.mean(), rtol=1e-9, atol=0)


def test_briggs_monotone_symmetric_and_flags():
    u, v, n, cell, nat = briggs_case(47)
    ws_ = [wt.briggs(u, v, n, n, cell, R, natural=nat) for R in (-2.0, -0.5, 0.0, 0.5, 2.0)]
    for a, b in zip(ws_, ws_[1:]):
        assert np.all(a <= b) and np.any(a < b)
    assert np.all(ws_[2] <= nat)
    # conjugating every sample, or permuting them, changes nothing
    assert np.allclose(wt.briggs(-u, -v, n, n, cell, 0.0, natural=nat), ws_[2], rtol=1e-13)
    perm = np.random.default_rng(48).permutation(u.size)
    assert np.allclose(wt.briggs(u[perm], v[perm], n, n, cell, 0.0, natural=nat[perm]),
                       ws_[2][perm], rtol=1e-13)
    # flagged samples get zero and leave the others as if absent
    flags = np.random.default_rng(49).random(u.size) < 0.3
    wf = wt.briggs(u, v, n, n, cell, 0.0, natural=nat, flags=flags)
    assert np.all(wf[flags] == 0)
    ws_sub = wt.briggs(u[~flags], v[~flags], n, n, cell, 0.0, natural=nat[~flags])
    assert np.allclose(wf[~flags], ws_sub, rtol=1e-13)
    # within one cell, the weight over the natural weight is the same for every sample,
    # and it falls as the cell's density grows
    ratio = ws_[2] / nat
    c = my_cells(u, v, n, cell)
    for cc in np.unique(c)[:20]:
        sel = c == cc
        assert np.ptp(ratio[sel]) <= 1e-13 * ratio[sel].max()
    W = np.zeros(n * n)
    np.add.at(W, c, nat)
    np.add.at(W, my_cells(-u, -v, n, cell), nat)
    order = np.argsort(W[c])
    assert np.all(np.diff(ratio[order]) <= 1e-15)
