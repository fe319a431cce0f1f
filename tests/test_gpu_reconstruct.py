"""GPU parity of the reconstruction diagnostics (Section 3.2: the truncated series of
eq. (series) over the retained modes, the relative RMSE of eq. (alps_relative_rmse)
and both sides of Parseval's identity, eq. (spectral_variance)) against the FP64
oracle, through the C ABI (enufft_reconstruct).

The GPU's own coefficients and kept sets are the input on both sides, so the
comparison isolates the type-2 evaluation.  Tolerances: h_rec rel-l2 <= 5e-5 (FP32)
and <= 1e-10 (FP64); the sample sums follow from that bound (below); the spectral
sums are FP64 sums of the same coefficients (rel 1e-12); sigma^2_phys carries the
FP32 window evaluation (rel 1e-5)."""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_2606_21278_amd as enf
import synth
from helpers import gpu_batch, rel_l2

pytestmark = pytest.mark.gpu

TOL = {"f32": 5e-5, "f64": 1e-10}


def _oracle_inputs(gb):
    inp = oracle.batch_inputs(gb.to(device="cpu"))
    return inp


def _check_diag(dg, ref, hr, hr_ref, offsets, prec):
    """diag against the oracle's: exact counts; the error sums within what the measured
    h_rec deviation allows; the rest to FP rounding."""
    assert np.array_equal(dg[:, 0], ref[:, 0])
    for c in range(len(dg)):
        a, b = offsets[c], offsets[c + 1]
        if b == a:
            continue
        # |sum (t - r)^2 - sum (t - r')^2| <= 2 |t - r'| |r - r'| + |r - r'|^2 (Cauchy-Schwarz)
        d_ref = math.sqrt(ref[c, 1])
        dev = np.linalg.norm(hr[a:b] - hr_ref[a:b])
        assert abs(dg[c, 1] - ref[c, 1]) <= 2.0 * d_ref * dev + dev * dev + 1e-12 * ref[c, 2], c
    rt = 1e-5 if prec == "f32" else 1e-11
    assert np.allclose(dg[:, 2], ref[:, 2], rtol=rt, atol=0)
    assert np.allclose(dg[:, 3], ref[:, 3], rtol=rt, atol=0)
    assert np.allclose(dg[:, 4], ref[:, 4], rtol=1e-12, atol=0)
    assert np.allclose(dg[:, 5], ref[:, 5], rtol=1e-12, atol=0)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_reconstruct_matches_oracle(prec):
    b = synth.config1(count_scale=0.01, n_cells=24, precision=prec)
    gb = gpu_batch(b)
    area = synth.hexagon_area()
    plan = enf.Plan(gb.cell_offsets, gb.windows, n_modes=gb.n_modes, sigma=gb.sigma,
                    eps=1e-10 if prec == "f64" else 1e-5, precision=prec, scale=1.0 / area)
    f = plan.type1(gb.x, gb.y, gb.h, gb.w)
    keep, ks, st = plan.ems(f)
    areas = torch.full((gb.n_cells,), area, dtype=torch.float64, device="cuda:0")
    hr, dg = plan.reconstruct(gb.x, gb.y, gb.h, gb.w, f, keep, areas)
    hr_all, dg_all = plan.reconstruct(gb.x, gb.y, gb.h, gb.w, f)        # every mode, |D| = 1
    torch.cuda.synchronize()
    inp = _oracle_inputs(gb)
    fg = f.cpu().numpy().astype(np.complex128)
    kg = keep.cpu().numpy()
    hr_ref, ref = oracle.reconstruct(inp["offsets"], inp["x"], inp["y"], inp["h"], inp["w"], inp["windows"],
                                     inp["n_modes"], fg, keep=kg, area=np.full(gb.n_cells, area))
    hra_ref, refa = oracle.reconstruct(inp["offsets"], inp["x"], inp["y"], inp["h"], inp["w"], inp["windows"],
                                       inp["n_modes"], fg)
    hr, dg = hr.cpu().numpy().astype(np.float64), dg.cpu().numpy()
    hra, dga = hr_all.cpu().numpy().astype(np.float64), dg_all.cpu().numpy()
    e1, e2 = rel_l2(hr, hr_ref), rel_l2(hra, hra_ref)
    print("%s: h_rec rel-l2 kept %.2e all %.2e; eps_rel median %.3f, Parseval ratio median %.3f (all modes %.3f)"
          % (prec, e1, e2, np.median(ref[:, 6]), np.median(ref[:, 7]), np.median(refa[:, 7])), flush=True)
    assert e1 <= TOL[prec] and e2 <= TOL[prec]
    _check_diag(dg, ref, hr, hr_ref, inp["offsets"], prec)
    _check_diag(dga, refa, hra, hra_ref, inp["offsets"], prec)


def test_reconstruct_band_limited_grid_is_exact_on_gpu():
    """A zero-mean band-limited field on a regular 64 x 64 grid of the 2 pi box, uniform
    weights, no window, scale 1/|D|: the GPU reconstruction reproduces the samples
    (eps_rel at FP64 round-off) and the Parseval ratio is 1, as for the oracle."""
    n, N = 64, 32
    g = -math.pi + 2 * math.pi * np.arange(n) / n
    X, Y = np.meshgrid(g, g)
    x, y = X.ravel(), Y.ravel()
    rng = np.random.default_rng(5)
    h = np.zeros_like(x)
    for _ in range(12):
        kx, ky = rng.integers(-12, 13, 2)
        if kx or ky:
            h += rng.normal() * np.cos(kx * x + ky * y + rng.uniform(0, 2 * math.pi))
    Q = len(x)
    area = (2 * math.pi) ** 2
    t = lambda v: torch.as_tensor(v, dtype=torch.float64, device="cuda:0")
    plan = enf.Plan(np.array([0, Q]), None, n_modes=(N, N), eps=1e-12, precision="f64", window="none",
                    scale=1.0 / area)
    xs, ys, hs, ws = t(x), t(y), t(h), t(np.full(Q, area / Q))
    f = plan.type1(xs, ys, hs, ws)
    hr, dg = plan.reconstruct(xs, ys, hs, ws, f, area=t([area]))
    torch.cuda.synchronize()
    dg = dg.cpu().numpy()
    print("grid: eps_rel %.2e ratio %.15f" % (dg[0, 6], dg[0, 7]), flush=True)
    assert rel_l2(hr.cpu().numpy(), h) < 1e-10
    assert dg[0, 6] < 1e-10
    assert abs(dg[0, 7] - 1.0) < 1e-10


def test_reconstruct_edge_cases():
    """Empty cells and single-point cells; an all-zero keep gives h_rec = 0 and eps_rel = 1;
    arguments are checked."""
    b = synth.uniform_box(counts=[0, 1, 300, 0, 57], n_modes=(16, 16), precision="f64", window_radius=3.0)
    gb = gpu_batch(b)
    plan = enf.Plan(gb.cell_offsets, gb.windows, n_modes=gb.n_modes, eps=1e-10, precision="f64")
    f = plan.type1(gb.x, gb.y, gb.h, gb.w)
    zero = torch.zeros(f.shape, dtype=torch.uint8, device="cuda:0")
    hr, dg = plan.reconstruct(gb.x, gb.y, gb.h, gb.w, f, zero)
    torch.cuda.synchronize()
    dg = dg.cpu().numpy()
    assert torch.count_nonzero(hr).item() == 0
    assert list(dg[:, 0]) == [0, 1, 300, 0, 57]
    live = dg[:, 2] > 0          # cells with some windowed height
    assert np.all(dg[~live, 6] == 0.0) and live[2] and live[4]
    assert np.allclose(dg[live, 6], 1.0, rtol=1e-14)
    inp = _oracle_inputs(gb)
    hr_ref, ref = oracle.reconstruct(inp["offsets"], inp["x"], inp["y"], inp["h"], inp["w"], inp["windows"],
                                     inp["n_modes"], f.cpu().numpy())
    hr2, dg2 = plan.reconstruct(gb.x, gb.y, gb.h, gb.w, f)
    torch.cuda.synchronize()
    assert rel_l2(hr2.cpu().numpy(), hr_ref) <= TOL["f64"]
    with pytest.raises(ValueError):
        plan.reconstruct(gb.x, gb.y, gb.h, gb.w, f.to(torch.complex64))
    with pytest.raises(enf.EnufftError):     # the C ABI rejects a missing coefficient array
        enf._check(plan._lib.enufft_reconstruct(plan._h, enf._ptr(gb.x), enf._ptr(gb.y), enf._ptr(gb.h),
                                                enf._ptr(gb.w), None, None, None, None, enf._ptr(dg2)), plan._h)
