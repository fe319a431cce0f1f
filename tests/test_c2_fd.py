"""The differentiation workload: central finite differences of the retained power.

P_c = sum over the kept modes of |f_c[k]|^2 with the kept set frozen.  On 8 seeded
cells of the 256-hexagon batch (64 x 64 modes, lognormal counts, median 2e4) and 64
seeded points per cell, each of h, x and y is perturbed by +-1e-6 (times
max(1, |value|)) in FP64 and P is re-evaluated with the oracle's direct sums.
Only one point moves, so the perturbed coefficients are the unperturbed ones plus
the difference of that point's own direct sums (the oracle's type-1 on a one-point
cell): the same values as a full re-evaluation, without summing every other point
again.

CPU: the oracle's analytic gradient (direct type-2 sums) agrees with the
differences to 1e-8 relative l2 (about 1e-10 measured).  GPU: the FP32 adjoint through the C ABI agrees with
the same differences to 5e-5 relative l2 per component.
"""
import numpy as np
import pytest
import torch

import oracle
import synth

STEP = 1e-6


def _sub_points(inp, cells, pts):
    """Sampled points of the chosen cells as arrays (FP64), with their cell's window."""
    idx = np.concatenate([inp["offsets"][c] + np.sort(p) for c, p in zip(cells, pts)])
    win = np.repeat(np.asarray(inp["windows"])[cells], [len(p) for p in pts], axis=0)
    return idx, win


def _one_point_coeffs(x, y, h, w, win, n_modes, kind):
    """Each point's own coefficients: the oracle's type-1 with one point per cell."""
    n = len(x)
    off = np.arange(n + 1, dtype=np.int64)
    return oracle.type1(off, x, y, h, w, win, n_modes, kind=kind)


def fd_gradients(inp, cells, pts, keep):
    """Central differences of sum_c P_c with respect to h, x, y at the sampled points.
    keep: uint8 [len(cells), N2, N1], the frozen kept sets of the sampled cells."""
    n_modes, kind = inp["n_modes"], inp["kind"]
    sub_off = np.concatenate([[0], np.cumsum([inp["offsets"][c + 1] - inp["offsets"][c] for c in cells])])
    idx_all = np.concatenate([np.arange(inp["offsets"][c], inp["offsets"][c + 1]) for c in cells])
    f = oracle.type1(sub_off, inp["x"][idx_all], inp["y"][idx_all], inp["h"][idx_all], inp["w"][idx_all],
                     np.asarray(inp["windows"])[cells], n_modes, kind=kind)
    idx, win = _sub_points(inp, cells, pts)
    cell_of = np.repeat(np.arange(len(cells)), [len(p) for p in pts])
    x0, y0, h0, w0 = (inp[k][idx] for k in ("x", "y", "h", "w"))
    base = _one_point_coeffs(x0, y0, h0, w0, win, n_modes, kind)
    out = {}
    for name in ("h", "x", "y"):
        v0 = {"x": x0, "y": y0, "h": h0}[name]
        d = STEP * np.maximum(1.0, np.abs(v0))
        vals = {}
        for sgn in (1, -1):
            a = {"x": x0, "y": y0, "h": h0}
            a = {k: (v + sgn * d if k == name else v) for k, v in a.items()}
            vals[sgn] = _one_point_coeffs(a["x"], a["y"], a["h"], w0, win, n_modes, kind)
        g = np.empty(len(idx))
        noise = np.empty(len(idx))
        for j in range(len(idx)):
            c = cell_of[j]
            fp = f[c] + (vals[1][j] - base[j])
            fm = f[c] + (vals[-1][j] - base[j])
            # P(+) - P(-) = sum_keep |fp|^2 - |fm|^2, written as Re((fp - fm) conj(fp + fm))
            # so that the difference of the two nearby totals is not formed by cancellation
            diff = np.sum(keep[c] * np.real((vals[1][j] - vals[-1][j]) * np.conj(fp + fm)))
            g[j] = diff / (2 * d[j])
            # rounding floor: fp - fm is a difference of two one-point sums of size |c_j|
            noise[j] = (16 * np.finfo(float).eps * np.sum(keep[c] * np.abs(base[j]) * np.abs(f[c]))
                        / d[j])
        out[name] = g
        out["noise_" + name] = noise
    return f, out


def analytic_gradients(inp, cells, pts, f, keep):
    """The oracle's analytic gradient of sum_c P_c at the sampled points: the VJP of
    the cotangent 2 f keep, evaluated only at those points (each point's gradient
    depends on its own coordinates and its cell's cotangent)."""
    idx, win = _sub_points(inp, cells, pts)
    off = np.concatenate([[0], np.cumsum([len(p) for p in pts])]).astype(np.int64)
    g = 2.0 * f * keep
    gh, gx, gy = oracle.type1_vjp(off, inp["x"][idx], inp["y"][idx], inp["h"][idx], inp["w"][idx],
                                  np.asarray(inp["windows"])[cells], inp["n_modes"], g, kind=inp["kind"])
    return {"h": gh, "x": gx, "y": gy}


def test_c2_oracle_gradient_matches_central_differences():
    """8 cells x 64 points of 256-hexagon data at 64 x 64 modes: the oracle's analytic
    gradient against FP64 central differences of its own forward."""
    b = synth.config1(n_cells=8, precision="f64")
    inp = oracle.batch_inputs(b)
    cells, pts = synth.fd_sample(b, n_cells=8, n_points=64)
    print("cells", list(cells), "counts", list(b.counts()[cells]), flush=True)
    sub = b.subset(list(cells))
    f_full = oracle.type1(**{k: v for k, v in oracle.batch_inputs(sub).items()})
    keep, _, _ = oracle.ems_batched(f_full, oracle.EmsParams())
    f, fd = fd_gradients(inp, cells, pts, keep)
    assert np.allclose(f, f_full, rtol=0, atol=1e-9 * np.abs(f_full).max())
    an = analytic_gradients(inp, cells, pts, f, keep)
    for name in ("h", "x", "y"):
        err = np.abs(fd[name] - an[name])
        rel = np.linalg.norm(fd[name] - an[name]) / np.linalg.norm(an[name])
        print("d/d%s: rel-l2 %.2e, worst point |fd - an| / (|an| + noise) %.2e"
              % (name, rel, np.max(err / (np.abs(an[name]) + fd["noise_" + name]))), flush=True)
        assert rel <= 1e-8
        assert np.all(err <= 1e-6 * np.abs(an[name]) + fd["noise_" + name])


@pytest.mark.gpu
def test_c2_gpu_adjoint_matches_central_differences():
    """The full 256-hexagon batch in FP32 on the GPU: batched type-1, EMS and the
    retained-power adjoint; on 8 seeded cells x 64 seeded points the GPU gradients
    agree with FP64 central differences (on the FP32 inputs, kept sets frozen at the
    GPU's) to 5e-5 relative l2 per component."""
    import paper_2606_21278_amd as enf
    dev = torch.device("cuda:0")
    b = synth.config1(device=dev, precision="f32")
    gb = b.to(device=dev, dtype=torch.float32)
    plan = enf.Plan(gb.cell_offsets, gb.windows, n_modes=gb.n_modes, sigma=gb.sigma, eps=gb.eps, precision="f32")
    f = plan.type1(gb.x, gb.y, gb.h, gb.w)
    keep, ks, st = plan.ems(f)
    gh, gx, gy = plan.retained_power_adjoint(gb.x, gb.y, gb.h, gb.w, f, keep)
    torch.cuda.synchronize()
    cells, pts = synth.fd_sample(gb, n_cells=8, n_points=64)
    print("C1 full:", gb.n_points, "points; FD cells", list(cells), flush=True)
    sub = gb.subset(list(cells)).to(device="cpu")
    inp_sub = oracle.batch_inputs(sub)
    local_pts = list(pts)
    keep_c = keep[list(cells)].cpu().numpy()
    f_or, fd = fd_gradients(inp_sub, list(range(len(cells))), local_pts, keep_c)
    idx = np.concatenate([gb.cell_offsets[c] + np.sort(p) for c, p in zip(cells, pts)])
    it = torch.as_tensor(idx, device=dev)
    got = {"h": gh[it].cpu().double().numpy(), "x": gx[it].cpu().double().numpy(),
           "y": gy[it].cpu().double().numpy()}
    an = analytic_gradients(inp_sub, list(range(len(cells))), local_pts, f_or, keep_c)
    for name in ("h", "x", "y"):
        e_gpu = np.linalg.norm(got[name] - fd[name]) / np.linalg.norm(fd[name])
        e_or = np.linalg.norm(an[name] - fd[name]) / np.linalg.norm(fd[name])
        print("d/d%s: GPU vs FD rel-l2 %.2e, oracle vs FD %.2e" % (name, e_gpu, e_or), flush=True)
        assert e_or <= 1e-7
        assert e_gpu <= 5e-5
