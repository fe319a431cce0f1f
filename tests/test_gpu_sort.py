"""GPU parity of the point sort (enufft_sort_points: a per-cell device counting sort of
the samples by the fine cell their kernel footprint starts in) and of the batched type-1
on the sorted samples, against the FP64 oracle, on samples stored in no spatial order:
the shuffled icosahedral cells and the hexagon batch as generated.

The sort moves data only: the sorted arrays are the inputs gathered through the returned
permutation, bit for bit, and the permutation maps every cell onto itself.  The sorted
and unsorted coefficients are sums of the same terms in another order: each within the
FP32 (5e-5) or FP64 (1e-10) tolerance of the oracle per cell, and within rounding of
each other."""
import numpy as np
import pytest
import torch

import paper_2606_21278_amd as enf
import synth
from helpers import gpu_batch, make_plan, oracle_f, per_cell_rel_l2, rel_l2

pytestmark = pytest.mark.gpu

TOL = {"f32": 5e-5, "f64": 1e-10}


def _check_sort(gb, out, plan):
    xs, ys, hs, ws, perm = (t.cpu().numpy() if t is not None else None for t in out)
    x, y, h, w = (t.cpu().numpy() for t in (gb.x, gb.y, gb.h, gb.w))
    off = gb.cell_offsets
    for c in range(gb.n_cells):
        a, b = int(off[c]), int(off[c + 1])
        assert np.array_equal(np.sort(perm[a:b]), np.arange(a, b))   # a permutation of the cell
    assert np.array_equal(xs, x[perm]) and np.array_equal(ys, y[perm])
    assert np.array_equal(hs, h[perm]) and np.array_equal(ws, w[perm])
    # sorted by fine cell: (row, column) of the footprint origin nondecreasing inside each
    # cell, up to the rounding of the fine coordinate at a cell boundary
    n1, n2 = plan.info()["grid"]
    W = plan.info()["kernel_width"]
    t = lambda v, n: np.ceil(v.astype(np.float64) * n / (2 * np.pi) - W / 2).astype(np.int64)
    key = (t(ys, n2) % n2) * n1 + (t(xs, n1) % n1)
    bad = 0
    for c in range(gb.n_cells):
        a, b = int(off[c]), int(off[c + 1])
        bad += int(np.sum(np.diff(key[a:b]) < 0))
    assert bad <= 1e-4 * max(1, gb.n_points)
    return xs, ys, hs, ws, perm


@pytest.mark.parametrize("which,prec", [("c3_shuffled", "f32"), ("c1", "f32"), ("c1", "f64")])
def test_sorted_type1_matches_oracle(which, prec):
    if which == "c1":
        b = synth.config1(count_scale=0.01, n_cells=24, precision=prec)
    else:
        b = synth.config3(n_cells=24, count_scale=0.05, precision=prec, shuffled=True)
    if prec == "f64":
        b.eps = 1e-10
    gb = gpu_batch(b)
    plan = make_plan(gb)
    f0 = plan.type1(gb.x, gb.y, gb.h, gb.w)
    out = plan.sort_points(gb.x, gb.y, gb.h, gb.w)
    f1 = plan.type1(*out[:4])
    torch.cuda.synchronize()
    _check_sort(gb, out, plan)
    ref = oracle_f(b)
    e0 = per_cell_rel_l2(f0.cpu().numpy(), ref)
    e1 = per_cell_rel_l2(f1.cpu().numpy(), ref)
    d = rel_l2(f1.cpu().numpy(), f0.cpu().numpy())
    print("%s %s: per-cell rel-l2 unsorted %.2e sorted %.2e; sorted vs unsorted %.2e"
          % (which, prec, e0.max(), e1.max(), d), flush=True)
    assert e0.max() <= TOL[prec] and e1.max() <= TOL[prec]
    assert d <= (1e-6 if prec == "f32" else 1e-13)


def test_sorted_gradients_map_back():
    """Gradients on the sorted samples, scattered back through the permutation, equal the
    gradients on the original order (same cotangent)."""
    b = synth.config3(n_cells=12, count_scale=0.05, precision="f32", shuffled=True)
    gb = gpu_batch(b)
    plan = make_plan(gb)
    xs, ys, hs, ws, perm = plan.sort_points(gb.x, gb.y, gb.h, gb.w)
    f = plan.type1(gb.x, gb.y, gb.h, gb.w)
    keep = torch.ones(f.shape, dtype=torch.uint8, device="cuda:0")
    g0 = plan.retained_power_adjoint(gb.x, gb.y, gb.h, gb.w, f, keep)
    g1 = plan.retained_power_adjoint(xs, ys, hs, ws, f, keep)
    torch.cuda.synchronize()
    p = perm.long()
    for a, s in zip(g0, g1):
        back = torch.empty_like(s)
        back[p] = s
        assert rel_l2(back.cpu().numpy(), a.cpu().numpy()) <= 1e-6


def test_sort_edge_cases():
    """Empty cells and a one-point cell, optional outputs, argument checks."""
    b = synth.uniform_box(counts=[0, 1, 3000, 0, 800], n_modes=(32, 32), precision="f32", window_radius=2.5)
    gb = gpu_batch(b)
    off = gb.cell_offsets
    idx = torch.cat([torch.arange(off[c], off[c + 1], device="cuda:0")[torch.randperm(int(off[c + 1] - off[c]),
                     device="cuda:0")] for c in range(gb.n_cells)])
    x, y, h, w = gb.x[idx].contiguous(), gb.y[idx].contiguous(), gb.h[idx].contiguous(), gb.w[idx].contiguous()
    plan = make_plan(gb)
    f0 = plan.type1(x, y, h, w)
    xs, ys, hs, ws, perm = plan.sort_points(x, y, h, w)
    xs2, ys2, hs2, ws2, perm2 = plan.sort_points(x, y, need_perm=False)
    f1 = plan.type1(xs, ys, hs, ws)
    torch.cuda.synchronize()
    assert hs2 is None and ws2 is None and perm2 is None
    assert rel_l2(f1.cpu().numpy(), f0.cpu().numpy()) <= 1e-6
    assert np.all(f1.cpu().numpy()[[0, 3]] == 0)
    # the multiset of sorted x per fine cell does not depend on the run
    assert np.array_equal(np.sort(xs2.cpu().numpy()[1:3001]), np.sort(xs.cpu().numpy()[1:3001]))
    with pytest.raises(enf.EnufftError):
        enf._check(plan._lib.enufft_sort_points(plan._h, enf._ptr(x), enf._ptr(y), None, None, None, enf._ptr(ys),
                                                None, None, None), plan._h)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_large_cell_sorted_input(prec):
    """Large cells: sorted by tile (and by fine cell inside each tile), the input lets
    type-1 and the adjoint skip their scatter (each call's counting pass finds the order)
    with the same results; one pair of far-apart samples swapped makes the order fail the
    check and the full sort runs."""
    b = synth.config4(Q=30000, precision=prec, n_modes=(128, 96))
    if prec == "f64":
        b.eps = 1e-10
    gb = gpu_batch(b)
    plan = make_plan(gb)
    f0 = plan.type1(gb.x, gb.y, gb.h, gb.w)
    xs, ys, hs, ws, perm = plan.sort_points(gb.x, gb.y, gb.h, gb.w)
    f1 = plan.type1(xs, ys, hs, ws)
    keep = torch.ones(f0.shape, dtype=torch.uint8, device="cuda:0")
    g0 = plan.retained_power_adjoint(gb.x, gb.y, gb.h, gb.w, f0, keep)
    g1 = plan.retained_power_adjoint(xs, ys, hs, ws, f0, keep)
    # a swap between the first and the last sorted sample
    i, j = 0, gb.n_points - 1
    xw, yw, hw, ww = xs.clone(), ys.clone(), hs.clone(), ws.clone()
    for t in (xw, yw, hw, ww):
        t[[i, j]] = t[[j, i]]
    f2 = plan.type1(xw, yw, hw, ww)
    torch.cuda.synchronize()
    x, xsn = gb.x.cpu().numpy(), xs.cpu().numpy()
    assert np.array_equal(np.sort(perm.cpu().numpy()), np.arange(gb.n_points))
    assert np.array_equal(xsn, x[perm.cpu().numpy()])
    lim = 1e-6 if prec == "f32" else 1e-13
    assert rel_l2(f1.cpu().numpy(), f0.cpu().numpy()) <= lim
    assert rel_l2(f2.cpu().numpy(), f0.cpu().numpy()) <= lim
    assert rel_l2(f0.cpu().numpy(), oracle_f(b)) <= TOL[prec]
    p = perm.long()
    for a, s in zip(g0, g1):
        back = torch.empty_like(s)
        back[p] = s
        assert rel_l2(back.cpu().numpy(), a.cpu().numpy()) <= lim


def _big_keys(x, y, info):
    """Tile-then-cell key of each sample's footprint origin (FP64 on the host)."""
    n1, n2 = info["grid"][0], info["grid"][1]
    W = info["kernel_width"]
    ix = (np.ceil(x.astype(np.float64) * n1 / (2 * np.pi) - W / 2).astype(np.int64)) & (n1 - 1)
    iy = (np.ceil(y.astype(np.float64) * n2 / (2 * np.pi) - W / 2).astype(np.int64)) & (n2 - 1)
    ntx = n1 // 32
    return ((iy // 32) * ntx + ix // 32) * 1024 + (iy % 32) * 32 + ix % 32


@pytest.mark.parametrize("eps", [1e-3, 1e-5, 1e-6])
def test_large_cell_runs_fp32(eps):
    """FP32 large cells in the order enufft_sort_points leaves (by tile, then by fine cell
    inside each tile): runs of samples with one footprint origin are summed in registers
    before they reach the FP64 sub-grid (W = 4, 6, 8).  Dense clusters (several samples per
    fine cell) give long runs.  Against the oracle's direct sum, and against the same
    samples unsorted (point-by-point spreading: sums in another order)."""
    b = synth.config4(Q=200000, precision="f32", n_modes=(128, 96))
    b.eps = eps
    gb = gpu_batch(b)
    plan = make_plan(gb)
    info = plan.info()
    xs, ys, hs, ws, perm = plan.sort_points(gb.x, gb.y, gb.h, gb.w)
    f0 = plan.type1(gb.x, gb.y, gb.h, gb.w)
    f1 = plan.type1(xs, ys, hs, ws)
    torch.cuda.synchronize()
    keys = _big_keys(xs.cpu().numpy(), ys.cpu().numpy(), info)
    # in key order, but for origins that the FP32 device coordinate and the FP64 host
    # one put on either side of a cell edge
    desc = int(np.sum(np.diff(keys) < 0))
    runs = np.diff(np.flatnonzero(np.diff(keys) != 0))
    print("W %d: %d key descents, mean run %.2f samples, longest %d" % (info["kernel_width"], desc, runs.mean(),
          runs.max()), flush=True)
    assert desc <= max(4, gb.n_points // 10000)
    assert runs.mean() > 2
    assert np.array_equal(np.sort(perm.cpu().numpy()), np.arange(gb.n_points))
    ref = oracle_f(b)
    tol = max(5.0 * eps, TOL["f32"])
    e1, e01 = rel_l2(f1.cpu().numpy(), ref), rel_l2(f1.cpu().numpy(), f0.cpu().numpy())
    print("rel-l2 against the oracle %.2e, against point-by-point %.2e" % (e1, e01), flush=True)
    assert e1 <= tol
    assert e01 <= 2e-6


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_large_cell_bound_points(prec):
    """enufft_bind_points: tile-ordered coordinates bound once; calls given exactly those
    tensors skip the tile sort and give the results of the unbound calls, with h changed
    between calls; unsorted coordinates are refused (the plan stays unbound); one of the
    two bound tensors alone is not the binding; unbinding restores the sorting calls."""
    b = synth.config4(Q=200000, precision=prec, n_modes=(128, 96))
    if prec == "f64":
        b.eps = 1e-10
    gb = gpu_batch(b)
    plan = make_plan(gb)
    xs, ys, hs, ws, _ = plan.sort_points(gb.x, gb.y, gb.h, gb.w, need_perm=False)
    f0 = plan.type1(xs, ys, hs, ws)
    keep = torch.ones(f0.shape, dtype=torch.uint8, device="cuda:0")
    f0h = plan.type1(xs, ys, 2 * hs, ws)
    g0 = plan.retained_power_adjoint(xs, ys, hs, ws, f0, keep)
    with pytest.raises(enf.EnufftError) as e:
        plan.bind_points(gb.x, gb.y)   # as generated: not in tile order
    assert e.value.status == enf.EINVAL
    plan.bind_points(xs, ys)
    f1 = plan.type1(xs, ys, hs, ws)
    f1h = plan.type1(xs, ys, 2 * hs, ws)
    g1 = plan.retained_power_adjoint(xs, ys, hs, ws, f0, keep)
    ys2 = ys.clone()
    f2 = plan.type1(xs, ys2, hs, ws)   # y is another tensor: sorted as usual
    plan.unbind_points()
    f3 = plan.type1(xs, ys, hs, ws)
    torch.cuda.synchronize()
    lim = 1e-6 if prec == "f32" else 1e-13
    for f, ref in ((f1, f0), (f1h, f0h), (f2, f0), (f3, f0)):
        assert rel_l2(f.cpu().numpy(), ref.cpu().numpy()) <= lim
    for a, c in zip(g1, g0):
        assert rel_l2(a.cpu().numpy(), c.cpu().numpy()) <= lim
    assert rel_l2(f0.cpu().numpy(), oracle_f(b)) <= TOL[prec]
    with pytest.raises(ValueError):
        plan.bind_points(xs, None)
