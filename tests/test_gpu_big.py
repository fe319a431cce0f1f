"""GPU parity of the large-cell path (mode boxes above 64 per axis: the fine grid
lives in HBM and the points are sorted by tile) against the FP64 oracle.

Small clustered cells compare every mode; the full high-resolution cell (1e8
clustered points, 512 x 512 modes on a 1024^2 grid) compares a seeded sample of
modes and of points, which the oracle computes one by one.  Tolerances as in
test_gpu_parity: rel-l2 <= 5e-5 (FP32) and <= 1e-10 (FP64), identical EMS
selections on identical coefficients."""
import numpy as np
import pytest
import torch

import oracle
import paper_2606_21278_amd as enf
import synth
from helpers import gpu_batch, make_plan, oracle_f, per_cell_rel_l2, rel_l2

pytestmark = pytest.mark.gpu

TOL = {"f32": 5e-5, "f64": 1e-10}


def _type1(batch, **kw):
    gb = gpu_batch(batch)
    plan = make_plan(gb, **kw)
    f = plan.type1(gb.x, gb.y, gb.h, gb.w)
    torch.cuda.synchronize()
    return plan, gb, f.cpu().numpy()


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_big_clustered_cell_all_modes(prec):
    b = synth.config4(Q=20000, precision=prec, n_modes=(128, 96))
    print("clustered cell", prec, b.n_points, flush=True)
    plan, gb, f = _type1(b)
    info = plan.info()
    print(info, flush=True)
    assert list(info["grid"]) == [256, 256]
    ref = oracle_f(b)
    err = rel_l2(f, ref)
    print("rel-l2 %.3e" % err, flush=True)
    assert err <= TOL[prec]
    f2 = plan.type1(gb.x, gb.y, gb.h, gb.w).cpu().numpy()   # counters reset themselves
    assert rel_l2(f2, ref) <= TOL[prec]


@pytest.mark.parametrize("n_modes", [(80, 72), (65, 8), (100, 131)])
def test_big_multi_cell_shapes(n_modes):
    """Several cells (one empty, one with a single point), odd and even boxes, grids
    widened to two tiles per axis."""
    b = synth.uniform_box(counts=[6000, 0, 1, 9000], n_modes=n_modes, precision="f64", window_radius=2.8)
    print("box", n_modes, flush=True)
    plan, gb, f = _type1(b)
    print(plan.info(), flush=True)
    ref = oracle_f(b)
    e = per_cell_rel_l2(f, ref)
    print("per-cell", e, flush=True)
    assert np.all(f[1] == 0)
    assert e.max() <= TOL["f64"]


def test_big_percell_loop_matches_batched():
    b = synth.uniform_box(counts=[3000, 5000], n_modes=(96, 96), precision="f32", window_radius=3.0)
    gb = gpu_batch(b)
    plan = make_plan(gb)
    f = plan.type1(gb.x, gb.y, gb.h, gb.w)
    keep, ks, st = plan.ems(f)
    f2, keep2, ks2, st2 = plan.percell_loop(gb.x, gb.y, gb.h, gb.w)
    torch.cuda.synchronize()
    assert rel_l2(f2.cpu().numpy(), f.cpu().numpy()) < 1e-6
    ref = oracle_f(b.to(dtype=torch.float32))
    assert per_cell_rel_l2(f2.cpu().numpy(), ref).max() <= TOL["f32"]


def _ems_plan_for(f_ref, prec):
    n, N2, N1 = f_ref.shape
    off = np.arange(n + 1, dtype=np.int64)
    return enf.Plan(off, np.tile([[0.0, 0.0, 1.0]], (n, 1)), n_modes=(N1, N2), precision=prec,
                    eps=1e-10 if prec == "f64" else 1e-5)


@pytest.mark.parametrize("prm", [oracle.EmsParams(),
                                 oracle.EmsParams(k_min=3, k_max=5000, alpha_min=0.5, alpha_max=0.99, delta=0.05,
                                                  w1=0.3, w2=0.7),
                                 oracle.EmsParams(use_pairs=0, exclude_dc=0, alpha_min=0.9, alpha_max=0.9)])
def test_big_ems_on_identical_coefficients(prm):
    """Unit tables above 4096 take the device sort; given the same FP64 coefficients the
    selection equals the oracle's exactly."""
    b = synth.config4(Q=4000, precision="f64", n_modes=(128, 96))
    ref = np.concatenate([oracle_f(b), oracle_f(synth.config4(Q=3000, precision="f64", n_modes=(128, 96),
                                                              seed_config=14))])
    plan = _ems_plan_for(ref, "f64")
    keep, ks, st = plan.ems(torch.from_numpy(ref).to("cuda:0"), enf.EmsParams(**prm.__dict__))
    keep, ks, st = keep.cpu().numpy(), ks.cpu().numpy(), st.cpu().numpy()
    ok_keep, ok_ks, ok_st = oracle.ems_batched(ref, prm)
    print("k_star", ks, ok_ks, "J", st[:, 7], flush=True)
    assert st[0, 7] > 4096
    assert np.array_equal(ks, ok_ks)
    assert np.array_equal(keep, ok_keep)
    assert np.allclose(st, ok_st, rtol=1e-11, atol=0)


def test_big_ems_weighted_on_identical_coefficients():
    """Eq. (weighted_e) on the device-sort path (above 4,096 units per cell): asymmetric
    per-mode weights with zeros give the oracle's selection exactly."""
    ref = oracle_f(synth.config4(Q=4000, precision="f64", n_modes=(128, 96)))
    rng = np.random.default_rng(41)
    om = rng.uniform(0.0, 2.0, size=ref.shape[1:])
    om[rng.random(om.shape) < 0.1] = 0.0
    plan = _ems_plan_for(ref, "f64")
    for prm in (oracle.EmsParams(), oracle.EmsParams(use_pairs=0, exclude_dc=0, alpha_min=0.9, alpha_max=0.9)):
        keep, ks, st = plan.ems(torch.from_numpy(ref).to("cuda:0"), enf.EmsParams(**prm.__dict__),
                                mode_weight=torch.from_numpy(om))
        ok_keep, ok_ks, ok_st = oracle.ems_batched(ref, prm, mode_weight=om)
        print("weighted k_star", ks.cpu().numpy(), ok_ks, "J", st[:, 7].cpu().numpy(), flush=True)
        assert st[0, 7].item() > 4096
        assert np.array_equal(ks.cpu().numpy(), ok_ks)
        assert np.array_equal(keep.cpu().numpy(), ok_keep)
        assert np.allclose(st.cpu().numpy(), ok_st, rtol=1e-11, atol=0)


def test_big_ems_ties_at_the_cut():
    """Many units share each energy level, so the cut splits a run of equal energies:
    the kept ones are the tied units of lowest id, as in the oracle.  Coefficients are
    integers times a power of i, so every energy is an exact integer on both sides
    (with arbitrary phases, |f|^2 rounds differently with and without a fused
    multiply-add and near-ties would order by rounding)."""
    rng = np.random.default_rng(5)
    N1, N2 = 128, 96
    f = (rng.integers(1, 4, size=(2, N2, N1)) * np.array([1, 1j, -1, -1j])[rng.integers(0, 4, size=(2, N2, N1))]).astype(np.complex128)
    f[1] = np.abs(f[1])
    plan = _ems_plan_for(f, "f64")
    for prm in (oracle.EmsParams(use_pairs=0, exclude_dc=0, alpha_min=0.5, alpha_max=0.5),
                oracle.EmsParams(k_min=1, k_max=3000, alpha_min=0.3, alpha_max=0.3)):
        keep, ks, st = plan.ems(torch.from_numpy(f).to("cuda:0"), enf.EmsParams(**prm.__dict__))
        ok_keep, ok_ks, ok_st = oracle.ems_batched(f, prm)
        print("ties k_star", ks.cpu().numpy(), ok_ks, flush=True)
        assert np.array_equal(ks.cpu().numpy(), ok_ks)
        assert np.array_equal(keep.cpu().numpy(), ok_keep)
        assert np.allclose(st.cpu().numpy(), ok_st, rtol=1e-11, atol=0)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_big_adjoint_matches_oracle_vjp(prec):
    b = synth.config4(Q=20000, precision=prec, n_modes=(128, 96))
    inp = oracle.batch_inputs(b)
    f = oracle_f(b)
    keep, ks, st = oracle.ems_batched(f, oracle.EmsParams())
    g = 2.0 * f * keep
    gh, gx, gy = oracle.type1_vjp(inp["offsets"], inp["x"], inp["y"], inp["h"], inp["w"], inp["windows"],
                                  inp["n_modes"], g)
    gb = gpu_batch(b)
    plan = make_plan(gb)
    ah, ax, ay = plan.adjoint(gb.x, gb.y, gb.h, gb.w, torch.from_numpy(g).to("cuda:0", plan.cdtype))
    errs = [rel_l2(a.cpu().numpy(), r) for a, r in ((ah, gh), (ax, gx), (ay, gy))]
    print(prec, "adjoint rel-l2 h %.3e x %.3e y %.3e" % tuple(errs), flush=True)
    assert max(errs) <= TOL[prec]


def test_big_fp64_polynomial_taps():
    """FP64 large-cell plans evaluate the kernel as per-tap FP64 polynomials (degree 13,
    mirror pairs) when the fit is ten times below eps; ENUFFT_POLY64=0 keeps the exact
    kernel.  Both plans' type-1 and adjoint are within the FP64 tolerance of the oracle,
    and the two differ by no more than the fit allows."""
    import os
    b = synth.config4(Q=20000, precision="f64", n_modes=(128, 96))
    inp = oracle.batch_inputs(b)
    ref = oracle_f(b)
    g = np.ascontiguousarray(2.0 * ref)
    rh, rx, ry = oracle.type1_vjp(inp["offsets"], inp["x"], inp["y"], inp["h"], inp["w"], inp["windows"],
                                  inp["n_modes"], g)
    gb = gpu_batch(b)
    out = {}
    for name, env in (("poly", None), ("exact", "0")):
        old = os.environ.pop("ENUFFT_POLY64", None)
        if env is not None:
            os.environ["ENUFFT_POLY64"] = env
        try:
            plan = make_plan(gb)
        finally:
            os.environ.pop("ENUFFT_POLY64", None)
            if old is not None:
                os.environ["ENUFFT_POLY64"] = old
        info = plan.info()
        f = plan.type1(gb.x, gb.y, gb.h, gb.w).cpu().numpy()
        adj = plan.adjoint(gb.x, gb.y, gb.h, gb.w, torch.from_numpy(g).to("cuda:0", plan.cdtype))
        torch.cuda.synchronize()
        adj = [a.cpu().numpy() for a in adj]
        e_f = rel_l2(f, ref)
        e_a = max(rel_l2(a, r) for a, r in zip(adj, (rh, rx, ry)))
        print(name, "W", info["kernel_width"], "fit %.2e" % info["kernel_poly_err"],
              "type-1 rel-l2 %.3e adjoint %.3e" % (e_f, e_a), flush=True)
        assert info["kernel_width"] == 12
        assert (info["kernel_poly_err"] > 0) == (name == "poly")
        assert info["kernel_poly_err"] <= 0.1 * b.eps
        assert e_f <= TOL["f64"] and e_a <= TOL["f64"]
        out[name] = (f, adj)
    assert rel_l2(out["poly"][0], out["exact"][0]) <= 1e-11
    for a, e in zip(out["poly"][1], out["exact"][1]):
        assert rel_l2(a, e) <= 1e-11


def test_big_retained_power_pipeline_fp32():
    """type-1, EMS and the retained-power adjoint on the GPU, checked against the
    oracle's vjp with the GPU's own cotangent 2 f keep."""
    b = synth.config4(Q=20000, precision="f32", n_modes=(128, 96))
    gb = gpu_batch(b)
    plan = make_plan(gb)
    f = plan.type1(gb.x, gb.y, gb.h, gb.w)
    keep, ks, st = plan.ems(f)
    lam = torch.tensor([0.75], dtype=torch.float64, device="cuda:0")
    gh, gx, gy = plan.retained_power_adjoint(gb.x, gb.y, gb.h, gb.w, f, keep, lam=lam)
    fg = f.cpu().numpy().astype(np.complex128)
    g = 2.0 * 0.75 * fg * keep.cpu().numpy()
    inp = oracle.batch_inputs(b)
    rh, rx, ry = oracle.type1_vjp(inp["offsets"], inp["x"], inp["y"], inp["h"], inp["w"], inp["windows"],
                                  inp["n_modes"], g)
    errs = [rel_l2(a.cpu().numpy(), r) for a, r in ((gh, rh), (gx, rx), (gy, ry))]
    print("pipeline adjoint rel-l2 h %.3e x %.3e y %.3e" % tuple(errs), flush=True)
    assert max(errs) <= TOL["f32"]


def test_big_forward_graph_replays_match_eager():
    """The captured type-1 + EMS graph of a large-cell plan (sort, spreading, FFT
    passes, device-sort EMS; every buffer cleared by kernels, not memsets) replayed
    several times, with eager work between replays, matches the eager launches."""
    b = synth.uniform_box(counts=[40000, 0, 25000], n_modes=(128, 128), precision="f32", window_radius=3.0)
    gb = gpu_batch(b)
    plan = make_plan(gb)
    f0 = plan.type1(gb.x, gb.y, gb.h, gb.w)
    k0, ks0, st0 = plan.ems(f0)
    torch.cuda.synchronize()
    f0, k0, ks0 = f0.cpu().numpy(), k0.cpu().numpy(), ks0.cpu().numpy()
    out = (plan.empty_modes(), torch.empty(f0.shape, dtype=torch.uint8, device="cuda:0"),
           torch.empty(b.n_cells, dtype=torch.int32, device="cuda:0"),
           torch.empty((b.n_cells, 8), dtype=torch.float64, device="cuda:0"))
    for rep in range(4):
        plan.forward_graph(gb.x, gb.y, gb.h, gb.w, out=out)
        torch.cuda.synchronize()
        f, keep, ks, st = [t.cpu().numpy() for t in out]
        assert rel_l2(f, f0) < 1e-6, rep
        assert np.array_equal(ks, ks0) and np.array_equal(keep, k0), rep
        g = plan.type1(gb.x, gb.y, gb.h, gb.w)
        plan.ems(g)
        torch.cuda.synchronize()
    ref = oracle_f(b.to(dtype=torch.float32))
    assert per_cell_rel_l2(f, ref).max() <= TOL["f32"]


# ----------------------------------------------------------- the full high-resolution cell

@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_full_c4_sampled(prec):
    """1e8 clustered points, 512 x 512 modes.  Coefficients on a central block of the box
    and on a seeded product set of random rows and columns over the whole box (direct
    sums on that set), EMS on the GPU's own coefficients, and gradients on 2,048 seeded
    points.  Default sample: the central 32 x 32 modes and 8 x 32 random ones;
    ENUFFT_C4_SPEC_SAMPLE=1 takes the central 64 x 64 and 16 x 256 = 4,096 random modes
    (about two minutes of oracle time on 16 host threads)."""
    import os
    spec = os.environ.get("ENUFFT_C4_SPEC_SAMPLE") == "1"
    dev = torch.device("cuda:0")
    b = synth.config4(device=dev, precision=prec, progress=lambda m: print(m, flush=True))
    print("C4", prec, b.n_points, "spec sample" if spec else "default sample", flush=True)
    plan = make_plan(b)
    f = plan.type1(b.x, b.y, b.h, b.w)
    keep, ks, st = plan.ems(f)
    gh, gx, gy = plan.retained_power_adjoint(b.x, b.y, b.h, b.w, f, keep)
    torch.cuda.synchronize()
    print("info", plan.info(), flush=True)
    N1, N2 = b.n_modes
    fg = f[0].cpu().numpy().astype(np.complex128)
    kg = keep[0].cpu().numpy()
    x = b.x.cpu().numpy().astype(np.float64)
    y = b.y.cpu().numpy().astype(np.float64)
    h = b.h.cpu().numpy().astype(np.float64)
    w = b.w.cpu().numpy().astype(np.float64)
    c = oracle.strength(x, y, h, w, b.windows[0])
    lo1, lo2 = -(N1 // 2), -(N2 // 2)
    nc, nr, ncol = (64, 16, 256) if spec else (32, 8, 32)
    rng = np.random.default_rng(404)
    blocks = [(np.arange(-nc // 2, nc // 2), np.arange(-nc // 2, nc // 2)),
              # random columns and rows, with the box's first and last ones among them
              (np.unique(np.concatenate([[lo1, lo1 + N1 - 1],
                                         rng.choice(np.arange(lo1 + 1, lo1 + N1 - 1), ncol - 2, replace=False)])),
               np.unique(np.concatenate([[lo2, lo2 + N2 - 1],
                                         rng.choice(np.arange(lo2 + 1, lo2 + N2 - 1), nr - 2, replace=False)])))]
    for name, (kxl, kyl) in zip(("central", "random rows x columns"), blocks):
        print("oracle: direct sums on %s, %d x %d modes" % (name, len(kyl), len(kxl)), flush=True)
        parts = []
        for r0 in range(0, len(kyl), 8):   # a few rows at a time, each reported when done
            parts.append(oracle.type1_axes(x, y, c, kxl, kyl[r0:r0 + 8]))
            print("  rows %d..%d of %d done" % (r0, min(len(kyl), r0 + 8) - 1, len(kyl)), flush=True)
        ref = np.concatenate(parts, axis=0)
        got = fg[np.ix_(kyl - lo2, kxl - lo1)]
        err = rel_l2(got, ref)
        print("%s rel-l2 %.3e" % (name, err), flush=True)
        assert err <= TOL[prec]
    # EMS on the GPU's own coefficients
    r = oracle.ems(fg, oracle.EmsParams())
    print("k_star", int(ks[0]), r.k_star, flush=True)
    assert int(ks[0]) == r.k_star
    assert np.array_equal(kg, r.keep)
    assert np.allclose(st[0].cpu().numpy(), r.stats, rtol=1e-9, atol=0)
    # gradients at sampled points, with the GPU's cotangent
    rng = np.random.default_rng(405)
    idx = np.sort(rng.choice(b.n_points, size=2048, replace=False))
    g = (2.0 * fg * kg)[None]
    print("oracle: vjp at sampled points", flush=True)
    rh, rx, ry = oracle.type1_vjp(np.array([0, idx.size], dtype=np.int64), x[idx], y[idx], h[idx], w[idx],
                                  b.windows[:1], (N1, N2), g)
    it = torch.as_tensor(idx, device=dev)
    errs = [rel_l2(a[it].cpu().numpy(), rr) for a, rr in ((gh, rh), (gx, rx), (gy, ry))]
    print("sampled-point adjoint rel-l2 h %.3e x %.3e y %.3e" % tuple(errs), flush=True)
    assert max(errs) <= TOL[prec]
