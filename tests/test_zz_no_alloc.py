"""The allocation-free forward (enufft_type1_batched_noalloc) through the C ABI: its
scratch (work counters, split-cell merge counters and partial grids) lives in one
fixed device array instead of the plan's workspace.  Two calls in a row, the second
on a smaller batch, each checked against enufft_type1_batched on the same plan and
against the FP64 oracle; plans needing more scratch than the array holds, and
large-cell plans, are refused with an error."""
import ctypes

import numpy as np
import pytest
import torch

import paper_2606_21278_amd as enf
import synth
from helpers import gpu_batch, make_plan, oracle_f, per_cell_rel_l2, rel_l2

pytestmark = pytest.mark.gpu


def _lib():
    L = enf.load_library()
    L.enufft_type1_batched_noalloc.argtypes = [ctypes.c_void_p] * 6
    L.enufft_type1_batched_noalloc.restype = ctypes.c_int
    return L


def _noalloc(plan, gb, f):
    L = _lib()
    plan._sync_stream()
    return L.enufft_type1_batched_noalloc(plan._h, enf._ptr(gb.x), enf._ptr(gb.y), enf._ptr(gb.h), enf._ptr(gb.w),
                                          enf._ptr(f))


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_noalloc_matches_batched_twice(prec):
    tol = 5e-5 if prec == "f32" else 1e-10
    # first call: cells split into chunks (partial grids in the scratch array)
    big = synth.uniform_box(counts=[90000, 3, 0, 40000, 1, 65000, 20000], n_modes=(64, 64), precision=prec,
                            window_radius=3.0)
    # second call: a smaller batch on another plan
    small = synth.config1(count_scale=0.005, n_cells=10, precision=prec)
    for b in (big, small):
        gb = gpu_batch(b)
        plan = make_plan(gb, eps=1e-10 if prec == "f64" else 1e-5)
        info = plan.info()
        print(prec, b.name, "cells", b.n_cells, "points", b.n_points, "split", info["n_split_cells"], flush=True)
        f0 = plan.type1(gb.x, gb.y, gb.h, gb.w)
        f1 = plan.empty_modes()
        f1.fill_(float("nan"))
        st = _noalloc(plan, gb, f1)
        assert st == enf.OK, enf.load_library().enufft_last_error(plan._h)
        torch.cuda.synchronize()
        f0, f1 = f0.cpu().numpy(), f1.cpu().numpy()
        assert np.all(np.isfinite(f1))
        assert rel_l2(f1, f0) <= (1e-6 if prec == "f32" else 1e-13)
        ref = oracle_f(b)
        e = per_cell_rel_l2(f1, ref)
        print("per-cell rel-l2 max %.2e" % e.max(), flush=True)
        assert e.max() <= tol
    assert big.n_points > small.n_points


def test_noalloc_refuses_what_does_not_fit(monkeypatch):
    # a plan cut into ~4,000 chunks of 1,024 points: its split-cell partial grids
    # (64 KiB each) exceed the fixed 64 MiB scratch array
    monkeypatch.setenv("ENUFFT_FWD_CHUNK_MIN", "1024")
    monkeypatch.setenv("ENUFFT_FWD_ITEMS_PER_SLOT", "64")
    b = synth.uniform_box(counts=[1_000_000] * 4, n_modes=(64, 64), precision="f32", window_radius=3.0)
    gb = gpu_batch(b)
    plan = make_plan(gb)
    monkeypatch.delenv("ENUFFT_FWD_CHUNK_MIN")
    monkeypatch.delenv("ENUFFT_FWD_ITEMS_PER_SLOT")
    f = plan.empty_modes()
    st = _noalloc(plan, gb, f)
    msg = enf.load_library().enufft_last_error(plan._h).decode()
    print(plan.info()["n_split_cells"], st, msg, flush=True)
    assert st == enf.EINVAL and "scratch" in msg
    # the plan stays usable
    f0 = plan.type1(gb.x, gb.y, gb.h, gb.w)
    torch.cuda.synchronize()
    assert torch.isfinite(f0).all()
    # large-cell plans are refused
    c = synth.config4(Q=3000, precision="f32", n_modes=(128, 96))
    gc = gpu_batch(c)
    pc = make_plan(gc)
    assert _noalloc(pc, gc, pc.empty_modes()) == enf.EUNSUPPORTED
