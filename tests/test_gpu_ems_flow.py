"""GPU parity of the flow-dependent, per-timestep Elastic Mode Selection
(enufft_ems_flow: eq. (weighted_e) with the launch weight of Appendix A7, re-selected
per timestep on fixed coefficients) against the FP64 oracle, through the C ABI.

Given the same coefficients and flow records, the selection must be identical (K*,
kept sets) and the FP64 statistics equal to rounding."""
import os

import numpy as np
import pytest
import torch

import oracle
import paper_2606_21278_amd as enf
import synth
from helpers import gpu_batch, make_plan, oracle_f

pytestmark = pytest.mark.gpu


def _flows(T, n, seed, box_m=20000.0):
    rng = np.random.default_rng(seed)
    fl = np.zeros((T, n, 6))
    fl[..., 0] = rng.normal(scale=8.0, size=(T, n))
    fl[..., 1] = rng.normal(scale=8.0, size=(T, n))
    fl[..., 2] = rng.uniform(0.01, 0.025, size=(T, n))
    fl[..., 3] = 1e-4
    fl[..., 4] = rng.uniform(0.5, 1.2, size=(T, n))
    fl[..., 5] = 2 * np.pi / box_m
    return fl


def _ems_plan_for(f_ref, prec):
    n, N2, N1 = f_ref.shape
    off = np.arange(n + 1, dtype=np.int64)
    return enf.Plan(off, np.tile([[0.0, 0.0, 1.0]], (n, 1)), n_modes=(N1, N2), precision=prec,
                    eps=1e-10 if prec == "f64" else 1e-5)


PARAMS = [oracle.EmsParams(),
          oracle.EmsParams(k_min=1, k_max=4, alpha_min=0.9, alpha_max=1.0),
          oracle.EmsParams(k_min=2, k_max=60, alpha_min=0.3, alpha_max=0.95, delta=0.05, use_pairs=0)]


@pytest.mark.parametrize("wide", ["0", "1"])
@pytest.mark.parametrize("prm", PARAMS)
def test_ems_flow_matches_oracle_fp64(prm, wide):
    """Both in-register forms (ENUFFT_EMS_WIDE: three waves of sixteen values per lane,
    or up to sixteen waves of four) give the oracle's selection."""
    b = synth.config1(count_scale=0.003, n_cells=12, precision="f64")
    ref = oracle_f(b)
    plan = _ems_plan_for(ref, "f64")
    T = 5
    fl = _flows(T, ref.shape[0], 91)
    f = torch.from_numpy(ref).to("cuda:0")
    old = os.environ.get("ENUFFT_EMS_WIDE")
    os.environ["ENUFFT_EMS_WIDE"] = wide
    try:
        keep, ks, st = plan.ems_flow(f, fl, enf.EmsParams(**prm.__dict__))
        _, ks2, st2 = plan.ems_flow(f, fl, enf.EmsParams(**prm.__dict__), need_keep=False)
        torch.cuda.synchronize()
    finally:
        if old is None:
            os.environ.pop("ENUFFT_EMS_WIDE", None)
        else:
            os.environ["ENUFFT_EMS_WIDE"] = old
    ok_keep, ok_ks, ok_st = oracle.ems_flow(ref, fl, prm)
    ks, keep, st = ks.cpu().numpy(), keep.cpu().numpy(), st.cpu().numpy()
    print("K* per step (cell 0):", ks[:, 0], ok_ks[:, 0], flush=True)
    assert np.array_equal(ks, ok_ks)
    assert np.array_equal(keep, ok_keep)
    assert np.allclose(st, ok_st, rtol=1e-11, atol=0)
    assert np.array_equal(ks2.cpu().numpy(), ks) and np.array_equal(st2.cpu().numpy(), st)
    # the flow changes the selection between steps (not a constant weighting)
    assert len({keep[s].tobytes() for s in range(T)}) > 1


def test_ems_flow_on_gpu_fp32_coefficients():
    """The pipeline form: FP32 coefficients from the batched type-1, then T selections;
    identical to the oracle on the same coefficients."""
    b = synth.config1(count_scale=0.01, n_cells=16)
    gb = gpu_batch(b)
    plan = make_plan(gb)
    f = plan.type1(gb.x, gb.y, gb.h, gb.w)
    T = 6
    fl = _flows(T, gb.n_cells, 92)
    prm = oracle.EmsParams(k_min=1, k_max=12, alpha_min=0.0, alpha_max=0.7)
    keep, ks, st = plan.ems_flow(f, fl, enf.EmsParams(**prm.__dict__))
    torch.cuda.synchronize()
    fg = f.cpu().numpy().astype(np.complex128)
    ok_keep, ok_ks, ok_st = oracle.ems_flow(fg, fl, prm)
    assert np.array_equal(ks.cpu().numpy(), ok_ks)
    assert np.array_equal(keep.cpu().numpy(), ok_keep)
    assert np.allclose(st.cpu().numpy(), ok_st, rtol=1e-9, atol=0)


def test_ems_flow_one_step_equals_weighted_ems():
    """One step of the flow mode is enufft_ems with the same weights passed as
    mode_weight (computed here by the oracle's launch-weight function)."""
    b = synth.config1(count_scale=0.003, n_cells=6, precision="f64")
    ref = oracle_f(b)
    plan = _ems_plan_for(ref, "f64")
    fl = _flows(1, 6, 93)
    fl[0, :, :] = fl[0, 0, :]          # one flow for all cells, so one weight array
    N2, N1 = ref.shape[1:]
    om = np.array([[oracle.mw_weight(kx, ky, fl[0, 0, 5], *fl[0, 0, :5]) for kx in range(-(N1 // 2), N1 - N1 // 2)]
                   for ky in range(-(N2 // 2), N2 - N2 // 2)])
    f = torch.from_numpy(ref).to("cuda:0")
    k1, s1, t1 = plan.ems_flow(f, fl)
    k2, s2, t2 = plan.ems(f, mode_weight=torch.from_numpy(om))
    torch.cuda.synchronize()
    assert np.array_equal(k1[0].cpu().numpy(), k2.cpu().numpy())
    assert np.array_equal(s1[0].cpu().numpy(), s2.cpu().numpy())
    assert np.allclose(t1[0].cpu().numpy(), t2.cpu().numpy(), rtol=1e-13, atol=0)


def test_ems_flow_rejects_large_unit_tables_and_bad_arguments():
    b = synth.config4(Q=2000, precision="f64", n_modes=(128, 96))
    gb = gpu_batch(b)
    plan = make_plan(gb)
    f = plan.type1(gb.x, gb.y, gb.h, gb.w)
    with pytest.raises(enf.EnufftError) as e:
        plan.ems_flow(f, _flows(2, 1, 94))
    assert e.value.status == enf.EUNSUPPORTED
    small = _ems_plan_for(np.zeros((2, 8, 8), dtype=np.complex128), "f64")
    with pytest.raises(ValueError):
        small.ems_flow(torch.zeros((2, 8, 8), dtype=torch.complex128, device="cuda:0"), np.zeros((3, 5, 6)))
