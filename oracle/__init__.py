"""FP64 CPU oracle for the ENUFFT hot path -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never loads it and
shares no code with it.  The arithmetic lives in ``oracle.c`` (plain C, FP64,
OpenMP); this module only marshals numpy arrays through ctypes and adds a few
compositions of those calls (coefficients -> EMS -> cotangent -> gradients).

Pins (checked by the CPU test suite): brute-force dense sums on tiny inputs,
the regular-grid reduction to ``numpy.fft`` (Section 2.1.1), single-point
closed forms, linearity, Hermitian symmetry of eq. (series), the shift
theorem, the Monte Carlo error law and leakage variance of Appendix A3, the
EMS closed forms of Appendix A4 and of the Fig. 2 spectral families, the
adjoint identity and central finite differences.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# Mutation tests point this at a deliberately broken build of oracle.c.
_LIB_OVERRIDE = os.environ.get("ENUFFT_ORACLE_LIB")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_u8p = ctypes.POINTER(ctypes.c_uint8)


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (gcc, FP64, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-fno-fast-math",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if _LIB_OVERRIDE:
            L = ctypes.CDLL(_LIB_OVERRIDE)
        else:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build()
            L = ctypes.CDLL(_LIB)
        L.oracle_hann.argtypes = [ctypes.c_int] + [ctypes.c_double] * 5 + [_dp] * 3
        L.oracle_type1.argtypes = [ctypes.c_int64, _i64p, _dp, _dp, _dp, _dp, _dp, ctypes.c_int,
                                   ctypes.c_int, ctypes.c_int, ctypes.c_double, _dp]
        L.oracle_strength.argtypes = [ctypes.c_int64, _dp, _dp, _dp, _dp, ctypes.c_int, _dp, _dp]
        L.oracle_type1_modes.argtypes = [ctypes.c_int64, _dp, _dp, _dp, ctypes.c_int64, _i32p, _i32p,
                                         ctypes.c_double, _dp]
        L.oracle_type1_axes.argtypes = [ctypes.c_int64, _dp, _dp, _dp, ctypes.c_int, _i32p, ctypes.c_int, _i32p,
                                        ctypes.c_double, _dp]
        L.oracle_ems.argtypes = [ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int, ctypes.c_int,
                                 ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_double, ctypes.c_int, ctypes.c_int, _dp, _u8p, _i32p, _dp,
                                 _i32p, _dp]
        L.oracle_ems.restype = ctypes.c_int
        L.oracle_ems_batched.argtypes = [ctypes.c_int64, ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int,
                                         ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int, _dp,
                                         _u8p, _i32p, _dp]
        L.oracle_type1_vjp.argtypes = [ctypes.c_int64, _i64p, _dp, _dp, _dp, _dp, _dp, ctypes.c_int,
                                       ctypes.c_int, ctypes.c_int, ctypes.c_double, _dp, _dp, _dp, _dp]
        L.oracle_mw_weight.argtypes = [ctypes.c_int, ctypes.c_int] + [ctypes.c_double] * 6
        L.oracle_mw_weight.restype = ctypes.c_double
        L.oracle_ems_flow.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int,
                                      ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int, _dp, _u8p, _i32p,
                                      _dp]
        L.oracle_cell_geometry.argtypes = [ctypes.c_int64, _i64p, _dp, _dp, _dp, _dp, ctypes.c_int, ctypes.c_int,
                                           ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                           _dp, _dp, _dp, _dp, _u8p, _dp, _i32p]
        L.oracle_cell_geometry.restype = ctypes.c_int
        L.oracle_reconstruct.argtypes = [ctypes.c_int64, _i64p, _dp, _dp, _dp, _dp, _dp, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_int, _dp, _u8p, _dp, _dp, _dp]
        _lib = L
    return _lib


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_dp)


def _nullable(a, ptype):
    return ctypes.cast(None, ptype) if a is None else a.ctypes.data_as(ptype)


@dataclass
class EmsParams:
    """EMS parameters of Section 2.2 (k_min, k_max, alpha bounds, delta, w1, w2)."""
    k_min: int = 1
    k_max: int = 1 << 30
    alpha_min: float = 0.95
    alpha_max: float = 0.95
    delta: float = 0.02
    w1: float = 0.5
    w2: float = 0.5
    use_pairs: int = 1
    exclude_dc: int = 1


def hann(x, y, cx, cy, R, kind=1):
    L = _load()
    W, a, b = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    L.oracle_hann(kind, float(x), float(y), float(cx), float(cy), float(R),
                  ctypes.byref(W), ctypes.byref(a), ctypes.byref(b))
    return W.value, a.value, b.value


def type1(offsets, x, y, h, w, windows, n_modes, scale=1.0, kind=1) -> np.ndarray:
    """Direct FP64 type-1 sums for every cell -> complex128 [n_cells, N2, N1]."""
    L = _load()
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    n_cells = len(off) - 1
    N1, N2 = int(n_modes[0]), int(n_modes[1])
    x, px = _d(x); y, py = _d(y); h, ph = _d(h); w, pw = _d(w)
    win, pwin = _d(np.asarray(windows, dtype=np.float64).reshape(n_cells, 3))
    out = np.zeros((n_cells, N2, N1, 2), dtype=np.float64)
    L.oracle_type1(n_cells, off.ctypes.data_as(_i64p), px, py, ph, pw, pwin, kind, N1, N2, float(scale),
                   out.ctypes.data_as(_dp))
    return out[..., 0] + 1j * out[..., 1]


def strength(x, y, h, w, window, kind=1) -> np.ndarray:
    L = _load()
    x, px = _d(x); y, py = _d(y); h, ph = _d(h); w, pw = _d(w)
    win, pwin = _d(np.asarray(window, dtype=np.float64).reshape(3))
    out = np.zeros(len(x))
    L.oracle_strength(len(x), px, py, ph, pw, kind, pwin, out.ctypes.data_as(_dp))
    return out


def type1_modes(x, y, c, kx, ky, scale=1.0) -> np.ndarray:
    """Direct sums at listed integer modes for given strengths c -> complex128 [M]."""
    L = _load()
    x, px = _d(x); y, py = _d(y); c, pc = _d(c)
    kx = np.ascontiguousarray(kx, dtype=np.int32); ky = np.ascontiguousarray(ky, dtype=np.int32)
    out = np.zeros((len(kx), 2))
    L.oracle_type1_modes(len(x), px, py, pc, len(kx), kx.ctypes.data_as(_i32p), ky.ctypes.data_as(_i32p),
                         float(scale), out.ctypes.data_as(_dp))
    return out[:, 0] + 1j * out[:, 1]


def type1_axes(x, y, c, kx_list, ky_list, scale=1.0) -> np.ndarray:
    """Direct sums on the product set ky_list x kx_list of integer modes for given
    strengths c -> complex128 [len(ky_list), len(kx_list)]."""
    L = _load()
    x, px = _d(x); y, py = _d(y); c, pc = _d(c)
    kx = np.ascontiguousarray(kx_list, dtype=np.int32); ky = np.ascontiguousarray(ky_list, dtype=np.int32)
    out = np.zeros((len(ky), len(kx), 2))
    L.oracle_type1_axes(len(x), px, py, pc, len(kx), kx.ctypes.data_as(_i32p), len(ky), ky.ctypes.data_as(_i32p),
                        float(scale), out.ctypes.data_as(_dp))
    return out[..., 0] + 1j * out[..., 1]


@dataclass
class EmsResult:
    keep: np.ndarray          # uint8 [N2, N1]
    k_star: int
    stats: np.ndarray         # (T, P, N_eff, S_delta, C, alpha_C, theta(K*), J*)
    sorted_id: np.ndarray
    sorted_e: np.ndarray


def ems(f: np.ndarray, prm: EmsParams = EmsParams(), mode_weight=None) -> EmsResult:
    """EMS for one cell's coefficients f (complex [N2, N1])."""
    L = _load()
    N2, N1 = f.shape
    fr = np.ascontiguousarray(np.stack([f.real, f.imag], axis=-1), dtype=np.float64)
    keep = np.zeros((N2, N1), dtype=np.uint8)
    ks = np.zeros(1, dtype=np.int32)
    st = np.zeros(8)
    sid = np.zeros(N1 * N2, dtype=np.int32)
    se = np.zeros(N1 * N2)
    mw = None if mode_weight is None else np.ascontiguousarray(mode_weight, dtype=np.float64)
    J = L.oracle_ems(N1, N2, fr.ctypes.data_as(_dp), int(prm.k_min), int(min(prm.k_max, 2**31 - 1)),
                     float(prm.alpha_min), float(prm.alpha_max), float(prm.delta), float(prm.w1),
                     float(prm.w2), int(prm.use_pairs), int(prm.exclude_dc), _nullable(mw, _dp),
                     keep.ctypes.data_as(_u8p), ks.ctypes.data_as(_i32p), st.ctypes.data_as(_dp),
                     sid.ctypes.data_as(_i32p), se.ctypes.data_as(_dp))
    if J < 0:
        raise ValueError("oracle_ems: bad arguments")
    return EmsResult(keep, int(ks[0]), st, sid[:J].copy(), se[:J].copy())


def ems_batched(f: np.ndarray, prm: EmsParams = EmsParams(), mode_weight=None):
    """EMS for every cell of f (complex [n_cells, N2, N1]) -> (keep, k_star, stats)."""
    L = _load()
    n, N2, N1 = f.shape
    fr = np.ascontiguousarray(np.stack([f.real, f.imag], axis=-1), dtype=np.float64)
    keep = np.zeros((n, N2, N1), dtype=np.uint8)
    ks = np.zeros(n, dtype=np.int32)
    st = np.zeros((n, 8))
    mw = None if mode_weight is None else np.ascontiguousarray(mode_weight, dtype=np.float64)
    L.oracle_ems_batched(n, N1, N2, fr.ctypes.data_as(_dp), int(prm.k_min), int(min(prm.k_max, 2**31 - 1)),
                         float(prm.alpha_min), float(prm.alpha_max), float(prm.delta), float(prm.w1),
                         float(prm.w2), int(prm.use_pairs), int(prm.exclude_dc), _nullable(mw, _dp),
                         keep.ctypes.data_as(_u8p), ks.ctypes.data_as(_i32p), st.ctypes.data_as(_dp))
    return keep, ks, st


def mw_weight(kx, ky, kscale, ux, uy, N, fc, rho):
    """Launch weight |A| / |h|^2 of one mode under a flow (Appendix A7)."""
    return _load().oracle_mw_weight(int(kx), int(ky), float(kscale), float(ux), float(uy), float(N), float(fc),
                                    float(rho))


def ems_flow(f: np.ndarray, flow: np.ndarray, prm: EmsParams = EmsParams()):
    """EMS per timestep with flow-dependent launch weights on fixed coefficients f
    (complex [n_cells, N2, N1]); flow float64 [n_steps, n_cells, 6] = (ux, uy, N, fc,
    rho, kscale) -> (keep [n_steps, n_cells, N2, N1], k_star [n_steps, n_cells],
    stats [n_steps, n_cells, 8])."""
    L = _load()
    n, N2, N1 = f.shape
    fl = np.ascontiguousarray(flow, dtype=np.float64)
    T = fl.shape[0]
    assert fl.shape == (T, n, 6)
    fr = np.ascontiguousarray(np.stack([f.real, f.imag], axis=-1), dtype=np.float64)
    keep = np.zeros((T, n, N2, N1), dtype=np.uint8)
    ks = np.zeros((T, n), dtype=np.int32)
    st = np.zeros((T, n, 8))
    L.oracle_ems_flow(T, n, N1, N2, fr.ctypes.data_as(_dp), int(prm.k_min), int(min(prm.k_max, 2**31 - 1)),
                      float(prm.alpha_min), float(prm.alpha_max), float(prm.delta), float(prm.w1), float(prm.w2),
                      int(prm.use_pairs), int(prm.exclude_dc), fl.ctypes.data_as(_dp), keep.ctypes.data_as(_u8p),
                      ks.ctypes.data_as(_i32p), st.ctypes.data_as(_dp))
    return keep, ks, st


def type1_vjp(offsets, x, y, h, w, windows, n_modes, g, scale=1.0, kind=1):
    """Gradients (grad_h, grad_x, grad_y) of a real loss whose cotangent on f is g
    (complex [n_cells, N2, N1], g = dL/dRe f + i dL/dIm f)."""
    L = _load()
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    n_cells = len(off) - 1
    N1, N2 = int(n_modes[0]), int(n_modes[1])
    x, px = _d(x); y, py = _d(y); h, ph = _d(h); w, pw = _d(w)
    win, pwin = _d(np.asarray(windows, dtype=np.float64).reshape(n_cells, 3))
    gr = np.ascontiguousarray(np.stack([g.real, g.imag], axis=-1), dtype=np.float64)
    n = len(x)
    gh, gx, gy = np.zeros(n), np.zeros(n), np.zeros(n)
    L.oracle_type1_vjp(n_cells, off.ctypes.data_as(_i64p), px, py, ph, pw, pwin, kind, N1, N2, float(scale),
                       gr.ctypes.data_as(_dp), gh.ctypes.data_as(_dp), gx.ctypes.data_as(_dp),
                       gy.ctypes.data_as(_dp))
    return gh, gx, gy


def retained_power_grad(offsets, x, y, h, w, windows, n_modes, prm: EmsParams = EmsParams(),
                        scale=1.0, kind=1, lam=None):
    """Forward type-1 + EMS, then d(sum_c lam_c P_c)/d(h, x, y) with the kept set frozen.

    P_c = sum over kept modes of |f_k|^2, so the cotangent is g = 2 lam_c f keep."""
    f = type1(offsets, x, y, h, w, windows, n_modes, scale, kind)
    keep, ks, st = ems_batched(f, prm)
    n_cells = f.shape[0]
    lam = np.ones(n_cells) if lam is None else np.asarray(lam, dtype=np.float64)
    g = 2.0 * lam[:, None, None] * f * keep
    gh, gx, gy = type1_vjp(offsets, x, y, h, w, windows, n_modes, g, scale, kind)
    return dict(f=f, keep=keep, k_star=ks, stats=st, grad_h=gh, grad_x=gx, grad_y=gy)


def reconstruct(offsets, x, y, h, w, windows, n_modes, coef, keep=None, area=None, kind=1):
    """Truncated-series reconstruction at every sample from coefficients coef (complex
    [n_cells, N2, N1]) over the kept modes (keep uint8, None: all), and the per-cell
    diagnostics of Section 3.2 -> (h_rec [Q], diag [n_cells, 8]) with diag columns
    (Q_c, sum (t - h_rec)^2, sum t^2, sigma2_phys, sigma2_spec (all k != 0),
    sigma2_spec over kept k != 0, eps_rel, sigma2_spec / sigma2_phys), t = W h."""
    L = _load()
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    n_cells = len(off) - 1
    N1, N2 = int(n_modes[0]), int(n_modes[1])
    x, px = _d(x); y, py = _d(y); h, ph = _d(h); w, pw = _d(w)
    win, pwin = _d(np.asarray(windows, dtype=np.float64).reshape(n_cells, 3))
    cr = np.ascontiguousarray(np.stack([coef.real, coef.imag], axis=-1), dtype=np.float64)
    kp = None if keep is None else np.ascontiguousarray(keep, dtype=np.uint8)
    ar, par = _d(np.ones(n_cells) if area is None else np.asarray(area, dtype=np.float64))
    hr = np.zeros(len(x))
    dg = np.zeros((n_cells, 8))
    L.oracle_reconstruct(n_cells, off.ctypes.data_as(_i64p), px, py, ph, pw, pwin, kind, N1, N2,
                         cr.ctypes.data_as(_dp), _nullable(kp, _u8p), par, hr.ctypes.data_as(_dp),
                         dg.ctypes.data_as(_dp))
    return hr, dg


FRAMES = {"centroid": 0, "edge": 1}
MASKS = {"square": 0, "triangle": 1, "circle": 2}
WEIGHTS = {"uniform": 0, "voronoi": 1}


def cell_geometry(offsets, tri, x, y, h, frame="edge", mask="triangle", weights="uniform", raster=64, eta=1.0,
                  floor_frac=0.5, deplane=True):
    """Local frames, masks, quadrature weights and deplaning of Appendices A1, A2, A6 ->
    dict(xb, yb, hb, wb (w_q / |D|, 0 outside), inside, counts (raster points per
    sample), info [n_cells, 8] = (xbar_x, xbar_y, cos, sin, H, |D|, Q_in, hbar))."""
    L = _load()
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    n_cells = len(off) - 1
    tr, ptr = _d(np.asarray(tri, dtype=np.float64).reshape(n_cells, 6))
    x, px = _d(x); y, py = _d(y); h, ph = _d(h)
    n = len(x)
    out = {k: np.zeros(n) for k in ("xb", "yb", "hb", "wb")}
    inside = np.zeros(n, dtype=np.uint8)
    counts = np.zeros(n, dtype=np.int32)
    info = np.zeros((n_cells, 8))
    r = L.oracle_cell_geometry(n_cells, off.ctypes.data_as(_i64p), ptr, px, py, ph, FRAMES[frame], MASKS[mask],
                               WEIGHTS[weights], int(raster), float(eta), float(floor_frac), int(deplane),
                               out["xb"].ctypes.data_as(_dp), out["yb"].ctypes.data_as(_dp),
                               out["hb"].ctypes.data_as(_dp), out["wb"].ctypes.data_as(_dp),
                               inside.ctypes.data_as(_u8p), info.ctypes.data_as(_dp), counts.ctypes.data_as(_i32p))
    if r != 0:
        raise ValueError("oracle_cell_geometry: bad arguments")
    out.update(inside=inside, counts=counts, info=info)
    return out


def batch_inputs(batch, cells=None):
    """Float64 host copies of a synth.Batch (optionally a subset of cells), for the oracle."""
    b = batch if cells is None else batch.subset(cells)
    g = lambda t: t.detach().to("cpu").double().numpy()
    kind = 1 if (b.windows[:, 2] > 0).all() else 0
    return dict(offsets=b.cell_offsets, x=g(b.x), y=g(b.y), h=g(b.h), w=g(b.w), windows=b.windows,
                n_modes=b.n_modes, kind=kind)
