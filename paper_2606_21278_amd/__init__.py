"""MI355X (gfx950) ENUFFT hot path: batched windowed type-1 NUFFT, Elastic Mode
Selection and the type-2 adjoint, behind the C ABI in include/enufft.h.

This module only marshals arguments to ``libenufft.so`` (ctypes); every step of
the computation runs in the library's HIP kernels.  PyTorch supplies device
memory and the current stream.  If the library is missing, importing the
binding raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libenufft.so")

OK, EINVAL, ENOMEM, EDEVICE, EEPS, ESTATE, EUNSUPPORTED = range(7)
_STATUS = {0: "ENUFFT_OK", 1: "ENUFFT_EINVAL", 2: "ENUFFT_ENOMEM", 3: "ENUFFT_EDEVICE", 4: "ENUFFT_EEPS",
           5: "ENUFFT_ESTATE", 6: "ENUFFT_EUNSUPPORTED"}
F32, F64 = 0, 1
WIN_NONE, WIN_HANN = 0, 1
KERNELS = {"es": 0, "kb_mirt": 1, "kb_fessler": 2}


class EnufftError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (_STATUS.get(status, str(status)), msg))
        self.status = status


class Opts(ctypes.Structure):
    _fields_ = [("n_modes", ctypes.c_int32 * 2), ("sigma", ctypes.c_double), ("eps", ctypes.c_double),
                ("precision", ctypes.c_int32), ("window_kind", ctypes.c_int32), ("scale", ctypes.c_double),
                ("autotune", ctypes.c_int32), ("kernel_width", ctypes.c_int32), ("kernel_kind", ctypes.c_int32)]


class Window(ctypes.Structure):
    _fields_ = [("cx", ctypes.c_double), ("cy", ctypes.c_double), ("radius", ctypes.c_double)]


class EmsParamsC(ctypes.Structure):
    _fields_ = [("k_min", ctypes.c_int32), ("k_max", ctypes.c_int32), ("alpha_min", ctypes.c_double),
                ("alpha_max", ctypes.c_double), ("delta", ctypes.c_double), ("w1", ctypes.c_double),
                ("w2", ctypes.c_double), ("use_pairs", ctypes.c_int32), ("exclude_dc", ctypes.c_int32)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("n_modes", ctypes.c_int32 * 2), ("grid", ctypes.c_int32 * 2), ("kernel_width", ctypes.c_int32),
                ("beta", ctypes.c_double), ("n_cells", ctypes.c_int64), ("n_points", ctypes.c_int64),
                ("n_items_fwd", ctypes.c_int64), ("n_split_cells", ctypes.c_int64),
                ("n_items_adj", ctypes.c_int64), ("adj_bands", ctypes.c_int32),
                ("fwd_threads", ctypes.c_int32), ("fwd_blocks", ctypes.c_int32),
                ("adj_threads", ctypes.c_int32), ("adj_blocks", ctypes.c_int32),
                ("workspace_bytes", ctypes.c_int64), ("kernel_poly_err", ctypes.c_double),
                ("tuned", ctypes.c_int32), ("tune_cache_hit", ctypes.c_int32), ("fwd_chunk_min", ctypes.c_int64),
                ("fwd_items_per_slot", ctypes.c_int32), ("adj_items_per_slot", ctypes.c_int32),
                ("adj_band_mult", ctypes.c_int32), ("fwd_acc", ctypes.c_int32),
                ("tune_fwd_ms", ctypes.c_double), ("tune_adj_ms", ctypes.c_double),
                ("kernel_kind", ctypes.c_int32), ("adj_kernel_width", ctypes.c_int32)]


class GeometryOptsC(ctypes.Structure):
    _fields_ = [("frame", ctypes.c_int32), ("mask", ctypes.c_int32), ("weights", ctypes.c_int32),
                ("raster", ctypes.c_int32), ("eta", ctypes.c_double), ("floor_frac", ctypes.c_double),
                ("deplane", ctypes.c_int32), ("reserved_", ctypes.c_int32)]


FRAMES = {"centroid": 0, "edge": 1}
MASKS = {"square": 0, "triangle": 1, "circle": 2}
WEIGHTS = {"uniform": 0, "voronoi": 1}


EXPORTS = ["enufft_default_opts", "enufft_plan", "enufft_set_stream", "enufft_type1_batched",
           "enufft_type1_batched_noalloc", "enufft_ems",
           "enufft_ems_flow",
           "enufft_type1_adjoint", "enufft_retained_power_adjoint", "enufft_reconstruct", "enufft_cell_geometry", "enufft_sort_points",
           "enufft_bind_points", "enufft_percell_loop",
           "enufft_forward_graph", "enufft_set_timing", "enufft_get_timing",
           "enufft_get_info", "enufft_destroy", "enufft_last_error", "enufft_version"]

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libenufft.so and declare its C signatures.  Raises if it is not built."""
    global _lib
    if _lib is not None and path == LIB_PATH:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libenufft.so is not built (run __graft_entry__.build() or "
                          "python -m paper_2606_21278_amd.build); there is no fallback")
    L = ctypes.CDLL(path)
    vp, i64, i32, dp = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)
    L.enufft_default_opts.argtypes = [ctypes.POINTER(Opts)]
    L.enufft_plan.argtypes = [ctypes.POINTER(vp), i64, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(Window),
                              ctypes.POINTER(Opts), vp]
    L.enufft_set_stream.argtypes = [vp, vp]
    L.enufft_type1_batched.argtypes = [vp] * 6
    L.enufft_type1_batched_noalloc.argtypes = [vp] * 6
    L.enufft_ems.argtypes = [vp, vp, ctypes.POINTER(EmsParamsC), vp, vp, vp, vp]
    L.enufft_ems_flow.argtypes = [vp, vp, ctypes.POINTER(EmsParamsC), i32, vp, vp, vp, vp]
    L.enufft_type1_adjoint.argtypes = [vp] * 9
    L.enufft_retained_power_adjoint.argtypes = [vp] * 11
    L.enufft_reconstruct.argtypes = [vp] * 10
    L.enufft_cell_geometry.argtypes = [vp] * 5 + [ctypes.POINTER(GeometryOptsC)] + [vp] * 7
    L.enufft_sort_points.argtypes = [vp] * 10
    L.enufft_bind_points.argtypes = [vp] * 3
    L.enufft_percell_loop.argtypes = [vp] * 6 + [ctypes.POINTER(EmsParamsC), vp, vp, vp, vp]
    L.enufft_forward_graph.argtypes = [vp] * 6 + [ctypes.POINTER(EmsParamsC), vp, vp, vp, vp]
    L.enufft_set_timing.argtypes = [vp, i32]
    L.enufft_get_timing.argtypes = [vp, dp]
    L.enufft_get_info.argtypes = [vp, ctypes.POINTER(PlanInfo)]
    L.enufft_destroy.argtypes = [vp]
    L.enufft_last_error.argtypes = [vp]
    L.enufft_last_error.restype = ctypes.c_char_p
    L.enufft_version.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name != "enufft_last_error" and name != "enufft_version":
            getattr(L, name).restype = ctypes.c_int
    if path == LIB_PATH:
        _lib = L
    return L


def _check(status: int, plan_handle=None):
    if status != OK:
        L = load_library()
        msg = L.enufft_last_error(plan_handle)
        raise EnufftError(status, msg.decode() if msg else "")


@dataclass
class EmsParams:
    """Elastic Mode Selection parameters (Section 2.2).  Defaults: keep the modes that
    cover 95 % of the power with no budget (alpha_min = alpha_max = 0.95)."""
    k_min: int = 1
    k_max: int = 2 ** 31 - 1
    alpha_min: float = 0.95
    alpha_max: float = 0.95
    delta: float = 0.02
    w1: float = 0.5
    w2: float = 0.5
    use_pairs: int = 1
    exclude_dc: int = 1

    def c(self) -> EmsParamsC:
        return EmsParamsC(int(self.k_min), int(self.k_max), float(self.alpha_min), float(self.alpha_max),
                          float(self.delta), float(self.w1), float(self.w2), int(self.use_pairs),
                          int(self.exclude_dc))


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Plan:
    """A batch layout (CSR cell offsets, per-cell windows) and transform options.

    All tensors passed to the methods live on the plan's CUDA/HIP device and use the
    plan's dtype (float32 or float64); coefficients are complex64 / complex128 of
    shape [n_cells, N2, N1] (k_y slow, k_x fast, each ascending from -floor(N/2))."""

    def __init__(self, cell_offsets, windows=None, n_modes=(64, 64), sigma=2.0, eps=1e-5,
                 precision="f32", window="hann", scale=1.0, autotune=False, kernel_width=0,
                 kernel="es", device=None, stream=None):
        self._lib = load_library()
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        off = np.ascontiguousarray(np.asarray(cell_offsets, dtype=np.int64))
        self.n_cells = len(off) - 1
        self.n_points = int(off[-1]) if self.n_cells >= 0 else 0
        self.offsets = off
        self.precision = precision
        self.dtype = torch.float64 if precision == "f64" else torch.float32
        self.cdtype = torch.complex128 if precision == "f64" else torch.complex64
        self.n_modes = (int(n_modes[0]), int(n_modes[1]))
        opts = Opts()
        opts.n_modes[0], opts.n_modes[1] = self.n_modes
        opts.sigma, opts.eps = float(sigma), float(eps)
        opts.precision = F64 if precision == "f64" else F32
        opts.window_kind = WIN_HANN if window == "hann" else WIN_NONE
        opts.scale = float(scale)
        # autotune: False / True (trials on raster-ordered points) / "raster" / "unordered"
        modes = {False: 0, True: 1, "raster": 1, "unordered": 2}
        if autotune not in modes:
            raise ValueError("autotune must be False, True, 'raster' or 'unordered'")
        opts.autotune = modes[autotune]
        opts.kernel_width = int(kernel_width)
        if kernel not in KERNELS:
            raise ValueError("kernel must be one of %s" % sorted(KERNELS))
        opts.kernel_kind = KERNELS[kernel]
        wins = None
        if windows is not None:
            wa = np.ascontiguousarray(np.asarray(windows, dtype=np.float64).reshape(-1, 3))
            wins = (Window * max(1, len(wa)))()
            for i, (cx, cy, r) in enumerate(wa):
                wins[i] = Window(cx, cy, r)
        with torch.cuda.device(self.device):
            s = stream if stream is not None else torch.cuda.current_stream(self.device)
            self._stream = s
            h = ctypes.c_void_p()
            st = self._lib.enufft_plan(ctypes.byref(h), self.n_cells,
                                       off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                       wins, ctypes.byref(opts), ctypes.c_void_p(s.cuda_stream))
            _check(st, None)
        self._h = h
        self._bound = None   # (x, y) bound by bind_points, kept referenced

    # -- helpers
    def _sync_stream(self):
        s = torch.cuda.current_stream(self.device)
        if s.cuda_stream != self._stream.cuda_stream:
            self._stream = s
            _check(self._lib.enufft_set_stream(self._h, ctypes.c_void_p(s.cuda_stream)), self._h)

    def _pts(self, *ts):
        for t in ts:
            if t is None:
                continue
            if t.device != self.device or t.dtype != self.dtype or not t.is_contiguous() or t.numel() != self.n_points:
                raise ValueError("point arrays must be contiguous %s tensors of length %d on %s"
                                 % (self.dtype, self.n_points, self.device))

    def info(self) -> dict:
        inf = PlanInfo()
        _check(self._lib.enufft_get_info(self._h, ctypes.byref(inf)), self._h)
        return {k: (list(getattr(inf, k)) if k in ("n_modes", "grid") else getattr(inf, k)) for k, _ in PlanInfo._fields_}

    def empty_modes(self):
        return torch.empty((self.n_cells, self.n_modes[1], self.n_modes[0]), dtype=self.cdtype, device=self.device)

    # -- compute
    def type1(self, x, y, h, w, out=None):
        self._pts(x, y, h, w)
        f = self.empty_modes() if out is None else out
        self._sync_stream()
        _check(self._lib.enufft_type1_batched(self._h, _ptr(x), _ptr(y), _ptr(h), _ptr(w), _ptr(f)), self._h)
        return f

    def type1_noalloc(self, x, y, h, w, out):
        """Batched type-1 through the allocation-free entry point: the forward's scratch
        comes from the library's fixed device array; out is a preallocated coefficient
        tensor (the call allocates nothing)."""
        self._pts(x, y, h, w)
        if out.dtype != self.cdtype or not out.is_contiguous() or out.shape != (self.n_cells,) + self.n_modes[::-1]:
            raise ValueError("out must be a contiguous %s tensor of shape %s" % (self.cdtype,
                                                                                (self.n_cells,) + self.n_modes[::-1]))
        self._sync_stream()
        _check(self._lib.enufft_type1_batched_noalloc(self._h, _ptr(x), _ptr(y), _ptr(h), _ptr(w), _ptr(out)),
               self._h)
        return out

    def ems(self, f, params: EmsParams = EmsParams(), mode_weight=None):
        if f.dtype != self.cdtype or not f.is_contiguous():
            raise ValueError("f must be contiguous %s" % self.cdtype)
        keep = torch.empty(f.shape, dtype=torch.uint8, device=self.device)
        ks = torch.empty(self.n_cells, dtype=torch.int32, device=self.device)
        st = torch.empty((self.n_cells, 8), dtype=torch.float64, device=self.device)
        mw = None
        if mode_weight is not None:
            mw = mode_weight.to(device=self.device, dtype=torch.float64).contiguous()
        prm = params.c()
        self._sync_stream()
        _check(self._lib.enufft_ems(self._h, _ptr(f), ctypes.byref(prm), _ptr(mw), _ptr(keep), _ptr(ks), _ptr(st)),
               self._h)
        return keep, ks, st

    def ems_flow(self, f, flow, params: EmsParams = EmsParams(), need_keep=True):
        """EMS per timestep under flow-dependent launch weights (Appendix A7) on fixed
        coefficients.  flow: float64 [n_steps, n_cells, 6] records (ux, uy, N, fc, rho,
        kscale).  Returns (keep [n_steps, n_cells, N2, N1] or None, k_star [n_steps,
        n_cells], stats [n_steps, n_cells, 8])."""
        if f.dtype != self.cdtype or not f.is_contiguous():
            raise ValueError("f must be contiguous %s" % self.cdtype)
        fl = torch.as_tensor(flow, dtype=torch.float64, device=self.device).contiguous()
        if fl.dim() != 3 or fl.shape[1] != self.n_cells or fl.shape[2] != 6:
            raise ValueError("flow must be [n_steps, n_cells, 6]")
        T = fl.shape[0]
        keep = torch.empty((T,) + tuple(f.shape), dtype=torch.uint8, device=self.device) if need_keep else None
        ks = torch.empty((T, self.n_cells), dtype=torch.int32, device=self.device)
        st = torch.empty((T, self.n_cells, 8), dtype=torch.float64, device=self.device)
        prm = params.c()
        self._sync_stream()
        _check(self._lib.enufft_ems_flow(self._h, _ptr(f), ctypes.byref(prm), int(T), _ptr(fl), _ptr(keep), _ptr(ks),
                                         _ptr(st)), self._h)
        return keep, ks, st

    def adjoint(self, x, y, h, w, fbar, need=(True, True, True)):
        self._pts(x, y, h, w)
        if fbar.dtype != self.cdtype or not fbar.is_contiguous():
            raise ValueError("fbar must be contiguous %s" % self.cdtype)
        outs = [torch.empty(self.n_points, dtype=self.dtype, device=self.device) if n else None for n in need]
        self._sync_stream()
        _check(self._lib.enufft_type1_adjoint(self._h, _ptr(x), _ptr(y), _ptr(h), _ptr(w), _ptr(fbar),
                                              _ptr(outs[0]), _ptr(outs[1]), _ptr(outs[2])), self._h)
        return tuple(outs)

    def retained_power_adjoint(self, x, y, h, w, f, keep, lam=None, need=(True, True, True)):
        """Gradients of sum_c lam_c P_c (kept set fixed); the cotangent is formed in-kernel."""
        self._pts(x, y, h, w)
        if f.dtype != self.cdtype or not f.is_contiguous() or keep.dtype != torch.uint8:
            raise ValueError("f must be contiguous %s and keep uint8" % self.cdtype)
        lam_t = None if lam is None else lam.to(device=self.device, dtype=torch.float64).contiguous()
        outs = [torch.empty(self.n_points, dtype=self.dtype, device=self.device) if n else None for n in need]
        self._sync_stream()
        _check(self._lib.enufft_retained_power_adjoint(self._h, _ptr(x), _ptr(y), _ptr(h), _ptr(w), _ptr(f),
                                                       _ptr(keep.contiguous()), _ptr(lam_t), _ptr(outs[0]),
                                                       _ptr(outs[1]), _ptr(outs[2])), self._h)
        return tuple(outs)

    def reconstruct(self, x, y, h, w, coef, keep=None, area=None, need_h_rec=True):
        """Truncated-series reconstruction over the kept modes and the Section 3.2
        diagnostics per cell -> (h_rec or None, diag float64 [n_cells, 8]); diag columns:
        Q_c, sum (t - h_rec)^2, sum t^2, sigma2_phys, sigma2_spec (k != 0), the same over
        kept modes, eps_rel, sigma2_spec / sigma2_phys (t = W h)."""
        self._pts(x, y, h, w)
        if coef.dtype != self.cdtype or not coef.is_contiguous():
            raise ValueError("coef must be contiguous %s" % self.cdtype)
        if keep is not None and keep.dtype != torch.uint8:
            raise ValueError("keep must be uint8")
        ar = None if area is None else torch.as_tensor(area, dtype=torch.float64, device=self.device).contiguous()
        hr = torch.empty(self.n_points, dtype=self.dtype, device=self.device) if need_h_rec else None
        dg = torch.empty((self.n_cells, 8), dtype=torch.float64, device=self.device)
        self._sync_stream()
        _check(self._lib.enufft_reconstruct(self._h, _ptr(x), _ptr(y), _ptr(h), _ptr(w), _ptr(coef),
                                            _ptr(None if keep is None else keep.contiguous()), _ptr(ar), _ptr(hr),
                                            _ptr(dg)), self._h)
        return hr, dg

    def sort_points(self, x, y, h=None, w=None, need_perm=True):
        """Sorted copies of the samples, every cell ordered by the fine cell its kernel
        footprint starts in (enufft_sort_points) -> (xs, ys, hs, ws, perm); hs / ws are
        None when h / w are, perm int32 (input index of each sorted sample) or None."""
        for v in (x, y, h, w):
            if v is None:
                continue
            if v.dtype != self.dtype or v.device != self.device or not v.is_contiguous() or v.numel() != self.n_points:
                raise ValueError("x, y, h, w must be contiguous %s of length %d on %s"
                                 % (self.dtype, self.n_points, self.device))
        new = lambda: torch.empty(self.n_points, dtype=self.dtype, device=self.device)
        xs, ys = new(), new()
        hs = new() if h is not None else None
        ws = new() if w is not None else None
        perm = torch.empty(self.n_points, dtype=torch.int32, device=self.device) if need_perm else None
        self._sync_stream()
        _check(self._lib.enufft_sort_points(self._h, _ptr(x), _ptr(y), _ptr(h), _ptr(w), _ptr(xs), _ptr(ys),
                                            _ptr(hs), _ptr(ws), _ptr(perm)), self._h)
        return xs, ys, hs, ws, perm

    def bind_points(self, x, y):
        """Bind tile-ordered coordinates (enufft_bind_points): later type-1 and adjoint
        calls given these same tensors skip the large-cell tile sort.  Their contents must
        not change while bound.  None, None unbinds.  The tensors are kept referenced while
        bound, so their memory cannot be reused by others."""
        if (x is None) != (y is None):
            raise ValueError("x and y are both given (bind) or both None (unbind)")
        for v in (x, y):
            if v is not None and (v.dtype != self.dtype or v.device != self.device or not v.is_contiguous()
                                  or v.numel() != self.n_points):
                raise ValueError("x, y must be contiguous %s of length %d on %s"
                                 % (self.dtype, self.n_points, self.device))
        self._sync_stream()
        self._bound = None
        _check(self._lib.enufft_bind_points(self._h, _ptr(x), _ptr(y)), self._h)
        self._bound = (x, y) if x is not None else None

    def unbind_points(self):
        """Drop a binding made by bind_points."""
        self.bind_points(None, None)

    def cell_geometry(self, tri, x, y, h, frame="edge", mask="triangle", weights="uniform", raster=64, eta=1.0,
                      floor_frac=0.5, deplane=True, need_inside=True, need_info=True, need_counts=False):
        """Local frames, masks, quadrature weights and deplaning of a triangular mesh
        (Appendices A1, A2, A6) -> dict of device tensors xb, yb, hb, wb (the plan's
        precision; wb = w_q / |D|), inside (uint8), info float64 [n_cells, 8] = (xbar_x,
        xbar_y, cos, sin, H, |D|, Q_in, hbar), counts (int32 raster points per sample)."""
        tri = torch.as_tensor(tri, dtype=torch.float64, device=self.device).reshape(self.n_cells, 6).contiguous()
        for v in (x, y, h):
            if v.dtype != self.dtype or v.device != self.device or not v.is_contiguous() or v.numel() != self.n_points:
                raise ValueError("x, y, h must be contiguous %s of length %d on %s"
                                 % (self.dtype, self.n_points, self.device))
        o = GeometryOptsC(FRAMES[frame], MASKS[mask], WEIGHTS[weights], int(raster), float(eta), float(floor_frac),
                          int(bool(deplane)), 0)
        out = {k: torch.empty(self.n_points, dtype=self.dtype, device=self.device) for k in ("xb", "yb", "hb", "wb")}
        out["inside"] = torch.empty(self.n_points, dtype=torch.uint8, device=self.device) if need_inside else None
        out["info"] = torch.empty((self.n_cells, 8), dtype=torch.float64, device=self.device) if need_info else None
        out["counts"] = torch.empty(self.n_points, dtype=torch.int32, device=self.device) if need_counts else None
        self._sync_stream()
        _check(self._lib.enufft_cell_geometry(self._h, _ptr(tri), _ptr(x), _ptr(y), _ptr(h), ctypes.byref(o),
                                              _ptr(out["xb"]), _ptr(out["yb"]), _ptr(out["hb"]), _ptr(out["wb"]),
                                              _ptr(out["inside"]), _ptr(out["info"]), _ptr(out["counts"])), self._h)
        return out

    def percell_loop(self, x, y, h, w, params: EmsParams | None = EmsParams(), mode_weight=None):
        self._pts(x, y, h, w)
        f = self.empty_modes()
        keep = torch.empty(f.shape, dtype=torch.uint8, device=self.device)
        ks = torch.empty(self.n_cells, dtype=torch.int32, device=self.device)
        st = torch.empty((self.n_cells, 8), dtype=torch.float64, device=self.device)
        prm = params.c() if params is not None else None
        mw = None if mode_weight is None else mode_weight.to(device=self.device, dtype=torch.float64).contiguous()
        self._sync_stream()
        _check(self._lib.enufft_percell_loop(self._h, _ptr(x), _ptr(y), _ptr(h), _ptr(w), _ptr(f),
                                             ctypes.byref(prm) if prm is not None else None, _ptr(mw),
                                             _ptr(keep), _ptr(ks), _ptr(st)), self._h)
        return f, keep, ks, st

    def forward_graph(self, x, y, h, w, params: EmsParams = EmsParams(), out=None, mode_weight=None):
        """Type-1 + EMS replayed as one captured HIP graph.  Reusing the same output
        tensors (pass ``out=(f, keep, k_star, stats)``) replays without re-capture."""
        self._pts(x, y, h, w)
        if out is None:
            f = self.empty_modes()
            keep = torch.empty(f.shape, dtype=torch.uint8, device=self.device)
            ks = torch.empty(self.n_cells, dtype=torch.int32, device=self.device)
            st = torch.empty((self.n_cells, 8), dtype=torch.float64, device=self.device)
        else:
            f, keep, ks, st = out
        mw = None if mode_weight is None else mode_weight.to(device=self.device, dtype=torch.float64).contiguous()
        prm = params.c()
        self._sync_stream()
        _check(self._lib.enufft_forward_graph(self._h, _ptr(x), _ptr(y), _ptr(h), _ptr(w), _ptr(f), ctypes.byref(prm),
                                              _ptr(mw), _ptr(keep), _ptr(ks), _ptr(st)), self._h)
        return f, keep, ks, st

    def set_timing(self, enable: bool):
        _check(self._lib.enufft_set_timing(self._h, int(enable)), self._h)

    def get_timing(self) -> dict:
        out = (ctypes.c_double * 8)()
        _check(self._lib.enufft_get_timing(self._h, out), self._h)
        return {"type1_ms": out[0], "ems_ms": out[1], "adjoint_ms": out[2], "graph_ms": out[3],
                "type1_launches": int(out[4]), "ems_launches": int(out[5]), "adjoint_launches": int(out[6]),
                "graph_launches": int(out[7])}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.enufft_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class RetainedPower(torch.autograd.Function):
    """P_c = sum over the EMS-kept modes of |f_c[k]|^2, with f = plan.type1(x, y, h, w).

    Forward: batched type-1 then EMS.  Backward: the type-2 adjoint with cotangent
    2 dL/dP_c f keep (the kept set, the weights and the windows are held fixed), giving
    gradients for h, x and y; w gets None."""

    @staticmethod
    def forward(ctx, x, y, h, w, plan: Plan, params: EmsParams = EmsParams()):
        f = plan.type1(x, y, h, w)
        keep, ks, st = plan.ems(f, params)
        ctx.plan = plan
        ctx.save_for_backward(x, y, h, w, f, keep)
        ctx.mark_non_differentiable(keep, ks)
        return st[:, 1].clone(), keep, ks

    @staticmethod
    def backward(ctx, gP, gkeep=None, gks=None):
        x, y, h, w, f, keep = ctx.saved_tensors
        plan = ctx.plan
        need = (ctx.needs_input_grad[2], ctx.needs_input_grad[0], ctx.needs_input_grad[1])
        gh, gx, gy = plan.retained_power_adjoint(x, y, h, w, f, keep, lam=gP, need=need)
        return gx, gy, gh, None, None, None


def retained_power(x, y, h, w, plan: Plan, params: EmsParams = EmsParams()):
    """Differentiable retained power per cell (float64 [n_cells])."""
    P, _, _ = RetainedPower.apply(x, y, h, w, plan, params)
    return P
