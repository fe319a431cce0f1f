"""Seeded synthetic inputs for the ENUFFT hot path.

This module is shared by the oracle side and the GPU side and holds none of
the method's arithmetic: it only draws point sets, terrain heights, quadrature
weights and window parameters.  The paper's own data (SRTM DEM tiles, the
monochromatic sweep generator, the PinCFlow runs) are not available, so these
workloads stand in for them, with the shapes described in the paper's setup
(Section 2.1: per-cell scattered samples {x_q, y_q, h_q} with quadrature
weights w_q; Appendix A1: local square spectral box; Appendix A2: uniform
weights |D|/Q).

Seeding.  Per-cell scalars (point counts, sinusoid wave vectors, amplitudes,
phases, spectral slopes, standard deviations) come from numpy PCG64 seeded by
``1000 * config + cell``, so they do not depend on the device or on cell
order.  Bulk per-point draws (positions, jitter, dropout, noise) come from a
``torch.Generator`` on the requested device seeded by ``1000 * config + 7``;
on the CPU and on the GPU they therefore differ, but each is reproducible.

Coordinates are in local box units: the periodic box has side 2*pi, so mode
wave numbers are integers (Appendix A1 with L = 2H = 2*pi).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import torch

TWO_PI = 2.0 * math.pi


@dataclass
class Batch:
    """A batch of cells in CSR layout (points of cell c are [off[c], off[c+1]))."""
    name: str
    x: torch.Tensor
    y: torch.Tensor
    h: torch.Tensor
    w: torch.Tensor
    cell_offsets: np.ndarray          # int64 [n_cells + 1]
    windows: np.ndarray               # float64 [n_cells, 3] = (cx, cy, R)
    n_modes: tuple = (64, 64)
    sigma: float = 2.0
    eps: float = 1e-5
    precision: str = "f32"
    areas: np.ndarray = field(default=None)   # float64 [n_cells], analysis-domain area

    @property
    def n_cells(self) -> int:
        return len(self.cell_offsets) - 1

    @property
    def n_points(self) -> int:
        return int(self.cell_offsets[-1])

    def counts(self) -> np.ndarray:
        return np.diff(self.cell_offsets)

    def to(self, device=None, dtype=None) -> "Batch":
        conv = lambda t: t.to(device=device if device is not None else t.device,
                              dtype=dtype if dtype is not None else t.dtype)
        prec = self.precision
        if dtype is not None:
            prec = "f64" if dtype == torch.float64 else "f32"
        return Batch(self.name, conv(self.x), conv(self.y), conv(self.h), conv(self.w),
                     self.cell_offsets.copy(), self.windows.copy(), self.n_modes,
                     self.sigma, self.eps, prec, None if self.areas is None else self.areas.copy())

    def cell(self, c: int):
        """Host float64 copies (x, y, h, w) of one cell."""
        a, b = int(self.cell_offsets[c]), int(self.cell_offsets[c + 1])
        g = lambda t: t[a:b].detach().to("cpu", torch.float64).numpy()
        return g(self.x), g(self.y), g(self.h), g(self.w)

    def subset(self, cells) -> "Batch":
        """A new batch made of the listed cells (same order), on the same device."""
        cells = [int(c) for c in cells]
        segs = [(int(self.cell_offsets[c]), int(self.cell_offsets[c + 1])) for c in cells]
        dev = self.x.device
        idx = torch.cat([torch.arange(a, b, device=dev) for a, b in segs]) if segs else \
            torch.zeros(0, dtype=torch.long, device=dev)
        cnt = np.array([b - a for a, b in segs], dtype=np.int64)
        off = np.concatenate([[0], np.cumsum(cnt)]).astype(np.int64)
        return Batch(self.name + "[subset]", self.x[idx], self.y[idx], self.h[idx], self.w[idx],
                     off, self.windows[cells].copy(), self.n_modes, self.sigma, self.eps,
                     self.precision, None if self.areas is None else self.areas[cells].copy())


# --------------------------------------------------------------------------- geometry

def hexagon_vertices(R: float = math.pi) -> np.ndarray:
    """Regular hexagon of circumradius R centred at 0, vertices at 0, 60, ... degrees."""
    ang = np.arange(6) * (math.pi / 3.0)
    return np.stack([R * np.cos(ang), R * np.sin(ang)], axis=1)


def hexagon_area(R: float = math.pi) -> float:
    return 1.5 * math.sqrt(3.0) * R * R


def _inside_hexagon(x: torch.Tensor, y: torch.Tensor, R: float) -> torch.Tensor:
    # flat-topped? No: vertices at 0 deg -> pointy along x.  |y| <= R*sqrt(3)/2 and
    # sqrt(3)|x| + |y| <= sqrt(3) R.
    s3 = math.sqrt(3.0)
    return (y.abs() <= R * s3 / 2.0) & (s3 * x.abs() + y.abs() <= s3 * R)


def icosphere_faces(level: int) -> np.ndarray:
    """Triangles of an icosahedron subdivided ``level`` times on the unit sphere.

    Returns float64 [20 * 4**level, 3, 3] (face, vertex, xyz).
    """
    t = (1.0 + math.sqrt(5.0)) / 2.0
    v = np.array([[-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0],
                  [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
                  [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1]], dtype=np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    f = np.array([[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
                  [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
                  [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
                  [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]])
    tri = v[f]
    for _ in range(level):
        a, b, c = tri[:, 0], tri[:, 1], tri[:, 2]
        ab = a + b; ab /= np.linalg.norm(ab, axis=1, keepdims=True)
        bc = b + c; bc /= np.linalg.norm(bc, axis=1, keepdims=True)
        ca = c + a; ca /= np.linalg.norm(ca, axis=1, keepdims=True)
        tri = np.concatenate([np.stack([a, ab, ca], 1), np.stack([ab, b, bc], 1),
                              np.stack([ca, bc, c], 1), np.stack([ab, bc, ca], 1)], 0)
    return tri


def local_triangles(level: int = 5) -> np.ndarray:
    """Icosahedral faces mapped to local tangent-plane triangles.

    Each face is projected orthographically onto the tangent plane at its
    centroid, rotated so its longest edge is parallel to x (the edge-aligned
    frame of Appendix A1), scaled so the longest edge is 2*pi, and shifted so
    its bounding box is centred at the origin.  Returns float64 [F, 3, 2].
    """
    tri = icosphere_faces(level)
    cen = tri.mean(axis=1)
    nrm = cen / np.linalg.norm(cen, axis=1, keepdims=True)
    ref = np.where(np.abs(nrm[:, 2:3]) < 0.9, np.array([[0.0, 0.0, 1.0]]), np.array([[1.0, 0.0, 0.0]]))
    e1 = np.cross(ref, nrm); e1 /= np.linalg.norm(e1, axis=1, keepdims=True)
    e2 = np.cross(nrm, e1)
    d = tri - cen[:, None, :]
    p = np.stack([(d * e1[:, None, :]).sum(-1), (d * e2[:, None, :]).sum(-1)], axis=-1)  # [F,3,2]
    edges = np.stack([p[:, 1] - p[:, 0], p[:, 2] - p[:, 1], p[:, 0] - p[:, 2]], axis=1)
    L = np.linalg.norm(edges, axis=-1)
    emax = edges[np.arange(len(p)), np.argmax(L, axis=1)]
    Lmax = L.max(axis=1)
    cth, sth = emax[:, 0] / Lmax, emax[:, 1] / Lmax
    # rotation R = [[c, s], [-s, c]] applied to centroid-relative coordinates
    pc = p - p.mean(axis=1, keepdims=True)
    u = np.stack([cth[:, None] * pc[..., 0] + sth[:, None] * pc[..., 1],
                  -sth[:, None] * pc[..., 0] + cth[:, None] * pc[..., 1]], axis=-1)
    u *= (TWO_PI / Lmax)[:, None, None]
    lo, hi = u.min(axis=1), u.max(axis=1)
    u -= ((lo + hi) / 2.0)[:, None, :]
    return u


def triangle_area(t: np.ndarray) -> np.ndarray:
    a, b, c = t[..., 0, :], t[..., 1, :], t[..., 2, :]
    return 0.5 * np.abs((b[..., 0] - a[..., 0]) * (c[..., 1] - a[..., 1])
                        - (c[..., 0] - a[..., 0]) * (b[..., 1] - a[..., 1]))


# --------------------------------------------------------------------------- terrain

@dataclass
class Terrain:
    """Per-cell sinusoid set: h = sum_i a_i cos(k_i . x + phi_i), rescaled, plus noise."""
    kx: np.ndarray      # [n_cells, S]
    ky: np.ndarray
    amp: np.ndarray
    phase: np.ndarray
    std: np.ndarray     # [n_cells] target standard deviation (m)
    noise: float        # additive N(0, noise) in m


def _draw_terrain(rng: np.random.Generator, S: int, kmax: float, slope: float):
    # |k| area-uniform on the annulus 1 <= |k| <= kmax, so that a = |k|^-slope gives a
    # 2D power spectrum proportional to |k|^(-2 slope).
    kmag = np.sqrt(rng.uniform(1.0, kmax * kmax, size=S))
    th = rng.uniform(0.0, TWO_PI, size=S)
    ph = rng.uniform(0.0, TWO_PI, size=S)
    return kmag * np.cos(th), kmag * np.sin(th), kmag ** (-slope), ph


def _eval_terrain(x: torch.Tensor, y: torch.Tensor, cell_of: torch.Tensor, terr: Terrain,
                  offsets: np.ndarray, gen: torch.Generator, chunk: int = 1 << 20, progress=None) -> torch.Tensor:
    """Evaluate the sinusoid sums (float64), rescale per cell to the target std, add noise."""
    dev = x.device
    kx = torch.as_tensor(terr.kx, device=dev)
    ky = torch.as_tensor(terr.ky, device=dev)
    am = torch.as_tensor(terr.amp, device=dev)
    ph = torch.as_tensor(terr.phase, device=dev)
    n = x.numel()
    raw = torch.empty(n, dtype=torch.float64, device=dev)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        c = cell_of[s:e]
        xx = x[s:e].to(torch.float64)[:, None]
        yy = y[s:e].to(torch.float64)[:, None]
        arg = xx * kx[c] + yy * ky[c] + ph[c]
        raw[s:e] = (torch.cos(arg) * am[c]).sum(dim=1)
        if progress and (s // chunk) % 128 == 127:
            progress("heights: %d of %d points" % (e, n))
    cnt = torch.as_tensor(np.diff(offsets), device=dev, dtype=torch.float64)
    mean = _segment_sum(raw, offsets) / cnt.clamp(min=1)
    dev2 = (raw - mean[cell_of]) ** 2
    var = _segment_sum(dev2, offsets) / cnt.clamp(min=1)
    scale = torch.as_tensor(terr.std, device=dev) / var.sqrt().clamp(min=1e-300)
    h = raw * scale[cell_of]
    h += terr.noise * torch.randn(n, dtype=torch.float64, device=dev, generator=gen)
    return h


def _segment_sum(v: torch.Tensor, offsets: np.ndarray, chunk: int = 1 << 24) -> torch.Tensor:
    """Per-cell sums of a cell-contiguous array (chunked prefix sums; no atomics)."""
    dev = v.device
    n_cells = len(offsets) - 1
    off = torch.as_tensor(offsets, device=dev)
    out = torch.zeros(n_cells, dtype=torch.float64, device=dev)
    for s in range(0, v.numel(), chunk):
        e = min(v.numel(), s + chunk)
        ps = torch.zeros(e - s + 1, dtype=torch.float64, device=dev)
        ps[1:] = torch.cumsum(v[s:e].to(torch.float64), 0)
        # the part of every cell inside [s, e)
        a = off[:-1].clamp(s, e) - s
        b = off[1:].clamp(s, e) - s
        out += ps[b] - ps[a]
    return out


def _cell_index(offsets: np.ndarray, device) -> torch.Tensor:
    cnt = torch.as_tensor(np.diff(offsets), device=device)
    return torch.repeat_interleave(torch.arange(len(cnt), device=device), cnt)


def _finish(name, x, y, h, offsets, areas, windows, n_modes, sigma, eps, precision) -> Batch:
    dt = torch.float64 if precision == "f64" else torch.float32
    dev = x.device
    cnt = np.diff(offsets)
    wq = torch.as_tensor(areas / np.maximum(cnt, 1), device=dev, dtype=torch.float64)
    w = torch.repeat_interleave(wq, torch.as_tensor(cnt, device=dev))
    return Batch(name, x.to(dt).contiguous(), y.to(dt).contiguous(), h.to(dt).contiguous(),
                 w.to(dt).contiguous(), offsets.astype(np.int64), windows.astype(np.float64),
                 tuple(n_modes), float(sigma), float(eps), precision, areas.astype(np.float64))


# --------------------------------------------------------------------------- hexagon cells

def _uniform_in_hexagon(counts: np.ndarray, R: float, gen: torch.Generator, device) -> tuple:
    """Uniform points in the hexagon by rejection, cell-contiguous, counts[c] per cell."""
    n_cells = len(counts)
    cand = np.ceil(counts * 1.5).astype(np.int64) + 256       # acceptance ratio is 3/4
    coff = np.concatenate([[0], np.cumsum(cand)])
    tot = int(coff[-1])
    ux = (torch.rand(tot, dtype=torch.float64, device=device, generator=gen) * 2 - 1) * R
    uy = (torch.rand(tot, dtype=torch.float64, device=device, generator=gen) * 2 - 1) * (R * math.sqrt(3) / 2)
    acc = _inside_hexagon(ux, uy, R)
    cell_of = torch.repeat_interleave(torch.arange(n_cells, device=device), torch.as_tensor(cand, device=device))
    idx = torch.nonzero(acc).flatten()
    ac_cell = cell_of[idx]
    first = torch.zeros(n_cells + 1, dtype=torch.long, device=device)
    first[1:] = torch.cumsum(torch.bincount(ac_cell, minlength=n_cells), 0)
    rank = torch.arange(idx.numel(), device=device) - first[ac_cell]
    keep = rank < torch.as_tensor(counts, device=device)[ac_cell]
    if int(keep.sum()) != int(counts.sum()):
        raise RuntimeError("rejection sampling ran short; raise the oversampling factor")
    sel = idx[keep]
    return ux[sel], uy[sel]


def config0(device="cpu", precision: str = "f64", Q: int = 2000, seed_config: int = 0) -> Batch:
    """One hexagon (circumradius pi), Q uniform points, 200-sinusoid |k|^-1.5 terrain with
    std 500 m plus N(0, 5 m) noise, weights area/Q, radial Hann over the circumradius,
    32 x 32 modes."""
    R = math.pi
    rng = np.random.Generator(np.random.PCG64(1000 * seed_config + 0))
    kx, ky, am, ph = _draw_terrain(rng, 200, 40.0, 1.5)
    terr = Terrain(kx[None], ky[None], am[None], ph[None], np.array([500.0]), 5.0)
    gen = torch.Generator(device=device).manual_seed(1000 * seed_config + 7)
    counts = np.array([Q], dtype=np.int64)
    x, y = _uniform_in_hexagon(counts, R, gen, device)
    off = np.array([0, Q], dtype=np.int64)
    h = _eval_terrain(x, y, _cell_index(off, device), terr, off, gen)
    win = np.array([[0.0, 0.0, R]])
    return _finish("C0 one hexagon Q=%d" % Q, x, y, h, off, np.array([hexagon_area(R)]), win,
                   (32, 32), 2.0, 1e-10 if precision == "f64" else 1e-5, precision)


def lognormal_counts(rng: np.random.Generator, n: int, median: float, s: float, lo: int, hi: int):
    return np.clip(np.round(rng.lognormal(math.log(median), s, size=n)), lo, hi).astype(np.int64)


def config1(device="cpu", n_cells: int = 256, count_scale: float = 1.0, seed_config: int = 1,
            precision: str = "f32") -> Batch:
    """256 hexagons, lognormal counts (median 2e4, sigma 1.0, clipped 2e3..2e5), per-cell
    slope U(1.25, 1.75) and std U(100, 1500) m, weights area/Q_c, Hann, 64 x 64 modes.

    ``count_scale`` shrinks every count (for oracle-sized tests); the default is the
    full workload."""
    R = math.pi
    rng0 = np.random.Generator(np.random.PCG64(1000 * seed_config))
    counts = lognormal_counts(rng0, n_cells, 2.0e4, 1.0, 2000, 200000)
    counts = np.maximum(1, np.round(counts * count_scale)).astype(np.int64)
    S = 200
    KX = np.zeros((n_cells, S)); KY = np.zeros_like(KX); AM = np.zeros_like(KX); PH = np.zeros_like(KX)
    STD = np.zeros(n_cells)
    for c in range(n_cells):
        rng = np.random.Generator(np.random.PCG64(1000 * seed_config + c + 1))
        slope = rng.uniform(1.25, 1.75)
        STD[c] = rng.uniform(100.0, 1500.0)
        KX[c], KY[c], AM[c], PH[c] = _draw_terrain(rng, S, 40.0, slope)
    terr = Terrain(KX, KY, AM, PH, STD, 5.0)
    gen = torch.Generator(device=device).manual_seed(1000 * seed_config + 7)
    x, y = _uniform_in_hexagon(counts, R, gen, device)
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    h = _eval_terrain(x, y, _cell_index(off, device), terr, off, gen)
    win = np.tile(np.array([[0.0, 0.0, R]]), (n_cells, 1))
    areas = np.full(n_cells, hexagon_area(R))
    return _finish("C1 %d hexagons" % n_cells, x, y, h, off, areas, win, (64, 64), 2.0, 1e-5, precision)


def fd_sample(batch: Batch, n_cells: int = 8, n_points: int = 64, seed: int = 2002):
    """Seeded choice of cells and points for finite-difference checks: returns
    (cells [n_cells], points [n_cells, n_points]) with point indices local to each cell."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cnt = batch.counts()
    cells = rng.choice(np.nonzero(cnt >= n_points)[0], size=n_cells, replace=False)
    pts = np.stack([rng.choice(int(cnt[c]), size=n_points, replace=False) for c in cells])
    return cells, pts


# --------------------------------------------------------------------------- icosahedral cells

def config3(device="cpu", n_cells: int | None = None, count_scale: float = 1.0, seed_config: int = 3,
            precision: str = "f32", shuffled: bool = False, chunk_candidates: int = 1 << 27,
            progress=None) -> Batch:
    """20,480 triangles of a 5x subdivided icosahedron in local tangent-plane frames (longest
    edge 2*pi), lognormal counts (median 2e4, sigma 1.2, clipped 500..5e5), jittered square
    lattice (spacing sqrt(0.7 area / Q_c), jitter +-0.25 spacing, 30 % dropout, raster order),
    heights as config 1, weights area/N_c, Hann centred on the centroid with R = max
    centroid-vertex distance, 64 x 64 modes.

    ``n_cells`` keeps the first n cells (same per-cell data as the full set).  ``progress``,
    if given, is called with a short text after each generation chunk."""
    tris = local_triangles(5)
    F = len(tris)
    rng0 = np.random.Generator(np.random.PCG64(1000 * seed_config))
    counts_all = lognormal_counts(rng0, F, 2.0e4, 1.2, 500, 500000)
    if n_cells is None:
        n_cells = F
    tris = tris[:n_cells]
    target = np.maximum(1, np.round(counts_all[:n_cells] * count_scale)).astype(np.int64)
    area = triangle_area(tris)
    S = 200
    KX = np.zeros((n_cells, S)); KY = np.zeros_like(KX); AM = np.zeros_like(KX); PH = np.zeros_like(KX)
    STD = np.zeros(n_cells)
    for c in range(n_cells):
        rng = np.random.Generator(np.random.PCG64(1000 * seed_config + c + 1))
        slope = rng.uniform(1.25, 1.75)
        STD[c] = rng.uniform(100.0, 1500.0)
        KX[c], KY[c], AM[c], PH[c] = _draw_terrain(rng, S, 40.0, slope)
    terr = Terrain(KX, KY, AM, PH, STD, 5.0)
    gen = torch.Generator(device=device).manual_seed(1000 * seed_config + 7)

    spacing = np.sqrt(area * 0.7 / target)
    lo = tris.min(axis=1); hi = tris.max(axis=1)
    nx = np.ceil((hi[:, 0] - lo[:, 0]) / spacing).astype(np.int64) + 1
    ny = np.ceil((hi[:, 1] - lo[:, 1]) / spacing).astype(np.int64) + 1
    ncand = nx * ny
    xs, ys, cnts = [], [], np.zeros(n_cells, dtype=np.int64)
    c0 = 0
    while c0 < n_cells:
        c1 = c0
        tot = 0
        while c1 < n_cells and (tot + ncand[c1] <= chunk_candidates or c1 == c0):
            tot += int(ncand[c1]); c1 += 1
        cc = torch.arange(c0, c1, device=device)
        cand = torch.as_tensor(ncand[c0:c1], device=device)
        cell_of = torch.repeat_interleave(cc, cand)
        start = torch.zeros(c1 - c0 + 1, dtype=torch.long, device=device)
        start[1:] = torch.cumsum(cand, 0)
        local = torch.arange(tot, device=device) - start[cell_of - c0]
        nxt = torch.as_tensor(nx, device=device)[cell_of]
        iy = torch.div(local, nxt, rounding_mode="floor")
        ix = local - iy * nxt
        sp = torch.as_tensor(spacing, device=device)[cell_of]
        lx = torch.as_tensor(lo[:, 0], device=device)[cell_of]
        ly = torch.as_tensor(lo[:, 1], device=device)[cell_of]
        jx = (torch.rand(tot, dtype=torch.float64, device=device, generator=gen) - 0.5) * 0.5
        jy = (torch.rand(tot, dtype=torch.float64, device=device, generator=gen) - 0.5) * 0.5
        px = lx + (ix.to(torch.float64) + 0.5 + jx) * sp
        py = ly + (iy.to(torch.float64) + 0.5 + jy) * sp
        T = torch.as_tensor(tris, device=device)[cell_of]          # [tot, 3, 2]
        inside = torch.ones(tot, dtype=torch.bool, device=device)
        sgn = None
        for e in range(3):
            a = T[:, e]; b = T[:, (e + 1) % 3]
            cr = (b[:, 0] - a[:, 0]) * (py - a[:, 1]) - (b[:, 1] - a[:, 1]) * (px - a[:, 0])
            if sgn is None:
                o = T[:, 2]
                sgn = torch.sign((b[:, 0] - a[:, 0]) * (o[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (o[:, 0] - a[:, 0]))
            inside &= (cr * sgn) >= 0
        keep = inside & (torch.rand(tot, dtype=torch.float64, device=device, generator=gen) >= 0.3)
        xs.append(px[keep]); ys.append(py[keep])
        cnts[c0:c1] = torch.bincount(cell_of[keep] - c0, minlength=c1 - c0).cpu().numpy()
        del T, px, py, jx, jy, local, cell_of
        c0 = c1
        if progress:
            progress("positions: %d of %d cells" % (c1, n_cells))
    x = torch.cat(xs); y = torch.cat(ys)
    off = np.concatenate([[0], np.cumsum(cnts)]).astype(np.int64)
    if shuffled:
        ci = _cell_index(off, device)
        key = ci.to(torch.float64) + torch.rand(x.numel(), dtype=torch.float64, device=device, generator=gen) * 0.5
        perm = torch.argsort(key)
        x, y = x[perm], y[perm]
    h = _eval_terrain(x, y, _cell_index(off, device), terr, off, gen, progress=progress)
    cen = tris.mean(axis=1)
    Rw = np.linalg.norm(tris - cen[:, None, :], axis=-1).max(axis=1)
    win = np.concatenate([cen, Rw[:, None]], axis=1)
    return _finish("C3 %d icosahedral triangles" % n_cells, x, y, h, off, area, win, (64, 64), 2.0, 1e-5, precision)


def config4(device="cpu", Q: int = 100_000_000, precision: str = "f32", n_modes=(512, 512),
            seed_config: int = 4, chunk: int = 1 << 24, progress=None) -> Batch:
    """One hexagon (circumradius pi) with Q points: 30 % uniform background, 70 % from a
    4-component isotropic Gaussian mixture (means area-uniform within radius 0.6 pi, sd
    U(0.1, 0.4), weights Dirichlet(1)), draws outside the hexagon redrawn; heights from 400
    sinusoids with |k| area-uniform in [1, 400] and amplitude |k|^-1.5, std 1,000 m, no
    noise; weights = bin area / points in the bin of a 256 x 256 histogram over
    [-pi, pi]^2 (inverse local density); radial Hann over the circumradius; 512 x 512
    modes, sigma 2, eps 1e-5 (FP32) or 1e-10 (FP64).  Positions are drawn in chunks of
    ``chunk`` candidates so memory stays bounded at Q = 1e8."""
    R = math.pi
    rng = np.random.Generator(np.random.PCG64(1000 * seed_config + 0))
    kx, ky, am, ph = _draw_terrain(rng, 400, 400.0, 1.5)
    terr = Terrain(kx[None], ky[None], am[None], ph[None], np.array([1000.0]), 0.0)
    rm = 0.6 * R * np.sqrt(rng.uniform(0.0, 1.0, size=4))
    tm = rng.uniform(0.0, TWO_PI, size=4)
    means = np.stack([rm * np.cos(tm), rm * np.sin(tm)], axis=1)
    sds = rng.uniform(0.1, 0.4, size=4)
    wts = rng.dirichlet(np.ones(4))
    n_bg = int(round(0.3 * Q))
    n_comp = rng.multinomial(Q - n_bg, wts)
    gen = torch.Generator(device=device).manual_seed(1000 * seed_config + 7)
    xs, ys = [], []
    if n_bg > 0:
        bx, by = _uniform_in_hexagon(np.array([n_bg], dtype=np.int64), R, gen, device)
        xs.append(bx); ys.append(by)
    for m in range(4):
        need = int(n_comp[m])
        while need > 0:
            nc = min(chunk, int(need * 1.3) + 1024)
            px = torch.randn(nc, dtype=torch.float64, device=device, generator=gen) * sds[m] + means[m, 0]
            py = torch.randn(nc, dtype=torch.float64, device=device, generator=gen) * sds[m] + means[m, 1]
            ok = torch.nonzero(_inside_hexagon(px, py, R)).flatten()[:need]
            xs.append(px[ok]); ys.append(py[ok])
            need -= ok.numel()
        if progress:
            progress("positions: component %d of 4" % (m + 1))
    x = torch.cat(xs); y = torch.cat(ys)
    del xs, ys
    off = np.array([0, Q], dtype=np.int64)
    h = _eval_terrain(x, y, torch.zeros(Q, dtype=torch.long, device=device), terr, off, gen, progress=progress)
    nb = 256
    bw = TWO_PI / nb
    ix = torch.clamp(torch.floor((x + R) / bw).to(torch.long), 0, nb - 1)
    iy = torch.clamp(torch.floor((y + R) / bw).to(torch.long), 0, nb - 1)
    b = iy * nb + ix
    cnt = torch.bincount(b, minlength=nb * nb).to(torch.float64)
    w = (bw * bw) / cnt[b]
    dt = torch.float64 if precision == "f64" else torch.float32
    return Batch("C4 one hexagon Q=%d clustered" % Q, x.to(dt).contiguous(), y.to(dt).contiguous(),
                 h.to(dt).contiguous(), w.to(dt).contiguous(), off, np.array([[0.0, 0.0, R]]),
                 tuple(n_modes), 2.0, 1e-10 if precision == "f64" else 1e-5, precision,
                 np.array([hexagon_area(R)]))


def uniform_box(device="cpu", counts=(1000,), n_modes=(16, 16), seed: int = 11, precision: str = "f64",
                lo: float = -math.pi, hi: float = math.pi, window_radius: float = 0.0) -> Batch:
    """Plain uniform points on a square, heights N(0,1), weights box-area/Q.  With
    window_radius <= 0 the windows are 'none' (radius 0 marks no window)."""
    gen = torch.Generator(device=device).manual_seed(seed)
    counts = np.asarray(counts, dtype=np.int64)
    n = int(counts.sum())
    x = lo + (hi - lo) * torch.rand(n, dtype=torch.float64, device=device, generator=gen)
    y = lo + (hi - lo) * torch.rand(n, dtype=torch.float64, device=device, generator=gen)
    h = torch.randn(n, dtype=torch.float64, device=device, generator=gen)
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    win = np.tile(np.array([[0.5 * (lo + hi), 0.5 * (lo + hi), window_radius]]), (len(counts), 1))
    areas = np.full(len(counts), (hi - lo) ** 2)
    return _finish("uniform box", x, y, h, off, areas, win, n_modes, 2.0,
                   1e-10 if precision == "f64" else 1e-5, precision)


def square_terrain(device="cpu", Q: int = 2000, n_modes=(41, 41), seed: int = 0, precision: str = "f64") -> Batch:
    """One square cell (the whole 2 pi box), Q uniform points, 200-sinusoid power-law
    terrain (|k| area-uniform in [1, 20], amplitude |k|^-1.5, std 500 m), weights
    box-area/Q, no window: the setting of the kernel comparison of Section 2.1.2 (a
    rectangular domain of 2,000 samples, modes |m|, |n| <= 20), with seeded power-law
    terrains standing in for its three unspecified synthetic terrains."""
    rng = np.random.Generator(np.random.PCG64(1000 * 9 + seed))
    kx, ky, am, ph = _draw_terrain(rng, 200, 20.0, 1.5)
    terr = Terrain(kx[None], ky[None], am[None], ph[None], np.array([500.0]), 0.0)
    gen = torch.Generator(device=device).manual_seed(1000 * 9 + 7 + seed)
    x = -math.pi + TWO_PI * torch.rand(Q, dtype=torch.float64, device=device, generator=gen)
    y = -math.pi + TWO_PI * torch.rand(Q, dtype=torch.float64, device=device, generator=gen)
    off = np.array([0, Q], dtype=np.int64)
    h = _eval_terrain(x, y, _cell_index(off, device), terr, off, gen)
    win = np.array([[0.0, 0.0, 0.0]])
    return _finish("square terrain seed %d" % seed, x, y, h, off, np.array([TWO_PI * TWO_PI]), win, n_modes,
                   2.0, 1e-10 if precision == "f64" else 1e-5, precision)


def mesh_cells(device="cpu", n_cells: int = 24, count_scale: float = 0.05, seed: int = 31, precision: str = "f64",
               clustered: float = 0.0, n_modes=(32, 32)):
    """Triangular-mesh cells as a mesh pipeline hands them over: C3's first ``n_cells``
    triangles and samples, each cell turned by a seeded angle and moved by a seeded
    offset (so the local frames are not the identity).  With ``clustered`` > 0 that
    fraction of each cell's samples is redrawn around one seeded point of the
    triangle (normal spread 0.15), giving the strongly non-uniform sampling Voronoi
    weights are meant for.  Returns (Batch without windows, tri float64 [n_cells, 6])."""
    b = config3(n_cells=n_cells, count_scale=count_scale, precision="f64", seed_config=3)
    tris = local_triangles(5)[:n_cells]
    rng = np.random.Generator(np.random.PCG64(seed))
    th = rng.uniform(0.0, TWO_PI, n_cells)
    sh = rng.uniform(-5.0, 5.0, (n_cells, 2))
    off = b.cell_offsets
    x = b.x.numpy().copy()
    y = b.y.numpy().copy()
    for c in range(n_cells):
        a0, a1 = int(off[c]), int(off[c + 1])
        if clustered > 0 and a1 > a0:
            m = int(round(clustered * (a1 - a0)))
            bary = rng.dirichlet([2.0, 2.0, 2.0])
            p = bary @ tris[c]
            x[a0:a0 + m] = p[0] + rng.normal(scale=0.15, size=m)
            y[a0:a0 + m] = p[1] + rng.normal(scale=0.15, size=m)
    tri = np.zeros((n_cells, 6))
    cs, sn = np.cos(th), np.sin(th)
    cell = np.repeat(np.arange(n_cells), np.diff(off))
    xr = cs[cell] * x - sn[cell] * y + sh[cell, 0]
    yr = sn[cell] * x + cs[cell] * y + sh[cell, 1]
    for i in range(3):
        tri[:, 2 * i] = cs * tris[:, i, 0] - sn * tris[:, i, 1] + sh[:, 0]
        tri[:, 2 * i + 1] = sn * tris[:, i, 0] + cs * tris[:, i, 1] + sh[:, 1]
    dt = torch.float64 if precision == "f64" else torch.float32
    t = lambda v: torch.as_tensor(v, dtype=torch.float64).to(device=device, dtype=dt).contiguous()
    win = np.zeros((n_cells, 3))
    batch = Batch("mesh cells", t(xr), t(yr), t(b.h.numpy()), t(b.w.numpy()), off.copy(), win, tuple(n_modes), 2.0,
                  1e-10 if precision == "f64" else 1e-5, precision, b.areas.copy())
    return batch, tri
