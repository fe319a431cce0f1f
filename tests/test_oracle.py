"""Pins for the FP64 oracle: checks against facts the paper and the mathematics fix.

None of these re-types the oracle's own code path: they compare it with a
library routine (numpy.fft), closed forms, invariants, statistics with known
laws, brute force evaluated a different way, or finite differences.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth

RNG = np.random.default_rng(12345)
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _cell(Q, lo=-math.pi, hi=math.pi, rng=RNG):
    x = rng.uniform(lo, hi, Q)
    y = rng.uniform(lo, hi, Q)
    h = rng.normal(size=Q)
    w = rng.uniform(0.5, 1.5, Q)
    return x, y, h, w


def _modes(N):
    return np.arange(-(N // 2), -(N // 2) + N)


# ----------------------------------------------------------------------------- type 1

@pytest.mark.parametrize("N1,N2", [(4, 4), (5, 3), (1, 6)])
def test_type1_brute_force_dense_matrix(N1, N2):
    """Tiny inputs: f = C h with C_kq = w_q W_q exp(-i k.x_q) built as a dense complex
    matrix from numpy's complex exponential (matrix form of the quadrature sum,
    Appendix A5 eq. (enufft_matrix))."""
    Q = 9
    x, y, h, w = _cell(Q)
    win = np.array([0.3, -0.2, 2.9])
    f = oracle.type1([0, Q], x, y, h, w, win, (N1, N2), scale=0.37, kind=1)[0]
    W = np.array([oracle.hann(a, b, *win)[0] for a, b in zip(x, y)])
    KX, KY = np.meshgrid(_modes(N1), _modes(N2))
    C = 0.37 * np.exp(-1j * (KX.reshape(-1, 1) * x[None, :] + KY.reshape(-1, 1) * y[None, :])) * (w * W)[None, :]
    ref = (C @ h).reshape(N2, N1)
    assert np.abs(f - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("n", [8, 12, 16])
def test_type1_regular_grid_reduces_to_fft(n):
    """On an equispaced grid the quadrature sum is the 2D DFT (Section 2.1.1).  With
    x_r = -pi + 2 pi r / n and w = (2 pi / n)^2, f_k = w (-1)^(kx+ky) FFT2(h)[k mod n]."""
    r = np.arange(n)
    xg = -math.pi + 2 * math.pi * r / n
    X, Y = np.meshgrid(xg, xg)           # h[s, r] at (x_r, y_s)
    H = RNG.normal(size=(n, n))
    w = np.full(n * n, (2 * math.pi / n) ** 2)
    N = n
    f = oracle.type1([0, n * n], X.ravel(), Y.ravel(), H.ravel(), w, [0, 0, 0], (N, N), kind=0)[0]
    F = np.fft.fft2(H)
    k = _modes(N)
    KX, KY = np.meshgrid(k, k)
    ref = w[0] * ((-1.0) ** (KX + KY)) * F[KY % n, KX % n]
    assert np.abs(f - ref).max() <= 1e-12 * np.abs(ref).max()


def test_type1_single_point_closed_form():
    """One point: f_k = scale c exp(-i k.x), so |f_k| = |scale c| for every k and
    f_{k+e_x} / f_k = exp(-i x), f_{k+e_y} / f_k = exp(-i y)."""
    x, y, h, w = np.array([1.234]), np.array([-2.5]), np.array([3.0]), np.array([0.7])
    win = np.array([0.5, -0.5, 3.5])
    f = oracle.type1([0, 1], x, y, h, w, win, (7, 6), scale=1.5, kind=1)[0]
    W = 0.5 * (1 + math.cos(math.pi * math.hypot(1.234 - 0.5, -2.5 + 0.5) / 3.5))
    c = 1.5 * 0.7 * W * 3.0
    assert np.allclose(np.abs(f), abs(c), rtol=1e-14, atol=0)
    assert np.allclose(f[:, 1:] / f[:, :-1], np.exp(-1j * 1.234), rtol=1e-13, atol=0)
    assert np.allclose(f[1:, :] / f[:-1, :], np.exp(1j * 2.5), rtol=1e-13, atol=0)
    assert np.isclose(f[3, 3], c, rtol=1e-14)     # k = 0 is the plain sum


def test_type1_linearity_hermitian_shift_period():
    Q = 300
    x, y, h1, w = _cell(Q)
    h2 = RNG.normal(size=Q)
    win = np.array([0.1, 0.2, 2.8])
    N = (9, 7)          # odd boxes are symmetric, so f_{-k} is always in the box
    f1 = oracle.type1([0, Q], x, y, h1, w, win, N)[0]
    f2 = oracle.type1([0, Q], x, y, h2, w, win, N)[0]
    f12 = oracle.type1([0, Q], x, y, 2.5 * h1 - 0.75 * h2, w, win, N)[0]
    assert np.abs(f12 - (2.5 * f1 - 0.75 * f2)).max() <= 1e-12 * np.abs(f12).max()
    # realness of eq. (series): f_{-k} = conj(f_k)
    assert np.abs(f1[::-1, ::-1] - np.conj(f1)).max() <= 1e-12 * np.abs(f1).max()
    # shift theorem (no window): moving every point by (a, b) multiplies f_k by exp(-i k.(a,b))
    g0 = oracle.type1([0, Q], x, y, h1, w, [0, 0, 0], N, kind=0)[0]
    g1 = oracle.type1([0, Q], x + 0.3, y - 1.1, h1, w, [0, 0, 0], N, kind=0)[0]
    KX, KY = np.meshgrid(_modes(N[0]), _modes(N[1]))
    assert np.abs(g1 - g0 * np.exp(-1j * (KX * 0.3 - KY * 1.1))).max() <= 1e-12 * np.abs(g0).max()
    # periodicity of the box: integer-mode sums do not see a 2 pi shift
    g2 = oracle.type1([0, Q], x + 2 * math.pi, y - 4 * math.pi, h1, w, [0, 0, 0], N, kind=0)[0]
    assert np.abs(g2 - g0).max() <= 1e-11 * np.abs(g0).max()


def test_type1_batched_cells_are_independent():
    counts = [5, 0, 17, 1]
    off = np.concatenate([[0], np.cumsum(counts)])
    x, y, h, w = _cell(int(off[-1]))
    wins = RNG.uniform(0.5, 3.0, size=(4, 3))
    f = oracle.type1(off, x, y, h, w, wins, (6, 4))
    for c in range(4):
        a, b = off[c], off[c + 1]
        fc = oracle.type1([0, b - a], x[a:b], y[a:b], h[a:b], w[a:b], wins[c], (6, 4))[0]
        assert np.array_equal(f[c], fc)
    assert np.all(f[1] == 0)


def test_type1_modes_agrees_with_full_box():
    Q = 200
    x, y, h, w = _cell(Q)
    win = np.array([0.0, 0.0, 3.0])
    f = oracle.type1([0, Q], x, y, h, w, win, (8, 6), scale=2.0)[0]
    c = oracle.strength(x, y, h, w, win)
    KX, KY = np.meshgrid(_modes(8), _modes(6))
    g = oracle.type1_modes(x, y, c, KX.ravel(), KY.ravel(), scale=2.0).reshape(6, 8)
    assert np.abs(f - g).max() <= 1e-12 * np.abs(f).max()


def test_type1_axes_agrees_with_box_and_listed_modes():
    """The product-set evaluation equals the full-box sum on the box's own axes, and the
    per-mode direct sums (a separate code path) on a seeded product set of wave numbers
    up to 300."""
    Q = 700
    x, y, h, w = _cell(Q, rng=np.random.default_rng(61))
    win = np.array([0.2, -0.1, 3.0])
    c = oracle.strength(x, y, h, w, win)
    N1, N2 = 6, 5
    box = oracle.type1([0, Q], x, y, h, w, win, (N1, N2), scale=1.3)[0]
    ax = oracle.type1_axes(x, y, c, _modes(N1), _modes(N2), scale=1.3)
    assert np.allclose(ax, box, rtol=0, atol=1e-12 * np.abs(box).max())
    rng = np.random.default_rng(62)
    kx = rng.integers(-300, 300, 7)
    ky = rng.integers(-300, 300, 4)
    ax = oracle.type1_axes(x, y, c, kx, ky)
    KX, KY = np.meshgrid(kx, ky)
    lm = oracle.type1_modes(x, y, c, KX.ravel(), KY.ravel()).reshape(KX.shape)
    assert np.allclose(ax, lm, rtol=0, atol=1e-11 * np.abs(lm).max())


def test_monte_carlo_error_law_and_leakage():
    """Appendix A3.1: for h = A cos(k_s.x) sampled at Q uniform points with uniform weights,
    the coefficient at k_s is A/2 plus an error with E|eps|^2 = A^2/(4Q).  Appendix A3.2:
    for h = 1 the coefficient at any k != 0 has E|C|^2 = 1/Q."""
    A, Q, S = 1000.0, 150, 300
    ks = (3, -2)
    area = (2 * math.pi) ** 2
    rng = np.random.default_rng(777)
    vals, leak = [], []
    for s in range(S):
        x = rng.uniform(0, 2 * math.pi, Q)
        y = rng.uniform(0, 2 * math.pi, Q)
        h = A * np.cos(ks[0] * x + ks[1] * y)
        w = np.full(Q, area / Q)
        f = oracle.type1([0, Q], x, y, h, w, [0, 0, 0], (9, 9), scale=1.0 / area, kind=0)[0]
        vals.append(f[ks[1] + 4, ks[0] + 4])
        g = oracle.type1([0, Q], x, y, np.ones(Q), w, [0, 0, 0], (9, 9), scale=1.0 / area, kind=0)[0]
        leak.append(g[4 + 1, 4 + 2])
    vals = np.array(vals)
    eps = vals - A / 2
    m2 = np.mean(np.abs(eps) ** 2)
    sd = A / (2 * math.sqrt(Q))
    assert abs(vals.real.mean() - A / 2) < 5 * sd / math.sqrt(S)
    assert abs(vals.imag.mean()) < 5 * sd / math.sqrt(S)
    # |eps|^2 / sd^2 is approximately exponential(1): the mean of S draws has rel. sd 1/sqrt(S)
    assert abs(m2 / sd ** 2 - 1.0) < 5 / math.sqrt(S)
    lm2 = np.mean(np.abs(np.array(leak)) ** 2)
    assert abs(lm2 * Q - 1.0) < 5 / math.sqrt(S)


# ----------------------------------------------------------------------------- window

def test_hann_values_and_gradient():
    cx, cy, R = 0.4, -0.3, 2.0
    assert oracle.hann(cx, cy, cx, cy, R) == (1.0, 0.0, 0.0)
    W, _, _ = oracle.hann(cx + 1.0, cy, cx, cy, R)
    assert abs(W - 0.5) < 1e-15
    assert oracle.hann(cx + 2.0, cy, cx, cy, R)[0] == 0.0
    assert oracle.hann(cx + 1.5, cy + 1.5, cx, cy, R) == (0.0, 0.0, 0.0)
    assert oracle.hann(5.0, 5.0, 0, 0, 1.0, kind=0) == (1.0, 0.0, 0.0)
    for (x, y) in [(0.9, 0.1), (-1.0, -0.8), (cx + 1e-9, cy), (0.4, 1.5)]:
        W, gx, gy = oracle.hann(x, y, cx, cy, R)
        e = 1e-6
        fx = (oracle.hann(x + e, y, cx, cy, R)[0] - oracle.hann(x - e, y, cx, cy, R)[0]) / (2 * e)
        fy = (oracle.hann(x, y + e, cx, cy, R)[0] - oracle.hann(x, y - e, cx, cy, R)[0]) / (2 * e)
        assert abs(fx - gx) < 1e-8 and abs(fy - gy) < 1e-8


# ----------------------------------------------------------------------------- EMS

def _ems_on_list(E, prm, perm_seed=None, real=False):
    """Run the oracle's EMS on a 1 x J box whose signed modes are the units (no pairing,
    DC kept), with |f_j|^2 = E_j placed in a shuffled order."""
    E = np.asarray(E, dtype=np.float64)
    J = len(E)
    order = np.arange(J) if perm_seed is None else np.random.default_rng(perm_seed).permutation(J)
    f = np.zeros((1, J), dtype=np.complex128)
    phase = np.ones(J) if real else np.exp(1j * np.linspace(0, 5, J))
    f[0, order] = np.sqrt(E) * phase
    p = oracle.EmsParams(**{**prm.__dict__, "use_pairs": 0, "exclude_dc": 0})
    r = oracle.ems(f, p)
    return r, order


def _closed_neff_geometric(r, J):
    return (1 - r ** J) ** 2 * (1 + r) / ((1 - r) * (1 - r ** (2 * J)))


def test_ems_fig2_families_closed_form():
    g = json.load(open(os.path.join(GOLDEN, "ems_fig2_families.json")))
    P = g["params"]
    prm = oracle.EmsParams(k_min=P["k_min"], k_max=P["k_max"], alpha_min=P["alpha_min"],
                           alpha_max=P["alpha_max"], delta=P["delta"], w1=P["w1"], w2=P["w2"])
    J, K, d = P["J_star"], P["k_max"], P["delta"]
    j = np.arange(1, J + 1)
    fam = {
        "uniform": np.full(J, 0.5),
        "exponential": np.exp(1.0 - j),
        "peak": np.where(j == 1, 1.0, 0.05),
        "step": np.where(j <= 5, 0.7, 0.35),
        "geometric": 0.9 * 0.85 ** (j - 1),
        "cosine": 0.9 * np.cos(math.pi * (j - 1) / (2 * J)),
    }
    assert set(fam) == set(g["families"])
    e1 = math.exp(-1.0)
    # closed forms (N_eff, S_delta, K*) per family; geometric sums for the decaying ones
    expect = {
        "uniform": (20.0, 1.0, 12),
        "exponential": (_closed_neff_geometric(e1, J), math.exp(-(math.e - 1) / d), 1),
        "peak": (1.95 ** 2 / (1 + 19 * 0.05 ** 2), (math.exp(-19 / d) + 10) / 11, 1),
        "step": (8.75 ** 2 / 4.2875, (10 + math.exp(-1 / d)) / 11, 12),
        "geometric": (_closed_neff_geometric(0.85, J), math.exp(-(1 / 0.85 - 1) / d), 3),
    }
    for name, E in fam.items():
        r, order = _ems_on_list(E, prm, perm_seed=len(name))
        T, Pk, neff, sdel, C, aC, th, Js = r.stats
        assert Js == J
        assert np.isclose(T, E.sum(), rtol=1e-15)
        if name in expect:
            n_ref, s_ref, k_ref = expect[name]
            assert np.isclose(neff, n_ref, rtol=1e-13), name
            assert np.isclose(sdel, s_ref, rtol=1e-12, atol=1e-300), name
            assert r.k_star == k_ref, name
        # C and alpha_C follow eqs. (c_score), (alpha_c) from N_eff and S_delta
        assert np.isclose(C, 0.5 * min(neff, K) / K + 0.5 * sdel, rtol=1e-15)
        assert np.isclose(aC, 0.7 * C, rtol=1e-15)
        # K* by brute force: scan the descending list for the first K with theta >= alpha_C
        Es = np.sort(E)[::-1]
        theta = np.cumsum(Es) / Es.sum()
        kc = int(np.argmax(theta >= aC)) + 1 if (theta >= aC).any() else J
        assert r.k_star == min(K, max(1, kc)), name
        assert np.isclose(th, theta[r.k_star - 1], rtol=1e-14)
        # the kept modes are exactly the top-K* energies
        kept = np.nonzero(r.keep[0])[0]
        assert len(kept) == r.k_star
        assert np.isclose(Pk, Es[:r.k_star].sum(), rtol=1e-14)
    # cosine family: N_eff and S_delta from their definitions on the (already sorted) list
    E = fam["cosine"]
    r, _ = _ems_on_list(E, prm, perm_seed=3)
    assert np.isclose(r.stats[2], E.sum() ** 2 / (E ** 2).sum(), rtol=1e-13)
    G = E[:K - 1] / E[1:K]
    assert np.isclose(r.stats[3], np.mean(np.exp(-(G - 1) / d)), rtol=1e-12)
    assert r.k_star == 7


@pytest.mark.parametrize("eps", [0.97, 0.5, 0.01])
def test_ems_flat_tail_closed_form(eps):
    """Appendix A4.1: E = (1, eps, ..., eps) in R^Kmax with J* = Kmax gives
    S_delta = [exp(-(1/eps - 1)/delta) + Kmax - 2]/(Kmax - 1) and
    N_eff = [1 + (Kmax - 1) eps]^2 / [1 + (Kmax - 1) eps^2]."""
    K, d = 12, 0.02
    E = np.array([1.0] + [eps] * (K - 1))
    prm = oracle.EmsParams(k_min=1, k_max=K, alpha_min=0.0, alpha_max=0.7, delta=d)
    r, _ = _ems_on_list(E, prm, perm_seed=5)
    s_ref = (math.exp(-(1 / eps - 1) / d) + K - 2) / (K - 1)
    n_ref = (1 + (K - 1) * eps) ** 2 / (1 + (K - 1) * eps ** 2)
    assert np.isclose(r.stats[3], s_ref, rtol=1e-13)
    assert np.isclose(r.stats[2], n_ref, rtol=1e-13)


@pytest.mark.parametrize("rho,p", [(0.8, 2), (0.9, 3), (0.95, 4)])
def test_ems_moment_degeneracy_closed_form(rho, p):
    """Appendix A4.2: the geometric spectrum rho^(j-1) and the two-level step (b x p, c x r)
    built by eqs. (dformula), (bcformula) share (M1, M2), hence N_eff; their S_delta are
    exp(-(1/rho - 1)/delta) and [(Kmax - 2) + exp(-(b/c - 1)/delta)] / (Kmax - 1)."""
    K, d = 12, 0.02
    A = rho ** np.arange(K)
    M1, M2 = A.sum(), (A ** 2).sum()
    r_ = K - p
    dd = math.sqrt((K * M2 - M1 ** 2) / (p * r_))
    b = M1 / K + r_ / K * dd
    c = M1 / K - p / K * dd
    assert c > 0
    B = np.array([b] * p + [c] * r_)
    prm = oracle.EmsParams(k_min=1, k_max=K, alpha_min=0.1, alpha_max=0.9, delta=d)
    ra, _ = _ems_on_list(A, prm, perm_seed=9)
    rb, _ = _ems_on_list(B, prm, perm_seed=10)
    assert np.isclose(ra.stats[2], rb.stats[2], rtol=1e-12)
    assert np.isclose(ra.stats[2], M1 ** 2 / M2, rtol=1e-13)
    assert np.isclose(ra.stats[3], math.exp(-(1 / rho - 1) / d), rtol=1e-12)
    assert np.isclose(rb.stats[3], (K - 2 + math.exp(-(b / c - 1) / d)) / (K - 1), rtol=1e-12)


def test_ems_pairs_scale_invariance_and_threshold_bruteforce():
    """Pair units on a real-data spectrum: K* depends only on ratios (scale invariance);
    with alpha_min = alpha_max the selection is the plain cumulative threshold (brute
    force over sorted pair energies); the kept set is closed under k -> -k."""
    Q = 400
    x, y, h, w = _cell(Q)
    win = np.array([0.0, 0.0, 3.0])
    N1 = N2 = 8
    f = oracle.type1([0, Q], x, y, h, w, win, (N1, N2))[0]
    prm = oracle.EmsParams(alpha_min=0.9, alpha_max=0.9)
    r = oracle.ems(f, prm)
    r2 = oracle.ems(f * 123.456, prm)
    assert r.k_star == r2.k_star and np.array_equal(r.keep, r2.keep)
    assert np.allclose(r.stats[2:5], r2.stats[2:5], rtol=1e-12)
    # brute force pair energies
    k = _modes(N1)
    units = {}
    for iy, ky in enumerate(k):
        for ix, kx in enumerate(k):
            if kx == 0 and ky == 0:
                continue
            e = abs(f[iy, ix]) ** 2
            mx, my = -kx, -ky
            key = frozenset({(kx, ky)})
            if k[0] <= mx <= k[-1] and k[0] <= my <= k[-1]:
                key = frozenset({(kx, ky), (mx, my)})
            units[key] = units.get(key, 0.0) + e
    # 8x8 box, k in [-4, 3]: 15 edge singletons (kx or ky = -4) and 48/2 interior pairs
    assert len(units) == r.stats[7] == 15 + 24
    Es = np.sort(np.array(list(units.values())))[::-1]
    th = np.cumsum(Es) / Es.sum()
    assert r.k_star == int(np.argmax(th >= 0.9)) + 1
    assert np.isclose(r.stats[0], Es.sum(), rtol=1e-13)
    kept = r.keep.astype(bool)
    for iy, ky in enumerate(k):
        for ix, kx in enumerate(k):
            if kept[iy, ix] and k[0] <= -kx <= k[-1] and k[0] <= -ky <= k[-1]:
                assert kept[list(k).index(-ky), list(k).index(-kx)]
    assert not kept[N2 // 2, N1 // 2]        # DC excluded


def test_ems_ties_break_by_unit_id_and_edge_cases():
    prm = oracle.EmsParams(k_min=1, k_max=3, alpha_min=0.99, alpha_max=0.99)
    r, order = _ems_on_list(np.ones(6), prm, perm_seed=4, real=True)   # exact ties
    assert r.k_star == 3
    assert list(np.nonzero(r.keep[0])[0]) == [0, 1, 2]
    assert list(r.sorted_id) == list(range(6))
    # zero total power: K* = min(K_min, J*)
    r0, _ = _ems_on_list(np.zeros(5), oracle.EmsParams(k_min=2, k_max=4))
    assert r0.k_star == 2 and r0.stats[0] == 0.0
    # one unit: S_delta = 1 by convention
    r1, _ = _ems_on_list(np.array([2.0]), oracle.EmsParams(k_min=1, k_max=4))
    assert r1.k_star == 1 and r1.stats[3] == 1.0
    # k_min above the threshold count
    r2, _ = _ems_on_list(np.array([10.0, 1, 1, 1]), oracle.EmsParams(k_min=3, k_max=4, alpha_min=0.5, alpha_max=0.5))
    assert r2.k_star == 3


def _box3(values):
    """3 x 3 mode box (k in {-1, 0, 1} per axis) from a dict {(kx, ky): |f|^2}."""
    f = np.zeros((3, 3), dtype=np.complex128)
    for (kx, ky), v in values.items():
        f[ky + 1, kx + 1] = math.sqrt(v) * np.exp(1j * (0.3 + kx - 2 * ky))
    return f


def test_ems_weighted_hand_computed():
    """Eq. (weighted_e) on a 3 x 3 box worked out by hand.  Mode powers |f|^2 (DC excluded):
    (1,0) 4 and (-1,0) 4; (-1,1) 1 and (1,-1) 9; (0,1) 2 and (0,-1) 2; (1,1) 3 and (-1,-1) 1.
    Weights: 0 on (1,-1), 3 on (1,1) and (-1,-1), 1 elsewhere.  Weighted pair energies
    (each member's power times its own weight): (1,1) 3*3 + 3*1 = 12, (1,0) 8, (0,1) 4,
    (-1,1) 1*1 + 0*9 = 1, total 25.  At alpha = 0.75 the running fractions are 0.48, 0.8,
    so K* = 2; the kept power is the unweighted 3 + 1 + 4 + 4 = 12; N_eff = 25^2 / 225."""
    pw = {(1, 0): 4, (-1, 0): 4, (-1, 1): 1, (1, -1): 9, (0, 1): 2, (0, -1): 2, (1, 1): 3, (-1, -1): 1,
          (0, 0): 100}
    f = _box3(pw)
    om = np.ones((3, 3))
    om[-1 + 1, 1 + 1] = 0.0          # (kx, ky) = (1, -1)
    om[1 + 1, 1 + 1] = 3.0           # (1, 1)
    om[-1 + 1, -1 + 1] = 3.0         # (-1, -1)
    prm = oracle.EmsParams(alpha_min=0.75, alpha_max=0.75)
    r = oracle.ems(f, prm, mode_weight=om)
    assert r.k_star == 2
    kept = {(ix - 1, iy - 1) for iy, ix in zip(*np.nonzero(r.keep))}
    assert kept == {(1, 1), (-1, -1), (1, 0), (-1, 0)}
    assert np.isclose(r.stats[0], 25.0, rtol=1e-15)
    assert np.isclose(r.stats[1], 12.0, rtol=1e-15)
    assert np.isclose(r.stats[2], 625.0 / 225.0, rtol=1e-14)
    assert np.isclose(r.stats[6], 20.0 / 25.0, rtol=1e-15)
    assert np.allclose(r.sorted_e, [12, 8, 4, 1], rtol=1e-14)
    # unweighted for contrast: (-1,1) pair 10 leads, then 8, then the tie 4 / 4 broken by id
    r0 = oracle.ems(f, prm)
    assert np.allclose(r0.sorted_e, [10, 8, 4, 4], rtol=1e-14)
    assert r0.sorted_id[2] == 2 * 3 + 1 and r0.sorted_id[3] == 2 * 3 + 2


@pytest.mark.parametrize("use_pairs", [1, 0])
def test_ems_weighted_equals_rescaled_coefficients(use_pairs):
    """A weight omega_k >= 0 on every signed mode multiplies that mode's power, so the
    weighted selection on f is the unweighted selection on sqrt(omega) f (same K*, kept
    set, T, N_eff, S_delta, C, alpha_C, theta); the retained power P stays the plain
    sum of |f_k|^2 over the kept modes.  Weights are asymmetric (omega_k != omega_-k)
    and include zeros."""
    Q = 600
    x, y, h, w = _cell(Q, rng=np.random.default_rng(77))
    f = oracle.type1([0, Q], x, y, h, w, np.array([0.0, 0.0, 3.0]), (12, 10))[0]
    rng = np.random.default_rng(78)
    om = rng.uniform(0.0, 2.0, size=f.shape)
    om[rng.random(f.shape) < 0.1] = 0.0
    for prm in (oracle.EmsParams(alpha_min=0.9, alpha_max=0.9, use_pairs=use_pairs),
                oracle.EmsParams(k_min=2, k_max=15, alpha_min=0.1, alpha_max=0.8, delta=0.05,
                                 use_pairs=use_pairs)):
        rw = oracle.ems(f, prm, mode_weight=om)
        rs = oracle.ems(np.sqrt(om) * f, prm)
        assert rw.k_star == rs.k_star
        assert np.array_equal(rw.keep, rs.keep)
        assert np.array_equal(rw.sorted_id, rs.sorted_id)
        assert np.allclose(rw.stats[[0, 2, 3, 4, 5, 6, 7]], rs.stats[[0, 2, 3, 4, 5, 6, 7]], rtol=1e-12)
        assert np.isclose(rw.stats[1], np.sum(np.abs(f) ** 2 * rw.keep), rtol=1e-13)
    # omega = 1 everywhere is the unweighted selection
    r1 = oracle.ems(f, oracle.EmsParams(use_pairs=use_pairs), mode_weight=np.ones(f.shape))
    r0 = oracle.ems(f, oracle.EmsParams(use_pairs=use_pairs))
    assert r1.k_star == r0.k_star and np.array_equal(r1.keep, r0.keep)


def test_ems_weighted_zero_and_scale():
    """A zero weight on both members of the strongest pair moves it to the end of the
    order (it is kept only if every other unit is); scaling all weights by one factor
    changes no selection and scales T by that factor."""
    Q = 500
    x, y, h, w = _cell(Q, rng=np.random.default_rng(91))
    f = oracle.type1([0, Q], x, y, h, w, np.array([0.0, 0.0, 3.0]), (8, 8))[0]
    prm = oracle.EmsParams(alpha_min=0.8, alpha_max=0.8)
    r0 = oracle.ems(f, prm)
    top = int(r0.sorted_id[0])
    iy, ix = divmod(top, 8)
    kx, ky = ix - 4, iy - 4
    om = np.ones((8, 8))
    om[iy, ix] = 0.0
    mirror = (-ky + 4, -kx + 4) if (-4 <= -kx <= 3 and -4 <= -ky <= 3) else (iy, ix)
    om[mirror] = 0.0
    r = oracle.ems(f, prm, mode_weight=om)
    assert r.sorted_id[-1] == top and r.sorted_e[-1] == 0.0
    assert not r.keep[iy, ix] and not r.keep[mirror]
    rs = oracle.ems(f, prm, mode_weight=7.5 * np.ones((8, 8)))
    assert rs.k_star == r0.k_star and np.array_equal(rs.keep, r0.keep)
    assert np.isclose(rs.stats[0], 7.5 * r0.stats[0], rtol=1e-13)


# ----------------------------------------------------------------------------- adjoint

def test_vjp_adjoint_identity():
    """<T1 c, g> = <c, Re T2 g> with the real inner product Re sum conj(a) b."""
    Q = 120
    x, y, c, _ = _cell(Q)
    N = (7, 6)
    g = RNG.normal(size=(1, N[1], N[0])) + 1j * RNG.normal(size=(1, N[1], N[0]))
    f = oracle.type1([0, Q], x, y, c, np.ones(Q), [0, 0, 0], N, scale=0.8, kind=0)
    u, _, _ = oracle.type1_vjp([0, Q], x, y, c, np.ones(Q), [0, 0, 0], N, g, scale=0.8, kind=0)
    lhs = np.real(np.sum(np.conj(f) * g))
    rhs = np.dot(c, u)
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + np.abs(f).sum() * np.abs(g).max())


def test_vjp_single_point_closed_form():
    """One point, keep all K modes: P = K (s w W h)^2, dP/dh = 2K s^2 w^2 W^2 h,
    dP/dx = 2K s^2 w^2 h^2 W dW/dx."""
    x, y, h, w = np.array([0.8]), np.array([-0.4]), np.array([2.0]), np.array([0.3])
    win = np.array([0.1, 0.2, 2.5])
    N = (5, 4)
    K = 20
    s = 0.9
    f = oracle.type1([0, 1], x, y, h, w, win, N, scale=s)
    W, dWx, dWy = oracle.hann(0.8, -0.4, *win)
    g = 2.0 * f
    gh, gx, gy = oracle.type1_vjp([0, 1], x, y, h, w, win, N, g, scale=s)
    assert np.isclose(np.sum(np.abs(f) ** 2), K * (s * 0.3 * W * 2.0) ** 2, rtol=1e-14)
    assert np.isclose(gh[0], 2 * K * s ** 2 * 0.09 * W ** 2 * 2.0, rtol=1e-12)
    assert np.isclose(gx[0], 2 * K * s ** 2 * 0.09 * 4.0 * W * dWx, rtol=1e-12)
    assert np.isclose(gy[0], 2 * K * s ** 2 * 0.09 * 4.0 * W * dWy, rtol=1e-12)


def test_vjp_finite_differences_on_retained_power():
    """Central differences (step 1e-6, FP64) of P = sum_keep |f_k|^2 with the kept set frozen
    match the analytic gradient from the direct type-2 sums."""
    b = synth.config1(count_scale=0.004, n_cells=3)
    inp = oracle.batch_inputs(b)
    inp["n_modes"] = (16, 16)
    prm = oracle.EmsParams(alpha_min=0.95, alpha_max=0.95)
    res = oracle.retained_power_grad(prm=prm, **inp)
    keep = res["keep"]
    off = inp["offsets"]

    def P(x, y, h):
        f = oracle.type1(off, x, y, h, inp["w"], inp["windows"], inp["n_modes"])
        return np.sum(np.abs(f) ** 2 * keep)

    rng = np.random.default_rng(5)
    idx = rng.choice(len(inp["x"]), size=6, replace=False)
    P0 = P(inp["x"], inp["y"], inp["h"])
    step = 1e-6
    for j in idx:
        for name, key in (("h", "grad_h"), ("x", "grad_x"), ("y", "grad_y")):
            a = {k: inp[k].copy() for k in ("x", "y", "h")}
            bb = {k: inp[k].copy() for k in ("x", "y", "h")}
            sc = step * max(1.0, abs(inp[name][j]))
            a[name][j] += sc
            bb[name][j] -= sc
            fd = (P(a["x"], a["y"], a["h"]) - P(bb["x"], bb["y"], bb["h"])) / (2 * sc)
            an = res[key][j]
            # rounding floor of a central difference of P in FP64
            noise = 64 * np.finfo(float).eps * P0 / (2 * sc)
            assert abs(fd - an) <= 1e-6 * abs(an) + noise, (name, j, fd, an, noise)


# ----------------------------------------------------------------------------- reconstruction

def _grid_points(n):
    g = -math.pi + 2 * math.pi * np.arange(n) / n
    X, Y = np.meshgrid(g, g)
    return X.ravel(), Y.ravel()


def test_reconstruct_band_limited_grid_is_exact_and_parseval_holds():
    """Section 3.2 diagnostics where the answer is known: a zero-mean band-limited field
    sampled on a regular n x n grid of the 2 pi box with uniform weights (2 pi / n)^2, no
    window, |D| = (2 pi)^2 and scale 1/|D| (eq. discrete_quadrature).  The quadrature is
    then the exact DFT, the truncated series reproduces every sample (eps_rel = 0) and
    Parseval's identity, eq. (spectral_variance), holds exactly (ratio 1)."""
    n, N = 24, 12
    x, y = _grid_points(n)
    rng = np.random.default_rng(71)
    h = np.zeros_like(x)
    for _ in range(9):
        kx, ky = rng.integers(-5, 6, 2)
        if kx == 0 and ky == 0:
            continue
        h += rng.normal() * np.cos(kx * x + ky * y + rng.uniform(0, 2 * np.pi))
    Q = len(x)
    area = (2 * math.pi) ** 2
    w = np.full(Q, area / Q)
    f = oracle.type1([0, Q], x, y, h, w, [0, 0, 1], (N, N), scale=1 / area, kind=0)
    hr, dg = oracle.reconstruct([0, Q], x, y, h, w, [0, 0, 1], (N, N), f, area=[area], kind=0)
    assert np.allclose(hr, h, rtol=0, atol=1e-12 * np.abs(h).max())
    assert dg[0, 0] == Q and dg[0, 6] < 1e-12
    assert np.isclose(dg[0, 3], np.mean(h ** 2), rtol=1e-13)
    assert np.isclose(dg[0, 7], 1.0, rtol=1e-12)
    assert np.isclose(dg[0, 4], dg[0, 5], rtol=1e-15)


def test_reconstruct_single_mode_closed_form():
    """h = A cos(k0 . x + phi) on a regular grid: hat h at +-k0 is (A/2) e^{+-i phi}, both
    variances are A^2 / 2, and keeping only the pair +-k0 reconstructs h; keeping
    nothing gives h_rec = 0 and eps_rel = 1."""
    n, N = 16, 8
    x, y = _grid_points(n)
    A, phi, k0 = 3.0, 0.7, (2, -3)
    h = A * np.cos(k0[0] * x + k0[1] * y + phi)
    Q = len(x)
    area = (2 * math.pi) ** 2
    w = np.full(Q, area / Q)
    f = oracle.type1([0, Q], x, y, h, w, [0, 0, 1], (N, N), scale=1 / area, kind=0)
    lo = -(N // 2)
    assert np.isclose(f[0, k0[1] - lo, k0[0] - lo], A / 2 * np.exp(1j * phi), atol=1e-13)
    keep = np.zeros((1, N, N), dtype=np.uint8)
    keep[0, k0[1] - lo, k0[0] - lo] = 1
    keep[0, -k0[1] - lo, -k0[0] - lo] = 1
    hr, dg = oracle.reconstruct([0, Q], x, y, h, w, [0, 0, 1], (N, N), f, keep=keep, area=[area], kind=0)
    assert np.allclose(hr, h, atol=1e-12)
    assert np.isclose(dg[0, 3], A * A / 2, rtol=1e-13) and np.isclose(dg[0, 5], A * A / 2, rtol=1e-12)
    hr0, dg0 = oracle.reconstruct([0, Q], x, y, h, w, [0, 0, 1], (N, N), f, keep=np.zeros_like(keep),
                                  area=[area], kind=0)
    assert np.all(hr0 == 0) and dg0[0, 6] == 1.0 and dg0[0, 5] == 0.0


def test_reconstruct_brute_force_with_window():
    """Off-grid samples, random coefficients (DC included), a random kept set and the Hann
    window: the series and every diagnostic against a numpy evaluation of their
    definitions (target t = W h, the windowed field the coefficients represent)."""
    rng = np.random.default_rng(72)
    N1, N2 = 5, 6
    offs = [0, 40, 40, 97]
    Q = offs[-1]
    x, y, h, w = _cell(Q, rng=rng)
    win = np.array([[0.1, -0.2, 2.5], [0.0, 0.0, 1.0], [-0.3, 0.2, 3.1]])
    coef = rng.normal(size=(3, N2, N1)) + 1j * rng.normal(size=(3, N2, N1))
    keep = (rng.random((3, N2, N1)) < 0.5).astype(np.uint8)
    area = np.array([7.0, 1.0, 11.0])
    hr, dg = oracle.reconstruct(offs, x, y, h, w, win, (N1, N2), coef, keep=keep, area=area)
    kx, ky = np.meshgrid(_modes(N1), _modes(N2))
    for c in range(3):
        a, b = offs[c], offs[c + 1]
        ph = np.outer(x[a:b], kx.ravel()) + np.outer(y[a:b], ky.ravel())
        rec = np.real(np.exp(1j * ph) @ (coef[c] * keep[c]).ravel())
        assert np.allclose(hr[a:b], rec, rtol=0, atol=1e-12 * max(1.0, np.abs(rec).max() if b > a else 1.0))
        t = np.array([oracle.hann(x[j], y[j], *win[c])[0] * h[j] for j in range(a, b)])
        nz = (kx.ravel() != 0) | (ky.ravel() != 0)
        p2 = np.abs(coef[c].ravel()) ** 2
        assert dg[c, 0] == b - a
        assert np.isclose(dg[c, 1], np.sum((t - rec) ** 2), rtol=1e-12)
        assert np.isclose(dg[c, 2], np.sum(t ** 2), rtol=1e-12, atol=0)
        assert np.isclose(dg[c, 3], np.sum(w[a:b] * t ** 2) / area[c], rtol=1e-12, atol=0)
        assert np.isclose(dg[c, 4], np.sum(p2[nz]), rtol=1e-13)
        assert np.isclose(dg[c, 5], np.sum((p2 * keep[c].ravel())[nz]), rtol=1e-13)
        if b > a:
            assert np.isclose(dg[c, 6], math.sqrt(dg[c, 1] / dg[c, 2]), rtol=1e-14)
            assert np.isclose(dg[c, 7], dg[c, 4] / dg[c, 3], rtol=1e-14)


# ----------------------------------------------------------------------------- flow-dependent EMS

def _action_weight(kx, ky, ks, ux, uy, N, fc, rho):
    """|A| / |h|^2 of eq. (mw_action) after eliminating m^2 with eq. (mw_dispersion):
    (|k|^2 + m^2) / |k|^2 = (N^2 - fc^2) / (omega^2 - fc^2), and |k . u| = |omega|, so
    w = (rho / 2) |omega| (N^2 - fc^2) / (omega^2 - fc^2) inside the band fc < |omega| < N."""
    om = -(ks * kx * ux + ks * ky * uy)
    if kx == 0 and ky == 0:
        return 0.0
    if not (abs(fc) < abs(om) < N):
        return 0.0
    return rho / 2 * abs(om) * (N * N - fc * fc) / (om * om - fc * fc)


def test_mw_weight_closed_form_and_band():
    """The launch weight of Appendix A7 against its closed form (the dispersion relation
    eliminated by hand); zero outside the propagating band and at k = 0; even in k and
    in u."""
    rng = np.random.default_rng(81)
    n_in = 0
    for _ in range(400):
        kx, ky = rng.integers(-32, 32, 2)
        ks = 10 ** rng.uniform(-4.5, -3)
        ux, uy = rng.normal(scale=10, size=2)
        N, fc, rho = 10 ** rng.uniform(-2.5, -1.5), 10 ** rng.uniform(-5, -3.5), rng.uniform(0.3, 1.3)
        w = oracle.mw_weight(kx, ky, ks, ux, uy, N, fc, rho)
        ref = _action_weight(kx, ky, ks, ux, uy, N, fc, rho)
        n_in += ref > 0
        assert np.isclose(w, ref, rtol=1e-12, atol=0), (kx, ky, w, ref)
        assert w == oracle.mw_weight(-kx, -ky, ks, ux, uy, N, fc, rho)
        assert w == oracle.mw_weight(kx, ky, ks, -ux, -uy, N, fc, rho)
    assert 40 < n_in < 360          # both sides of the band are exercised
    assert oracle.mw_weight(0, 0, 1e-3, 10, 0, 0.02, 1e-4, 1) == 0.0
    # k perpendicular to the wind: omega = 0, no launch (Section 3.3, the first mode)
    assert oracle.mw_weight(0, 5, 1e-3, 10, 0, 0.02, 1e-4, 1) == 0.0


def test_ems_flow_equals_ems_with_closed_form_weights():
    """Per step and cell, the flow-dependent selection is EMS (eq. weighted_e) with the
    closed-form launch weights; outputs are ordered step-major."""
    Q = 500
    rng = np.random.default_rng(82)
    fs = []
    for c in range(3):
        x, y, h, w = _cell(Q, rng=rng)
        fs.append(oracle.type1([0, Q], x, y, h, w, [0.0, 0.0, 3.0], (10, 8))[0])
    f = np.stack(fs)
    T = 4
    flow = np.zeros((T, 3, 6))
    flow[..., 0] = rng.normal(scale=8, size=(T, 3))
    flow[..., 1] = rng.normal(scale=8, size=(T, 3))
    flow[..., 2] = 0.02
    flow[..., 3] = 1e-4
    flow[..., 4] = rng.uniform(0.5, 1.2, size=(T, 3))
    flow[..., 5] = 2 * np.pi / 20000.0
    for prm in (oracle.EmsParams(alpha_min=0.9, alpha_max=0.9),
                oracle.EmsParams(k_min=1, k_max=4, alpha_min=0.9, alpha_max=1.0)):
        keep, ks, st = oracle.ems_flow(f, flow, prm)
        for s_ in range(T):
            for c in range(3):
                ux, uy, N, fc, rho, k0 = flow[s_, c]
                om = np.array([[_action_weight(kx, ky, k0, ux, uy, N, fc, rho) for kx in _modes(10)]
                               for ky in _modes(8)])
                r = oracle.ems(f[c], prm, mode_weight=om)
                assert ks[s_, c] == r.k_star and np.array_equal(keep[s_, c], r.keep)
                assert np.allclose(st[s_, c], r.stats, rtol=1e-12, atol=0)


def test_ems_flow_mountain_wave_modes():
    """The Section 3.3 mode set: N_mu = 4 modes k_mu = (mu - 1) 2 pi / lambda0 along x and
    l = 2 pi / lambda0 along y with equal amplitudes, zonal wind u0.  The first mode has
    k . u = 0, so zero launch weight: it is never kept while another mode carries
    weight, and reversing the wind changes nothing."""
    lam0, u0 = 10000.0, 10.0
    N1 = N2 = 16
    f = np.zeros((1, N2, N1), dtype=np.complex128)
    lo = -(N1 // 2)
    for mu in range(4):
        f[0, 1 - lo, mu - lo] = 1.0          # (kx, ky) = (mu - 1 + 1, 1) in box units: kx = mu
    ks = 2 * np.pi / lam0
    flow = np.array([[[u0, 0.0, 0.02, 1e-4, 1.0, ks]], [[-u0, 0.0, 0.02, 1e-4, 1.0, ks]]])
    prm = oracle.EmsParams(k_min=1, k_max=4, alpha_min=0.9, alpha_max=1.0, use_pairs=0, exclude_dc=1)
    keep, kstar, st = oracle.ems_flow(f, flow, prm)
    assert not keep[0, 0, 1 - lo, 0 - lo] and not keep[1, 0, 1 - lo, 0 - lo]
    assert np.array_equal(keep[0], keep[1]) and kstar[0, 0] == kstar[1, 0] >= 1
    w = [_action_weight(mu, 1, ks, u0, 0, 0.02, 1e-4, 1.0) for mu in range(4)]
    assert w[0] == 0.0 and all(v > 0 for v in w[1:])


# ----------------------------------------------------------------------------- cell geometry

def test_geometry_edge_frame_hand_worked():
    """Triangle (0,0), (4,0), (1,3): edges (4,0), (-3,3), (-1,-3); the longest is (-3,3)
    (length 3 sqrt 2), at 135 degrees, so cos = -1/sqrt 2, sin = 1/sqrt 2 and that edge
    maps onto +x with length 3 sqrt 2.  Centroid (5/3, 1).  Rotated vertices span
    3 sqrt 2 along x; the height of the triangle over that edge is area * 2 / base =
    12 / (3 sqrt 2) = 2 sqrt 2 along y, so H = (eta / 2) 3 sqrt 2.  The vertex (4, 0) lies
    7 / (3 sqrt 2) from the centroid along the local x axis, outside the square at eta = 1
    (H = 3 / sqrt 2), inside at eta = 1.5."""
    tri = np.array([0.0, 0.0, 4.0, 0.0, 1.0, 3.0])
    x = np.array([5 / 3, 0.0, 4.0, 1.0, 10.0])
    y = np.array([1.0, 0.0, 0.0, 3.0, 10.0])
    h = np.array([1.0, 2.0, 3.0, 4.0, 5.0])
    for eta in (1.0, 1.5):
        g = oracle.cell_geometry([0, 5], tri, x, y, h, frame="edge", mask="triangle", eta=eta, deplane=False)
        cx, cy, cs, sn, H, A, qin, hbar = g["info"][0]
        s2 = math.sqrt(2)
        assert np.allclose([cx, cy, cs, sn], [5 / 3, 1.0, -1 / s2, 1 / s2], atol=1e-15)
        assert np.isclose(H, eta / 2 * 3 * s2, rtol=1e-15)
        if eta == 1.0:
            assert list(g["inside"]) == [1, 1, 0, 1, 0] and A < 6.0
            continue
        assert np.isclose(A, 6.0, rtol=1e-15)                 # the triangle's area
        assert list(g["inside"]) == [1, 1, 1, 1, 0]            # vertices count as inside
        # the longest edge (from (4,0) to (1,3)) is parallel to x in the local frame
        assert np.isclose(g["yb"][2], g["yb"][3], atol=1e-14) and g["xb"][3] > g["xb"][2]
        assert np.isclose(g["xb"][3] - g["xb"][2], 3 * s2 * math.pi / H, rtol=1e-14)
        assert np.allclose(g["wb"], [0.25, 0.25, 0.25, 0.25, 0.0])
        assert np.array_equal(g["hb"], h)
    gc = oracle.cell_geometry([0, 5], tri, x, y, h, frame="centroid", mask="square", eta=1.0)
    cx, cy, cs, sn, H, A, qin, hbar = gc["info"][0]
    assert (cs, sn) == (1.0, 0.0) and np.isclose(H, 2.0) and np.isclose(A, 16.0)   # extents 4 and 3
    # the square is centred on the centroid (5/3, 1): the vertex (4, 0) is 7/3 > H away
    assert list(gc["inside"]) == [1, 1, 0, 1, 0]


def test_geometry_triangle_clipped_by_its_square():
    """An equilateral triangle of side s in the edge-aligned frame at eta = 1: H = s / 2
    and the centroid-centred square cuts off the apex above y = s / 2 (the apex sits at
    s / sqrt 3).  |D| = sqrt 3 s^2 / 4 minus the cut-off triangle, whose height is
    s / sqrt 3 - s / 2 and whose base is that height times 2 / sqrt 3."""
    s_ = 2.0
    tri = np.array([0.0, 0.0, s_, 0.0, s_ / 2, s_ * math.sqrt(3) / 2])
    g = oracle.cell_geometry([0, 0], tri, np.zeros(0), np.zeros(0), np.zeros(0), frame="edge", mask="triangle",
                             eta=1.0)
    H, A = g["info"][0, 4], g["info"][0, 5]
    hc = s_ / math.sqrt(3) - s_ / 2
    assert np.isclose(H, s_ / 2, rtol=1e-15)
    assert np.isclose(A, math.sqrt(3) / 4 * s_ * s_ - 0.5 * hc * (2 * hc / math.sqrt(3)), rtol=1e-13)
    # a looser square (eta = 1.3) holds the whole triangle
    g = oracle.cell_geometry([0, 0], tri, np.zeros(0), np.zeros(0), np.zeros(0), frame="edge", mask="triangle",
                             eta=1.3)
    assert np.isclose(g["info"][0, 5], math.sqrt(3) / 4 * s_ * s_, rtol=1e-13)


def test_geometry_masks_and_deplaning():
    """Circle and square masks on a random cloud, uniform weights 1/Q_in, and the deplaned
    heights have zero weighted mean over the mask (eq. alps_deplaning)."""
    rng = np.random.default_rng(101)
    tri = np.array([-1.0, -0.5, 2.0, -0.2, 0.3, 1.9])
    x = rng.uniform(-2, 3, 600)
    y = rng.uniform(-2, 3, 600)
    h = rng.normal(size=600) + 3.0
    for mask in ("square", "circle", "triangle"):
        g = oracle.cell_geometry([0, 600], tri, x, y, h, frame="edge", mask=mask, eta=1.2)
        cx, cy, cs, sn, H, A, qin, hbar = g["info"][0]
        u = np.stack([cs * (x - cx) + sn * (y - cy), -sn * (x - cx) + cs * (y - cy)])
        if mask == "square":
            ref = (np.abs(u[0]) <= H) & (np.abs(u[1]) <= H)
            assert np.isclose(A, 4 * H * H)
        elif mask == "circle":
            ref = u[0] ** 2 + u[1] ** 2 <= H * H
            assert np.isclose(A, math.pi * H * H)
        else:
            ref = g["inside"].astype(bool)
            # at eta = 1.2 this triangle fits its square: |D| is the triangle's area
            assert np.isclose(A, 0.5 * abs((tri[2] - tri[0]) * (tri[5] - tri[1]) - (tri[4] - tri[0]) * (tri[3] - tri[1])))
            assert np.all(np.abs(u[:, ref]) <= H)
        assert np.array_equal(g["inside"].astype(bool), ref)
        assert qin == ref.sum() > 0
        assert np.allclose(g["wb"][ref], 1.0 / qin) and np.all(g["wb"][~ref] == 0)
        assert np.isclose(hbar, np.mean(h[ref]), rtol=1e-13)
        assert abs(np.sum(g["wb"] * g["hb"])) < 1e-12
        assert np.allclose(g["xb"], u[0] * math.pi / H) and np.allclose(g["yb"], u[1] * math.pi / H)


def test_geometry_voronoi_closed_forms():
    """Raster Voronoi weights where the answer is exact: two samples split the square
    along their perpendicular bisector (here a raster line), so the weights are the two
    area fractions; a regular lattice with the raster aligned to it gets equal weights;
    weights sum to 1; an isolated empty sample gets the floor and the rest renormalise."""
    # square mask, centroid frame, H = 2: samples at x = -1 and x = +0.5 -> bisector at -0.25
    tri = np.array([-2.0, -2.0, 2.0, -2.0, 0.0, 2.0])       # extents 4 x 4, centroid (0, -2/3)
    cy = -2 / 3
    x = np.array([-1.0, 0.5])
    y = np.array([cy, cy])
    g = oracle.cell_geometry([0, 2], tri, x, y, np.zeros(2), frame="centroid", mask="square",
                             weights="voronoi", raster=16, eta=1.0)
    assert np.isclose(g["info"][0, 4], 2.0)
    assert np.allclose(g["wb"], [(2 - 0.25) / 4, (2 + 0.25) / 4], atol=1e-15)
    assert g["counts"].sum() == 256
    # 8 x 8 lattice of samples at raster-aligned cell centres: equal weights
    gx = -2 + 0.5 * (np.arange(8) + 0.5)
    X, Y = np.meshgrid(gx, gx + cy)
    g = oracle.cell_geometry([0, 64], tri, X.ravel(), Y.ravel(), np.zeros(64), frame="centroid", mask="square",
                             weights="voronoi", raster=32, eta=1.0)
    assert np.allclose(g["wb"], 1 / 64, atol=1e-15) and np.all(g["counts"] == 16)
    # a sample with no raster point of its own (an exact duplicate: ties go to the lower
    # index) gets the floor weight
    x3 = np.array([-1.0, 0.5, 0.5])
    y3 = np.array([cy, cy, cy])
    g = oracle.cell_geometry([0, 3], tri, x3, y3, np.zeros(3), frame="centroid", mask="square",
                             weights="voronoi", raster=16, eta=1.0, floor_frac=0.5)
    assert g["counts"][2] == 0 and g["counts"][1] > 0
    assert np.isclose(g["wb"].sum(), 1.0, rtol=1e-15)
    assert np.isclose(g["wb"][2] / g["wb"][0], 0.5 / g["counts"][0], rtol=1e-13)


def test_geometry_voronoi_brute_force():
    """Raster Voronoi counts on a random cloud and the triangle mask against a numpy
    nearest-sample assignment of the raster cell centres inside the rotated triangle."""
    rng = np.random.default_rng(102)
    tri = np.array([0.3, 0.1, 3.1, 0.8, 1.0, 2.7])
    x = rng.uniform(0, 3.2, 120)
    y = rng.uniform(0, 2.8, 120)
    g = oracle.cell_geometry([0, 120], tri, x, y, np.ones(120), frame="edge", mask="triangle", weights="voronoi",
                             raster=48, eta=1.1)
    cx, cy, cs, sn, H, A, qin, hbar = g["info"][0]
    ins = g["inside"].astype(bool)
    ux = cs * (x - cx) + sn * (y - cy)
    uy = -sn * (x - cx) + cs * (y - cy)
    vt = np.array([[cs * (tri[2 * i] - cx) + sn * (tri[2 * i + 1] - cy),
                    -sn * (tri[2 * i] - cx) + cs * (tri[2 * i + 1] - cy)] for i in range(3)])
    step = 2 * H / 48
    c = -H + step * (np.arange(48) + 0.5)
    GX, GY = np.meshgrid(c, c)
    P = np.stack([GX.ravel(), GY.ravel()], 1)

    def side(p, a, b):
        return (p[:, 0] - b[0]) * (a[1] - b[1]) - (a[0] - b[0]) * (p[:, 1] - b[1])
    d = np.stack([side(P, vt[0], vt[1]), side(P, vt[1], vt[2]), side(P, vt[2], vt[0])], 1)
    inside_g = ~((d < 0).any(1) & (d > 0).any(1))
    P = P[inside_g]
    idx = np.nonzero(ins)[0]
    D2 = (P[:, None, 0] - ux[idx][None]) ** 2 + (P[:, None, 1] - uy[idx][None]) ** 2
    near = idx[np.argmin(D2, axis=1)]
    counts = np.bincount(near, minlength=120)
    assert np.array_equal(g["counts"], counts)
    assert np.isclose(g["wb"].sum(), 1.0) and np.all(g["wb"][~ins] == 0)
