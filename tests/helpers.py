"""Shared helpers for the parity tests (no arithmetic of the method here)."""
import numpy as np
import torch

import oracle
import paper_2606_21278_amd as enf


def rel_l2(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    d = np.linalg.norm((a - b).ravel())
    n = np.linalg.norm(b.ravel())
    return d / n if n > 0 else d


def per_cell_rel_l2(f_gpu, f_ref):
    out = []
    for c in range(f_ref.shape[0]):
        n = np.linalg.norm(f_ref[c].ravel())
        d = np.linalg.norm((f_gpu[c] - f_ref[c]).ravel())
        out.append(d / n if n > 0 else d)
    return np.array(out)


def make_plan(batch, **kw):
    args = dict(n_modes=batch.n_modes, sigma=batch.sigma, eps=batch.eps, precision=batch.precision,
                window="hann" if (batch.windows[:, 2] > 0).all() else "none")
    args.update(kw)
    return enf.Plan(batch.cell_offsets, batch.windows, **args)


def gpu_batch(batch):
    """The batch on cuda:0 in its precision."""
    dt = torch.float64 if batch.precision == "f64" else torch.float32
    return batch.to(device="cuda:0", dtype=dt)


def oracle_f(batch, cells=None):
    inp = oracle.batch_inputs(batch, cells)
    return oracle.type1(inp["offsets"], inp["x"], inp["y"], inp["h"], inp["w"], inp["windows"],
                        inp["n_modes"], kind=inp["kind"])


def unit_energy_bounds(f_ref, dev, prm):
    """Per-unit energy perturbation bounds dE_u = sum_k (2 |f_k| d_k + d_k^2) for
    per-mode deviations d_k, in the oracle's sorted unit order."""
    N2, N1 = f_ref.shape
    lo1, lo2 = -(N1 // 2), -(N2 // 2)
    a = np.abs(f_ref)
    per_mode = 2 * a * dev + dev ** 2
    r = oracle.ems(f_ref, prm)
    out = np.zeros(len(r.sorted_id))
    for j, uid in enumerate(r.sorted_id):
        iy, ix = divmod(int(uid), N1)
        v = per_mode[iy, ix]
        if prm.use_pairs:
            kx, ky = ix + lo1, iy + lo2
            mx, my = -kx, -ky
            if (kx, ky) != (0, 0) and lo1 <= mx <= lo1 + N1 - 1 and lo2 <= my <= lo2 + N2 - 1:
                v += per_mode[my - lo2, mx - lo1]
        out[j] = v
    return r, out


def robust_selection(f_ref, f_gpu, r, prm):
    """'Input without ties' for a coefficient set: the oracle's kept set is the only
    outcome for every spectrum within the measured per-mode deviation of the GPU
    coefficients from the oracle's.  Checks that the kept units stay strictly above
    the rest and that the power threshold (alpha_C fixed: alpha_min = alpha_max) cuts
    at the same count for all such spectra."""
    if prm.alpha_min != prm.alpha_max:
        raise ValueError("robust_selection needs a fixed alpha_C")
    dev = np.abs(np.asarray(f_gpu) - np.asarray(f_ref))
    r, dE = unit_energy_bounds(f_ref, dev, prm)
    E = r.sorted_e
    K, J = r.k_star, len(E)
    if K < J and K >= 1 and not (E[K - 1] - dE[K - 1] > np.max(E[K:] + dE[K:])):
        return False
    if K >= 1 and K < J and np.min(E[:K] - dE[:K]) <= np.max(E[K:] + dE[K:]):
        return False
    T, DT = E.sum(), dE.sum()
    if T - DT <= 0:
        return False
    S = np.cumsum(E)
    D = np.cumsum(dE)
    a = prm.alpha_min
    Jmax = min(J, prm.k_max)
    thmin = (S - D) / (T + DT)
    thmax = (S + D) / (T - DT)
    # the first K with theta(K) >= alpha must be the same for every admissible spectrum
    kc_lo = int(np.argmax(thmax >= a)) + 1 if (thmax >= a).any() else J
    kc_hi = int(np.argmax(thmin >= a)) + 1 if (thmin >= a).any() else J
    clamp = lambda kc: min(Jmax, max(prm.k_min, kc))
    return clamp(kc_lo) == clamp(kc_hi) == K
