"""Error metrics for comparing the HIP path with the oracle.

Per cell: |x - y| / max(|y|, f) with y the oracle value.  Densities and the total
energy (gas and dust densities) use f = 1e-300 (plain relative error); the momenta,
which pass through zero, use f = rho c_s of the oracle cell (gas) or rho_d c_s (dust).
"""
import numpy as np


def sound_speed(E, gamma):
    rho = E[4]
    m2 = E[0] ** 2 + E[1] ** 2 + E[2] ** 2
    p = (gamma - 1.0) * (E[3] - 0.5 * m2 / rho)
    return np.sqrt(gamma * np.maximum(p, 0.0) / rho), p


def field_errors(gpu, ref, gamma, n_dust):
    """Returns a dict name -> max relative error over cells (A-metric above)."""
    cs, p_ref = sound_speed(ref, gamma)
    _, p_gpu = sound_speed(gpu, gamma)
    out = {}
    names = ["rho_u", "rho_v", "rho_w", "E", "rho"]
    for f in range(5):
        if f < 3:
            scale = np.maximum(np.abs(ref[f]), ref[4] * cs)
        else:
            scale = np.maximum(np.abs(ref[f]), 1e-300)
        out[names[f]] = float(np.max(np.abs(gpu[f] - ref[f]) / scale))
    # pressure is derived: p = (gamma-1)(E - KE) with KE/p ~ Mach^2, so a relative
    # agreement eps of the conserved variables is an agreement eps (gamma-1) E in p
    out["p"] = float(np.max(np.abs(p_gpu - p_ref) / ((gamma - 1.0) * np.abs(ref[3]))))
    for s in range(n_dust):
        o = 5 + 4 * s
        rd = ref[o + 3]
        for q, nm in enumerate(("u", "v", "w")):
            scale = np.maximum(np.abs(ref[o + q]), np.abs(rd) * cs)
            scale = np.maximum(scale, 1e-300)
            out[f"dust{s}_rho_{nm}"] = float(np.max(np.abs(gpu[o + q] - ref[o + q]) / scale))
        out[f"dust{s}_rho"] = float(np.max(np.abs(gpu[o + 3] - rd) / np.maximum(np.abs(rd), 1e-300)))
    return out


def worst(errs):
    k = max(errs, key=errs.get)
    return k, errs[k]


def cell_errors(gpu, ref, gamma):
    """Per-cell error array over the gas fields and pressure (same metric as above)."""
    cs, p_ref = sound_speed(ref, gamma)
    _, p_gpu = sound_speed(gpu, gamma)
    out = []
    for f in range(5):
        if f < 3:
            scale = np.maximum(np.abs(ref[f]), ref[4] * cs)
        else:
            scale = np.maximum(np.abs(ref[f]), 1e-300)
        out.append(np.abs(gpu[f] - ref[f]) / scale)
    out.append(np.abs(p_gpu - p_ref) / ((gamma - 1.0) * np.abs(ref[3])))
    return np.max(np.array(out), axis=0)


def conditioned_check(gpu, ref, ref_perturbed, gamma, tol=1e-10, factor=100.0):
    """Parity limited by the conditioning of the scheme: every cell agrees to tol, or to
    within `factor` times the oracle's own divergence under a rounding-sized input
    perturbation (ref_perturbed).  Returns (ok, stats)."""
    e = cell_errors(gpu, ref, gamma)
    s = cell_errors(ref_perturbed, ref, gamma)
    bound = np.maximum(tol, factor * s)
    ok = bool(np.all(e <= bound))
    stats = dict(max_err=float(e.max()), frac_over_tol=float(np.mean(e > tol)),
                 max_self_sensitivity=float(s.max()), frac_sensitive=float(np.mean(factor * s > tol)),
                 worst_ratio=float(np.max(e / bound)))
    return ok, stats
