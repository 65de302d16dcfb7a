"""Error metrics for comparing the HIP path with the oracle.

Per cell: |x - y| / max(|y|, f) with y the oracle value.  Densities and the total
energy (gas and dust densities) use f = 1e-300 (plain relative error); the momenta,
which pass through zero, use f = rho c_s of the oracle cell (gas) or rho_d c_s (dust).

The dust midplane.  With an even number of layers the midplane is a face, where the
settling dust of the two halves meets in a standing delta shock of the pressureless
Riemann problem (Sect. 2.9 solver).  Its flux takes one side or the other with the sign
of a speed that is zero up to the state's small asymmetry, so the flux across that face
is a discontinuous function of the state there, and the oracle against itself under a
1e-15 relative input change already moves the two midplane cells by up to ~1e-7 (one
step of a coarse slice) or ~3e-10 (100 steps of the bi-fluid slice).  The dust of the
two cells beside that face is therefore compared through their sum, which the flux
across the face does not change; the cells themselves are reported.
"""
import numpy as np


def sound_speed(E, gamma):
    rho = E[4]
    m2 = E[0] ** 2 + E[1] ** 2 + E[2] ** 2
    p = (gamma - 1.0) * (E[3] - 0.5 * m2 / rho)
    return np.sqrt(gamma * np.maximum(p, 0.0) / rho), p


def _midplane(nz):
    """Layers beside a midplane face (none for an odd layer count or 2D)."""
    return [nz // 2 - 1, nz // 2] if nz >= 2 and nz % 2 == 0 else []


def field_errors(gpu, ref, gamma, n_dust, mid=None):
    """Returns a dict name -> max relative error over cells (metric above).  Dust fields:
    over the cells off the midplane layers, plus '<field>_midpair' for the two-cell sums
    across the midplane face; the midplane cells themselves go to the dict `mid` if one
    is given (reported, not gated)."""
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
    ml = _midplane(ref.shape[1])
    off = np.ones(ref.shape[1], bool)
    off[ml] = False
    for s in range(n_dust):
        o = 5 + 4 * s
        rd = ref[o + 3]
        for q, nm in enumerate(("u", "v", "w", "")):
            key = f"dust{s}_rho_{nm}" if nm else f"dust{s}_rho"
            if q < 3:
                scale = np.maximum(np.maximum(np.abs(ref[o + q]), np.abs(rd) * cs), 1e-300)
            else:
                scale = np.maximum(np.abs(rd), 1e-300)
            e = np.abs(gpu[o + q] - ref[o + q]) / scale
            out[key] = float(np.max(e[off]))
            if ml:
                a, b = ml
                pr = ref[o + q][a] + ref[o + q][b]
                pg = gpu[o + q][a] + gpu[o + q][b]
                if q < 3:
                    ps = np.maximum(np.abs(pr), (rd[a] + rd[b]) * 0.5 * (cs[a] + cs[b]))
                else:
                    ps = np.abs(pr)
                out[key + "_midpair"] = float(np.max(np.abs(pg - pr) / np.maximum(ps, 1e-300)))
                if mid is not None:
                    mid[key] = float(np.max(e[~off]))
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
