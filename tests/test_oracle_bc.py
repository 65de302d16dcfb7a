"""Pins of the oracle's boundary conditions (Sect. 2.4): wave-killing radial zones,
sheared damped vertical zones and the vertical outflow condition.

The paper names these conditions without formulas; the damping form (quadratic ramp,
relaxation over damp_tau orbital periods) is a reading, so its constants are unpinned.
What is pinned: the stationary flow is untouched by every option (bitwise, over many
steps, and the empty-run residual is unchanged); damping is a local, linear relaxation of
the five gas deviations at one rate per cell, confined to the zones, growing toward the
boundary and leaving the dust alone; the outflow condition is the same operator as a
taller domain whose extra layers carry the boundary cell's relative deviation (brute
force).
"""
import math

import numpy as np
import pytest

from paper_2207_04252_amd import synth

GAS_DISC = synth.C3_BIFLUID.scaled(24, 32, 8).with_(vortex_amp=0.0, noise_amp=0.0, stokes=(),
                                                     eps_dust=(), hd_over_h=())


@pytest.mark.parametrize("bc", [dict(bc_r=1), dict(bc_z=1), dict(bc_z=2),
                                dict(bc_r=1, bc_z=1), dict(bc_r=1, bc_z=2)])
def test_equilibrium_bitwise_and_residual_unchanged(oracle_mod, bc):
    cfg = GAS_DISC.with_(**bc)
    o = oracle_mod.Oracle(cfg)
    ref = oracle_mod.Oracle(GAS_DISC)
    assert np.array_equal(o.residual(), ref.residual())
    s0 = o.state()
    st, _ = o.step(30)
    assert st == 0
    assert np.array_equal(o.state(), s0)
    o.close()
    ref.close()


def _perturbed(oracle_mod, cfg, seed):
    o = oracle_mod.Oracle(cfg)
    s = o.state()
    rng = np.random.default_rng(seed)
    s[:5] *= 1.0 + 1e-3 * rng.standard_normal(s[:5].shape)
    for f in (0, 2):   # the stationary flow has u = w = 0
        s[f] += 1e-5 * s[4] * rng.standard_normal(s[4].shape)
    o.set_state(s)
    return o, s


def test_damping_is_local_linear_relaxation(oracle_mod):
    base = synth.C3_BIFLUID.scaled(40, 16, 16).with_(vortex_amp=0.0, noise_amp=0.0)
    on = base.with_(bc_r=1, bc_z=2)
    g = None
    rates = []
    for seed in (1, 2):
        o_off, s = _perturbed(oracle_mod, base, seed)
        o_on = oracle_mod.Oracle(on)
        o_on.set_state(s)
        g = o_on.geometry()
        E0 = oracle_mod.Oracle(base).state()
        dG = o_on.eval_G(True, True) - o_off.eval_G(True, True)
        dev = s - E0
        # dust untouched
        assert np.all(dG[5:] == 0.0)
        rc, zc, V = g["rc"], g["zc"], g["V"]
        in_r = (rc < on.damp_r_in * on.r_in) | (rc > on.damp_r_out * on.r_out)
        in_z = np.abs(zc) > on.damp_z * on.z_half
        zone = in_z[:, None] | in_r[None, :]
        # outside the zones: no change at all
        assert np.all(dG[:5][:, ~zone] == 0.0)
        # inside: dG = -V k E' with one rate k per cell for the five gas fields
        k = -dG[:5] / (V[None, None, :, None] * dev[:5])
        kc = np.median(k, axis=(0, 3))
        assert np.all(kc[zone] > 0)
        assert np.allclose(k[:, zone, :], kc[zone][None, :, None], rtol=1e-9)
        rates.append(kc)
    # the rate is a property of the cell, not of the state
    assert np.allclose(rates[0], rates[1], rtol=1e-12)
    kc = rates[0]
    # radial zones (midplane-adjacent layer, below the vertical zone): rising toward each
    # radial boundary, at most one e-fold per damp_tau orbital period at the boundary
    kmid = kc[on.nz // 2]
    inner = np.where(rc < on.damp_r_in * on.r_in)[0]
    outer = np.where(rc > on.damp_r_out * on.r_out)[0]
    assert np.all(np.diff(kmid[inner]) < 0) and np.all(np.diff(kmid[outer]) > 0)
    om = lambda r: math.sqrt(on.GM / r ** 3)
    assert 0 < kmid[0] <= om(on.r_in) / (2 * math.pi * on.damp_tau)
    assert 0 < kmid[-1] <= om(on.r_out) / (2 * math.pi * on.damp_tau)
    # vertical zone (a column outside the radial zones): rising toward |z| = z_half
    i = int(np.argmin(np.abs(rc - 1.0)))
    col = kc[:, i]
    top = np.where(zc > on.damp_z * on.z_half)[0]
    assert np.all(np.diff(col[top]) > 0)
    assert np.allclose(col[::-1], col, rtol=1e-12)          # mirror symmetric in z
    assert col[-1] <= om(rc[i]) / (2 * math.pi * on.damp_tau)


def test_outflow_equals_extended_domain(oracle_mod):
    """nz layers with outflow ghosts against nz + 4 layers (same dz, stationary ghosts)
    whose two extra layers on each side carry the boundary cell's gas deviation relative
    to the stationary density and its dust variables: the operator of the original cells
    agrees (gas and dust), with no positivity fallback or NaN."""
    nz, ext = 8, 2
    base = synth.C3_BIFLUID.scaled(16, 16, nz).with_(vortex_amp=0.0, noise_amp=0.0)
    cfg = base.with_(bc_z=1)
    big = base.with_(nz=nz + 2 * ext, z_half=base.z_half * (nz + 2 * ext) / nz)
    o, s = _perturbed(oracle_mod, cfg, 7)
    # dust perturbed too, so that its ghosts matter
    rng = np.random.default_rng(8)
    s[5:] *= 1.0 + 1e-2 * rng.standard_normal(s[5:].shape)
    o.set_state(s)
    E0 = oracle_mod.Oracle(base).state()
    ob = oracle_mod.Oracle(big)
    Eb0 = ob.state()
    assert np.allclose(Eb0[:, ext:-ext], E0, rtol=1e-13, atol=0)
    sb = Eb0.copy()
    sb[:5, ext:-ext] = Eb0[:5, ext:-ext] + (s[:5] - E0[:5])
    sb[5:, ext:-ext] = s[5:]
    for q in range(ext):
        # the boundary cell's deviation relative to the stationary density
        lo = Eb0[4, q] / E0[4, 0]
        hi = Eb0[4, -1 - q] / E0[4, -1]
        sb[:5, q] = Eb0[:5, q] + (s[:5, 0] - E0[:5, 0]) * lo[None]
        sb[:5, -1 - q] = Eb0[:5, -1 - q] + (s[:5, -1] - E0[:5, -1]) * hi[None]
        sb[5:, q] = s[5:, 0]
        sb[5:, -1 - q] = s[5:, -1]
    ob.set_state(sb)
    G = o.eval_G(True, True)
    Gb = ob.eval_G(True, True)[:, ext:-ext]
    assert np.all(np.isfinite(G))
    scale = np.abs(G).max(axis=(1, 2, 3), keepdims=True)
    assert np.all(np.abs(G - Gb) <= 1e-11 * scale), np.abs(G - Gb).max(axis=(1, 2, 3)) / scale[:, 0, 0, 0]
    # and differs from the stationary-ghost operator in the boundary layers only
    o2 = oracle_mod.Oracle(base)
    o2.set_state(s)
    d = np.abs(G - o2.eval_G(True, True)).max(axis=(0, 2, 3))
    assert d[2:-2].max() == 0.0 and d[0] > 0 and d[-1] > 0
