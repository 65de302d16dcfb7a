"""Pins of the oracle's Epstein / Stokes drag law (Sect. 2.9).

The stopping time of a grain of radius r_p and material density rho_s in gas of density
rho and isothermal sound speed c_s is pinned by what physics fixes independently of the
printed formula: the Epstein time scales as 1/(rho c_s) and reproduces the Stokes number
it was built from at r = 1 of the stationary disc; the Stokes-regime time is the
textbook viscous law 2 rho_s r_p^2 / (9 eta) with the kinetic-theory viscosity
eta = rho lambda c_s / 2, independent of the gas density; the two regimes meet
continuously at r_p = 9 lambda / 4 with the large grains in dense gas on the Stokes side.
The drag operator and the stiffness check are then tied to these stopping times.
"""
import math

import numpy as np
import pytest

from paper_2207_04252_amd import synth


def _box(oracle_mod, sizes, rho_s=2.0, mfp=1e-3, n=64):
    """2D uniform-grid box, gas at rest with per-cell density and sound speed set by hand."""
    cfg = synth.C1_SOD.with_(nr=n, nth=4, nz=1, GM=1.0, stokes=(0.1,) * len(sizes),
                             eps_dust=(0.0,) * len(sizes), hd_over_h=(1.0,) * len(sizes),
                             drag_law=1, grain_size=tuple(sizes),
                             grain_density=(rho_s,) * len(sizes), mfp_coef=mfp)
    return cfg, oracle_mod.Oracle(cfg)


def _set_gas(o, cfg, rho, cs):
    """rho, cs: arrays over r (length nr), isothermal cs^2 = p / rho."""
    s = o.state()
    s[:] = 0.0
    p = rho * cs * cs
    s[4] = rho[None, :, None]
    s[3] = (p / (cfg.gamma - 1.0))[None, :, None]
    for q in range(cfg.n_dust):
        s[5 + 4 * q + 3] = 1e-3
    o.set_state(s)


def test_epstein_scaling(oracle_mod):
    """Small grains (Epstein everywhere): t doubles when rho halves at fixed c_s and when
    c_s halves at fixed rho; t rho c_s is the constant rho_s r_p."""
    rp, rs = 1e-4, 2.0
    cfg, o = _box(oracle_mod, (rp,), rho_s=rs, mfp=1e-3)
    rho = np.geomspace(1e-3, 1.0, cfg.nr)      # switch at 9 mfp/(4 r_p) = 22.5: Epstein
    for cs in (0.3, 0.15):
        _set_gas(o, cfg, rho, np.full(cfg.nr, cs))
        t = o.stopping_times()[0, 0, :, 0]
        assert np.allclose(t * rho * cs, rs * rp, rtol=1e-14, atol=0)
        assert np.allclose(t[:-1] / t[1:], rho[1:] / rho[:-1], rtol=1e-13)
    t1 = None
    for cs in (0.3, 0.15):
        _set_gas(o, cfg, rho, np.full(cfg.nr, cs))
        t = o.stopping_times()[0, 0, :, 0]
        if t1 is None:
            t1 = t
        else:
            assert np.allclose(t / t1, 2.0, rtol=1e-14)
    o.close()


def test_stokes_regime_is_viscous_law(oracle_mod):
    """Large grains in dense gas: t = 2 rho_s r_p^2 / (9 eta), eta = rho lambda c_s / 2,
    lambda = mfp / rho; the same at every density above the switch."""
    rp, rs, mfp, cs = 0.05, 3.0, 1e-3, 0.2
    cfg, o = _box(oracle_mod, (rp,), rho_s=rs, mfp=mfp)
    rho = np.geomspace(0.1, 10.0, cfg.nr)       # switch at 9 mfp / (4 r_p) = 0.045
    _set_gas(o, cfg, rho, np.full(cfg.nr, cs))
    t = o.stopping_times()[0, 0, :, 0]
    lam = mfp / rho
    eta = 0.5 * rho * lam * cs
    assert np.allclose(t, 2.0 * rs * rp * rp / (9.0 * eta), rtol=1e-14, atol=0)
    assert np.ptp(t) <= 1e-14 * t.max()
    o.close()


def test_regime_switch_continuous_and_oriented(oracle_mod):
    """Across rho* = 9 mfp / (4 r_p) the stopping time is continuous; below rho* it goes
    as 1/rho (Epstein), above it is flat (Stokes)."""
    rp, mfp, cs = 0.01, 2e-3, 0.1
    cfg, o = _box(oracle_mod, (rp,), mfp=mfp, n=8)
    rs = 9.0 * mfp / (4.0 * rp)
    rho = rs * np.array([0.25, 0.5, 1 - 1e-9, 1 + 1e-9, 2.0, 4.0, 8.0, 16.0])
    _set_gas(o, cfg, rho, np.full(cfg.nr, cs))
    t = o.stopping_times()[0, 0, :, 0]
    assert abs(t[2] - t[3]) <= 1e-8 * t[2]
    assert np.allclose(t[0] / t[1], 2.0, rtol=1e-13)
    assert np.allclose(t[4:], t[4], rtol=1e-13)
    assert abs(t[4] - t[3]) <= 1e-8 * t[3]
    o.close()


def test_disc_grains_reproduce_stokes_number(oracle_mod):
    """epstein_grains sizes the grains so that Omega_K t^E = St at r = 1, z = 0 of the
    stationary disc; the smallest species is in the Epstein regime there."""
    base = synth.C4_LARGE.scaled(64, 4, 2).with_(vortex_amp=0.0, noise_amp=0.0, log_r=False,
                                                  r_in=0.5, r_out=1.5)
    cfg = synth.epstein_grains(base)
    o = oracle_mod.Oracle(cfg)
    t = o.stopping_times()
    g = o.geometry()
    i = int(np.argmin(np.abs(g["rc"] - 1.0)))
    r = g["rc"][i]
    # stationary midplane (App. A): rho = rho_mid0 r^beta_rho exp(GM/c^2 (1/s - 1/r)) at
    # |z| = dz/2, c^2 = h0^2 GM r^beta_T; Epstein t = rho_s r_p / (rho c)
    zc = cfg.z_half / 2.0
    c2 = cfg.h0 ** 2 * cfg.GM * r ** cfg.beta_T
    rho = cfg.rho_mid0 * r ** cfg.beta_rho * math.exp(cfg.GM / c2 * (1 / math.hypot(r, zc) - 1 / r))
    te = cfg.grain_density[0] * cfg.grain_size[0] / (rho * math.sqrt(c2))
    assert abs(t[0, 1, i, 0] / te - 1.0) < 1e-12
    # at r = 1 exactly the Stokes number is recovered (closed form of the sizing)
    st1 = cfg.grain_density[0] * cfg.grain_size[0] / (cfg.rho_mid0 * cfg.h0)
    assert abs(st1 - cfg.stokes[0]) < 1e-15
    o.close()


def test_drag_operator_uses_law(oracle_mod):
    """Gas at rest, dust moving in w with two grain sizes (one per regime): the
    w-components of G are +-rho_d w_d V / t_s with the pinned stopping times, the
    exchange is exact, and the energy source is zero (gas at rest)."""
    rp = (1e-4, 0.05)
    cfg, o = _box(oracle_mod, rp, rho_s=2.0, mfp=1e-3, n=16)
    rho = np.geomspace(0.05, 5.0, cfg.nr)
    cs = 0.2
    _set_gas(o, cfg, rho, np.full(cfg.nr, cs))
    s = o.state()
    wd = (0.03, -0.02)
    for q in range(2):
        s[5 + 4 * q + 2] = s[5 + 4 * q + 3] * wd[q]
    o.set_state(s)
    t = o.stopping_times()
    G = o.eval_G(with_dust=True, subtract_R0=False)
    V = o.geometry()["V"]
    for i in range(3, cfg.nr - 3):
        d = [1e-3 * wd[q] / t[q, 0, i, 0] * V[i] for q in range(2)]
        assert np.allclose(G[2, 0, i], d[0] + d[1], rtol=1e-13, atol=0)
        for q in range(2):
            assert np.allclose(G[5 + 4 * q + 2, 0, i], -d[q], rtol=1e-13, atol=0)
    o.close()


def test_stiffness_uses_cell_stopping_time(oracle_mod):
    """min_stopping_time is the minimum over cells; a step with dt at that value is
    refused with ESTIFF, one just below it is taken."""
    cfg, o = _box(oracle_mod, (1e-4,), mfp=1e-3, n=16)
    rho = np.geomspace(0.05, 5.0, cfg.nr)
    _set_gas(o, cfg, rho, np.full(cfg.nr, 0.2))
    t = o.stopping_times()
    tmin = o.min_stopping_time()
    assert tmin == t.min()
    st, _ = o.step(1, dt=tmin)
    assert st == -7
    o.close()
    cfg, o = _box(oracle_mod, (1e-4,), mfp=1e-3, n=16)
    _set_gas(o, cfg, rho, np.full(cfg.nr, 0.2))
    st, _ = o.step(1, dt=0.5 * tmin)
    assert st == 0
    o.close()


def test_workload_spans_both_regimes(oracle_mod):
    """The Epstein-law disc of the parity tests holds cells of each regime for the middle
    species."""
    cfg = synth.epstein_grains(synth.C4_LARGE.scaled(96, 64, 16))
    o = oracle_mod.Oracle(cfg, noise=synth.noise(cfg))
    s = o.state()
    rho = s[4]
    rsw = 9.0 * cfg.mfp_coef / (4.0 * cfg.grain_size[1])
    frac = float(np.mean(rho > rsw))
    assert 0.05 < frac < 0.95, frac
    o.close()
