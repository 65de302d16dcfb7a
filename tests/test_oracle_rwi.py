"""Pins of the oracle's Rossby-wave-instability initial state (Sect. 4.3).

The state is a Gaussian overdensity bump on the stationary disc at unchanged temperature,
with the azimuthal velocity rebalanced radially and an m-mode radial-velocity seed.  Pinned
by what the construction must satisfy independently of its formulas: the density ratio
to the stationary flow is the printed bump, the temperature is untouched, the continuous
radial momentum balance (centrifugal = gravity + pressure gradient) holds to the accuracy
of a finite-difference check that converges at second order, and the radial velocity has
the single azimuthal mode m with the printed amplitude.
"""
import math

import numpy as np

from paper_2207_04252_amd import synth


def _fields(o, cfg):
    s = o.state()
    rho = s[4]
    u, v = s[0] / rho, s[1] / rho
    p = (cfg.gamma - 1) * (s[3] - 0.5 * rho * (u * u + v * v))
    return rho, u, v, p


def test_bump_density_and_temperature(oracle_mod):
    cfg = synth.C6_RWI.scaled(64, 16, 8).with_(noise_amp=0.0)
    base = cfg.with_(rwi_delta=0.0, rwi_eps=0.0)
    o, o0 = oracle_mod.Oracle(cfg), oracle_mod.Oracle(base)
    rho, _, _, p = _fields(o, cfg)
    rho0, _, _, p0 = _fields(o0, base)
    rc = o.geometry()["rc"]
    bump = 1 + cfg.rwi_delta * np.exp(-((rc - cfg.rwi_r0) / (math.sqrt(2) * cfg.rwi_dr)) ** 2)
    assert np.allclose(rho / rho0, bump[None, :, None], rtol=1e-14, atol=0)
    assert np.allclose(p / rho, p0 / rho0, rtol=1e-12, atol=0)
    o.close(); o0.close()


def test_radial_balance_converges(oracle_mod):
    """Midplane residual of v^2/r - GM r/s^3 - (1/rho) dP/dr with dP/dr from central
    differences of the sampled state: second order in the sampling step, so a wrong
    rebalancing term would leave an O(1) residual."""
    res = []
    for nr in (400, 800):
        cfg = synth.C6_RWI.with_(nr=nr, nth=4, nz=1, noise_amp=0.0, rwi_eps=0.0, log_r=False,
                                 r_in=0.7, r_out=1.3)
        o = oracle_mod.Oracle(cfg)
        rho, _, v, p = _fields(o, cfg)
        r = o.geometry()["rc"]
        rho, v, p = rho[0, :, 0], v[0, :, 0], p[0, :, 0]
        dpdr = (p[2:] - p[:-2]) / (r[2:] - r[:-2])
        rr = r[1:-1]
        resid = v[1:-1] ** 2 / rr - cfg.GM / rr ** 2 - dpdr / rho[1:-1]
        res.append(np.abs(resid).max() / (cfg.GM / 1.0))
        o.close()
    assert res[1] < 0.3 * res[0], res          # second order: ratio ~ 1/4
    assert res[1] < 1e-5, res


def test_seed_is_single_mode(oracle_mod):
    cfg = synth.C6_RWI.scaled(32, 64, 4).with_(noise_amp=0.0)
    o = oracle_mod.Oracle(cfg)
    _, u, _, _ = _fields(o, cfg)
    base = oracle_mod.Oracle(cfg.with_(rwi_delta=0.0, rwi_eps=0.0))
    _, _, v0, _ = _fields(base, cfg)
    rc = o.geometry()["rc"]
    spec = np.fft.rfft(u, axis=-1) * 2 / cfg.nth
    m = cfg.rwi_m
    other = np.delete(np.abs(spec), m, axis=-1).max()
    assert other < 1e-12 * np.abs(spec[..., m]).max()
    # amplitude eps v_theta0 exp(-(r - r0)^2 / (2 dr^2)); the phase is that of
    # sin(m theta) sampled at the cell centres theta_j = (j + 1/2) dtheta
    want = cfg.rwi_eps * v0.mean(axis=-1) * np.exp(-((rc - cfg.rwi_r0) / cfg.rwi_dr) ** 2 / 2)
    got = np.abs(spec[..., m])
    phase = np.angle(spec[..., m][np.abs(spec[..., m]) > 1e-3 * np.abs(spec[..., m]).max()])
    assert np.allclose(phase, m * np.pi / cfg.nth - np.pi / 2, atol=1e-9)
    assert np.allclose(got, want, rtol=1e-9, atol=1e-14 * cfg.rwi_eps)
    o.close(); base.close()
