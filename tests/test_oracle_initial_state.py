"""Pins of the oracle's initial disc state: the dust layer (Sect. 4.4 profile, read with
the configuration's scale height) and the column Gaussian vortex (the configuration's
recipe: centre vorticity 2 Ro Omega_K with Ro = -amplitude), each against what
quadrature or finite differences of the sampled state give."""
import numpy as np
import pytest

from paper_2207_04252_amd import synth


def test_dust_layer_column_and_scale_height(oracle_mod):
    """At r = 1 the dust column over the gas column is the dust-to-gas ratio eps (to the
    thin-disc correction of the gas column, O((H/r)^2)), and the dust's second vertical
    moment is H_d^2 with H_d = 0.3 H and H = c_iso / Omega_K = 0.05 (the configuration's
    scale height, exp(-z^2 / 2H^2) for the gas)."""
    eps, hd = 0.01, 0.3
    cfg = synth.C3_BIFLUID.scaled(4, 4, 512).with_(
        r_in=0.999, r_out=1.001, z_half=0.3, vortex_amp=0.0, noise_amp=0.0,
        eps_dust=(eps,), hd_over_h=(hd,))
    o = oracle_mod.Oracle(cfg)
    s = o.state()
    zc = o.geometry()["zc"]
    i = 1
    gas = s[4][:, i, 0]
    dust = s[8][:, i, 0]
    ratio = dust.sum() / gas.sum()
    assert ratio == pytest.approx(eps, rel=5e-3), ratio
    H = 0.05 * o.geometry()["rc"][i] ** 1.25        # c_iso / Omega_K with T ~ r^-1/2
    m2 = np.sum(zc ** 2 * dust) / dust.sum()
    assert np.sqrt(m2) == pytest.approx(hd * H, rel=1e-6), (np.sqrt(m2), hd * H)
    # the gas layer's own second moment is H (thin disc), not sqrt(2) H
    mg = np.sqrt(np.sum(zc ** 2 * gas) / gas.sum())
    assert mg == pytest.approx(H, rel=1e-2), (mg, H)


def test_vortex_centre_vorticity(oracle_mod):
    """The vertical vorticity of the velocity perturbation at the vortex centre, by central
    differences of the sampled state on a fine 2D mesh, is 2 Ro Omega_K(r_v) with
    Ro = -amplitude (anticyclonic), and the perturbation vanishes far from the centre."""
    amp = 1e-3
    cfg = synth.C2_DISC.with_(nr=400, nth=2048, nz=1, r_in=0.9, r_out=1.1, vortex_amp=amp,
                              noise_amp=0.0, name="vortex_2d")
    o = oracle_mod.Oracle(cfg)
    s = o.state()
    g = o.geometry()
    rc = g["rc"]
    th = (np.arange(cfg.nth) + 0.5) * 2 * np.pi / cfg.nth
    v0 = np.array([oracle_mod.equilibrium(cfg, r, 0.0)[2] for r in rc])
    rho = s[4][0]
    ur = s[0][0] / rho
    dvt = s[1][0] / rho - v0[:, None]
    i = int(np.argmin(np.abs(rc - cfg.vortex_r0)))
    j = int(np.argmin(np.abs(th - cfg.vortex_th0)))
    dr = (rc[i + 1] - rc[i - 1])
    dth = th[j + 1] - th[j - 1]
    r = rc[i]
    omega = ((rc[i + 1] * dvt[i + 1, j] - rc[i - 1] * dvt[i - 1, j]) / dr
             - (ur[i, j + 1] - ur[i, j - 1]) / dth) / r
    # the centre lies between mesh points: evaluate the closed-form shape's drop there
    X = r - cfg.vortex_r0
    Y = cfg.vortex_r0 * (th[j] - cfg.vortex_th0)
    shape = np.exp(-X ** 2 / (2 * cfg.vortex_sig_r ** 2) - Y ** 2 / (2 * cfg.vortex_sig_a ** 2))
    want = 2 * (-amp) * np.sqrt(cfg.GM / cfg.vortex_r0 ** 3)
    assert omega / shape == pytest.approx(want, rel=2e-3), (omega, want, shape)
    assert omega < 0
    far = np.abs(th - cfg.vortex_th0) > 1.5
    assert np.max(np.abs(ur[:, far])) < 1e-12 and np.max(np.abs(dvt[:, far])) < 1e-12
