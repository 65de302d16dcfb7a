"""Pins of the oracle's indirect gravity (Sect. 2.10): the star, accelerated by an
asymmetric disc, drags the star-centred frame; every fluid element feels the opposite
of the star's acceleration.

For the stationary disc with its density (gas and dust) modulated by 1 + eps cos(theta -
phi) -- velocities and temperature unchanged -- discrete orthogonality over the theta
cells gives the sums in closed form, A = eps (n/2) cos(phi) W and B = eps (n/2) sin(phi) W
with W = sum over (z, r) cells of the column density times V r / (r^2 + z^2)^(3/2); the
extra source in the radial momentum of a cell is -GM rho V (A cos(theta) + B sin(theta)):
inward where the excess mass sits (the star is pulled towards it), outward opposite."""
import numpy as np
import pytest

import oracle
from paper_2207_04252_amd import synth

BASE = synth.C5_ADJOINT.scaled(10, 24, 8).with_(vortex_amp=0.0, noise_amp=0.0)


def modulated(cfg, eps, phi):
    o = oracle.Oracle(cfg)
    x = o.state()
    th = (np.arange(cfg.nth) + 0.5) * 2 * np.pi / cfg.nth
    mod = 1.0 + eps * np.cos(th - phi)
    return x * mod[None, None, None, :], x


def ring_weight(cfg, o, x0):
    """W = sum over (z, r) of the column density (gas + dust) V r / (r^2 + z^2)^(3/2)."""
    geo = o.geometry()
    rc, zc, V = geo["rc"], geo["zc"], geo["V"]
    col = x0[4, :, :, 0] + sum(x0[5 + 4 * s + 3, :, :, 0] for s in range(cfg.n_dust))
    w = V[None, :] * rc[None, :] / (rc[None, :] ** 2 + zc[:, None] ** 2) ** 1.5
    return float(np.sum(col * w))


def test_axisymmetric_state_has_no_indirect_term():
    """The sums of an axisymmetric state vanish to rounding (sum of cos over the ring)."""
    cfg = BASE.with_(indirect=True)
    o = oracle.Oracle(cfg)
    W = ring_weight(cfg, o, o.state())
    A, B = o.indirect_sums()
    assert abs(A) < 1e-14 * cfg.nth * W and abs(B) < 1e-14 * cfg.nth * W


@pytest.mark.parametrize("phi", [0.3, 2.0, 4.4])
def test_m1_sums_closed_form(phi):
    cfg = BASE.with_(indirect=True)
    eps = 1e-2
    x, x0 = modulated(cfg, eps, phi)
    o = oracle.Oracle(cfg)
    o.set_state(x)
    A, B = o.indirect_sums()
    W = ring_weight(cfg, o, x0)
    n = cfg.nth
    assert A == pytest.approx(eps * n / 2 * np.cos(phi) * W, rel=1e-12)
    assert B == pytest.approx(eps * n / 2 * np.sin(phi) * W, rel=1e-12)


def test_m1_force_direction_and_size():
    phi = 1.1
    eps = 1e-2
    cfg = BASE.with_(indirect=True)
    x, x0 = modulated(cfg, eps, phi)
    on = oracle.Oracle(cfg)
    on.set_state(x)
    off = oracle.Oracle(cfg.with_(indirect=False))
    off.set_state(x)
    d = on.eval_G() - off.eval_G()
    A, B = on.indirect_sums()
    geo = on.geometry()
    th = (np.arange(cfg.nth) + 0.5) * 2 * np.pi / cfg.nth
    # radial momentum: -GM rho V (A cos + B sin) = -GM rho V (n/2) eps W cos(theta - phi)
    expect = -cfg.GM * x[4] * geo["V"][None, :, None] * (A * np.cos(th) + B * np.sin(th))[None, None, :]
    np.testing.assert_allclose(d[0], expect, rtol=1e-10, atol=1e-12 * np.abs(expect).max())
    jn = int(np.argmin(np.abs(np.angle(np.exp(1j * (th - phi))))))
    jf = int(np.argmin(np.abs(np.angle(np.exp(1j * (th - phi - np.pi))))))
    assert np.all(d[0][:, :, jn] < 0) and np.all(d[0][:, :, jf] > 0)
    # no vertical component, no mass source; dust feels the same acceleration
    assert np.all(d[2] == 0.0) and np.all(d[4] == 0.0)
    np.testing.assert_allclose(d[5] / x[8] / geo["V"][None, :, None], d[0] / x[4] / geo["V"][None, :, None],
                               rtol=1e-9, atol=1e-12 * np.abs(d[0] / x[4]).max())
