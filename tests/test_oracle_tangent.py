"""Pins of the oracle's forward-mode (dual-number) derivatives against central finite
differences of the oracle's own FP64 step: the tangent of n RK2 steps (Sect. 2.5) with
respect to the state, and the tangents of the vortex-core dust mass with respect to the
initial vortex amplitude and the Stokes number.  These are the references the GPU
adjoint is checked against.

The limited reconstruction and the pressureless dust solver are only piecewise smooth.
Finite differences measure the derivative only away from their kinks, so the pins use
directions and states that stay clear of them: smooth perturbation patterns, a vortex
centred off the mesh's faces (a centre on a face makes one-sided differences of the
velocities exactly zero there), and scalar functionals rather than per-cell values.
Two kinks of the primitive-variable reconstruction sit on the initial disc itself and are
avoided explicitly: the pressure deviation of the initial state is zero up to rounding
(the vortex and the density noise leave the pressure unchanged), so the gas pin starts
from a state ten steps into the run of a noise-free disc; and the settling dust layer is
mirror-symmetric about the midplane, where it meets in a standing delta shock whose
flux switches side with the sign of its speed (Sect. 2.9 solver), so amplitude directions
are taken mirror-symmetric too."""
import numpy as np
import pytest

import oracle
from paper_2207_04252_amd import synth

GAS = synth.C2_DISC.scaled(10, 24, 8).with_(vortex_r0=1.0137, vortex_th0=3.1829, noise_amp=0.0)
DUST = synth.C5_ADJOINT.scaled(10, 24, 8).with_(vortex_r0=1.0137, vortex_th0=3.1829)


def smooth_direction(cfg, x0, rng):
    """Each gas field's deviation from the stationary flow, modulated by a smooth random
    pattern (mirror-symmetric about the midplane)."""
    bg = oracle.Oracle(cfg).background(0)  # (nz, nr, nf)
    th = (np.arange(cfg.nth) + 0.5) * 2 * np.pi / cfg.nth
    rr = (np.arange(cfg.nr) + 0.5) / cfg.nr
    zz = (np.arange(cfg.nz) + 0.5) / cfg.nz
    v = np.zeros_like(x0)
    for f in range(5):
        a, b = rng.uniform(0, 2 * np.pi, size=2)
        mod = (1.0 + 0.5 * np.sin(2 * th[None, None, :] + a) * np.cos(np.pi * rr[None, :, None] + b)
               * np.cos(2 * np.pi * (zz[:, None, None] - 0.5)))
        v[f] = 1e-2 * (x0[f] - bg[:, :, f][:, :, None]) * mod
    return v


def test_tangent_state_matches_finite_differences():
    cfg = GAS
    o = oracle.Oracle(cfg)
    assert o.step(10)[0] == 0
    x0 = o.state()
    st, dts = o.step(3)
    assert st == 0
    rng = np.random.default_rng(11)
    v = smooth_direction(cfg, x0, rng)
    status, xn, dxn = oracle.tangent_state(cfg, x0, v, None, dts)
    assert status == 0
    assert np.array_equal(xn, o.state())
    h = 1e-4
    outs = []
    for sg in (1.0, -1.0):
        o2 = oracle.Oracle(cfg)
        o2.set_state(x0 + sg * h * v)
        assert o2.step(len(dts), dt_list=dts)[0] == 0
        outs.append(o2.state())
    fd = (outs[0] - outs[1]) / (2 * h)
    for f in range(5):
        w = smooth_direction(cfg, x0, rng)[f] / np.abs(dxn[f]).max()
        a, b = float(np.sum(w * dxn[f])), float(np.sum(w * fd[f]))
        assert abs(a - b) <= 1e-5 * np.sum(np.abs(w * dxn[f])), (f, a, b)


def core_mass_fd(cfg, xi, amp, dts, d_amp=None, d_st=None, h=1e-4):
    Js = []
    for sg in (1.0, -1.0):
        c2 = cfg if d_st is None else cfg.with_(stokes=tuple(s + sg * h * d for s, d in zip(cfg.stokes, d_st)))
        a2 = amp if d_amp is None else amp + sg * h * d_amp
        o2 = oracle.Oracle(c2, noise=xi, amp=a2)
        assert o2.step(len(dts), dt_list=dts)[0] == 0
        Js.append(o2.core_dust_mass())
    return (Js[0] - Js[1]) / (2 * h)


def test_tangent_vortex_amplitude_matches_fd():
    cfg = DUST
    xi = synth.noise(cfg)
    amp = synth.amplitude_field(cfg)
    o = oracle.Oracle(cfg, noise=xi, amp=amp)
    st, dts = o.step(4)
    assert st == 0
    d = synth.random_direction(cfg, seed=3) * cfg.vortex_amp
    d = 0.5 * (d + d[::-1])  # mirror-symmetric about the midplane
    status, J, dJ = oracle.tangent(cfg, xi, amp, d, None, dts)
    assert status == 0
    assert J == pytest.approx(o.core_dust_mass(), rel=1e-14)
    assert dJ == pytest.approx(core_mass_fd(cfg, xi, amp, dts, d_amp=d, h=1e-3), rel=1e-6)


def test_tangent_stokes_matches_fd():
    cfg = DUST
    xi = synth.noise(cfg)
    amp = synth.amplitude_field(cfg)
    o = oracle.Oracle(cfg, noise=xi, amp=amp)
    st, dts = o.step(4)
    assert st == 0
    status, J, dJ = oracle.tangent(cfg, xi, amp, None, [1.0], dts)
    assert status == 0
    assert dJ != 0.0
    assert dJ == pytest.approx(core_mass_fd(cfg, xi, amp, dts, d_st=[1.0], h=1e-5), rel=1e-6)
