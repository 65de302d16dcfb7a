"""Pins of the oracle's reading of the reconstruction (Sect. 2.7) at the disc's Mach
numbers.

The parabola and its MinMod limiter act on the primitive variables of the gas (velocity,
pressure and density, as deviations from the stationary flow) and of each dust fluid.
At Mach 14-20 the pressure is about 1% of the total energy, so a limiter that clips the
increments of rho u, E and rho one by one turns every clipped increment into a face
pressure error of order Mach^2 times the clip.  The pins below fail under that reading
(each was run against it): a small acoustic pulse must stay bounded, the operator of a
disc with a smooth density bump must converge with resolution, and two runs whose
inputs differ at rounding level must stay together.  The vacuum and Sod pins of the
other files still hold under the primitive reading.
"""
import numpy as np
import pytest

import oracle
from paper_2207_04252_amd import synth
from tests.parity import cell_errors


def _gas_primitives(s, gamma):
    rho = s[4]
    u, v, w = s[0] / rho, s[1] / rho, s[2] / rho
    p = (gamma - 1.0) * (s[3] - 0.5 * rho * (u * u + v * v + w * w))
    return rho, u, v, w, p


def test_mach20_pulse_stays_bounded(oracle_mod):
    """A 1e-3 isentropic-free (density and pressure at fixed temperature) pulse at r = 1.45
    of the 2D disc (H/r = 0.05: Mach ~20) travels and disperses; its largest relative density
    deviation must stay below the initial amplitude up to t = 12 (about two orbits at the
    pulse).  Limiting the conservative variables one by one grows a two-cell mode here from
    t ~ 8 to tens of percent."""
    cfg = synth.C2_DISC.with_(nr=128, nth=4, nz=1, vortex_amp=0.0, noise_amp=0.0,
                              name="pulse_2d_128")
    o = oracle_mod.Oracle(cfg)
    s0 = o.state()
    rc = o.geometry()["rc"]
    bump = 1.0 + 1e-3 * np.exp(-(rc - 1.45) ** 2 / (2 * 0.02 ** 2))
    rho, u, v, w, p = _gas_primitives(s0, cfg.gamma)
    rho2, p2 = rho * bump[None, :, None], p * bump[None, :, None]
    s = s0.copy()
    s[4] = rho2
    s[0] = 0.0
    s[1] = rho2 * v
    s[2] = 0.0
    s[3] = p2 / (cfg.gamma - 1.0) + 0.5 * rho2 * v * v
    o.set_state(s)
    t, worst = 0.0, 0.0
    while t < 12.0:
        st, dts = o.step(50)
        assert st == 0
        t += float(dts.sum())
        worst = max(worst, float(np.max(np.abs(o.state()[4] / s0[4] - 1.0))))
    assert worst < 1e-3, worst


def _bump_residual(oracle_mod, nr):
    cfg = synth.C6_RWI.with_(nr=nr, nth=4, nz=1, rwi_eps=0.0, noise_amp=0.0, name=f"bump_{nr}")
    o = oracle_mod.Oracle(cfg)
    G, s, g = o.eval_G(), o.state(), o.geometry()
    V = g["V"][None, :, None]
    om = g["rc"][None, :, None] ** -1.5
    return max(float(np.max(np.abs(G[4]) / (V * s[4] * om))),
               float(np.max(np.abs(G[3]) / (V * s[3] * om))))


def test_bumped_disc_operator_converges(oracle_mod):
    """The stationary flow with the Rossby-wave density bump (Sect. 4.3 seed, no m-mode) is
    an exact equilibrium of the continuous equations; the discrete operator's relative
    rates of mass and energy change (per orbital frequency) must fall as the radial mesh is
    refined.  Under per-variable conservative limiting they were 8e-2, 3e-1, 2e-1."""
    res = [_bump_residual(oracle_mod, nr) for nr in (128, 256, 512)]
    assert res[1] < res[0] and res[2] < 0.5 * res[0], res
    assert res[0] < 1e-2, res


def test_rounding_perturbation_stays_small(oracle_mod):
    """Two 100-step runs of a vortex-disc slice whose inputs differ by 1e-13 relative stay
    within 1e-11 per cell (gas fields and pressure): the discrete dynamics does not amplify
    rounding (per-variable conservative limiting gave 1.6e-3 on the slice of the
    parity tests)."""
    cfg = synth.C2_DISC.scaled(24, 48, 32, name="disc_24x48x32")
    xi = synth.noise(cfg)
    o = oracle_mod.Oracle(cfg, noise=xi)
    o2 = oracle_mod.Oracle(cfg)
    o2.set_state(o.state() * (1.0 + 1e-13 * synth.random_direction(cfg, seed=3)[None]))
    st, dts = o.step(100)
    assert st == 0
    assert o2.step(100, dt_list=dts)[0] == 0
    e = cell_errors(o2.state(), o.state(), cfg.gamma)
    assert float(e.max()) < 1e-11, float(e.max())


def test_equilibrium_face_states_exact(oracle_mod):
    """The reconstructed variables of the stationary flow are exactly zero, so its face
    states are the closed-form face values and its operator is the empty-run residual
    bit for bit (Sect. 2.7, 2.8): G - R0 of the unperturbed disc is exactly zero in every
    field, dust included (the dust layer is reconstructed whole, so only the gas)."""
    cfg = synth.C2_DISC.scaled(12, 16, 8).with_(vortex_amp=0.0, noise_amp=0.0)
    o = oracle_mod.Oracle(cfg)
    G = o.eval_G()
    assert np.all(G == 0.0)
