"""Pins of the oracle's exact drag integration (Sect. 2.9 forces, integrated over steps
longer than the stopping times): one species against the closed form of the relative
velocity decay exp(-(1 + eps) tau / t_s); three species against an independent stiff ODE
integration of the same force law; the long-time limit (every velocity reaches the centre
of mass velocity); species without dust left alone; the split step structure (half-step
relaxation, RK2 stages without drag, half-step relaxation); steps far above the stopping
time accepted and stable; second order in dt where the drag is not stiff."""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from paper_2207_04252_amd import synth

GAMMA = 1.4


def _cell(n_dust, rho=1.0, p=0.7, u=(0.1, 1.0, -0.2), dust=()):
    q = np.zeros(5 + 4 * n_dust)
    q[4] = rho
    q[0:3] = rho * np.array(u)
    q[3] = p / (GAMMA - 1.0) + 0.5 * rho * np.dot(u, u)
    for s, (rd, ud) in enumerate(dust):
        o = 5 + 4 * s
        q[o + 3] = rd
        q[o:o + 3] = rd * np.array(ud)
    return q


def _pressure(q):
    return (GAMMA - 1.0) * (q[3] - 0.5 * np.dot(q[0:3], q[0:3]) / q[4])


@pytest.mark.parametrize("ratio", [0.01, 1.0, 10.0, 1000.0])
def test_single_species_closed_form(oracle_mod, ratio):
    cfg = synth.C3_BIFLUID.scaled(8, 8, 4)
    r, rd = 1.3, 0.3
    q = _cell(1, dust=[(rd, (-0.4, 0.5, 0.3))])
    ts = cfg.stokes[0] / math.sqrt(cfg.GM / r ** 3)
    out = oracle_mod.drag_relax(cfg, r, q, ratio * ts)
    dv0 = q[5:8] / rd - q[0:3] / q[4]
    dv1 = out[5:8] / rd - out[0:3] / out[4]
    assert np.allclose(dv1, dv0 * math.exp(-(1.0 + rd) * ratio), rtol=1e-12, atol=1e-15)
    assert np.allclose(out[0:3] + out[5:8], q[0:3] + q[5:8], rtol=0, atol=1e-14)
    assert _pressure(out) == pytest.approx(_pressure(q), rel=1e-14)
    assert out[4] == q[4] and out[8] == q[8]


def test_three_species_against_ode_integration(oracle_mod):
    cfg = synth.C3_BIFLUID.scaled(8, 8, 4).with_(stokes=(0.01, 0.1, 1.0), eps_dust=(0.01,) * 3,
                                                 hd_over_h=(0.3,) * 3)
    r = 0.9
    omk = math.sqrt(cfg.GM / r ** 3)
    ts = np.array(cfg.stokes) / omk
    dust = [(0.02, (0.3, 0.9, 0.1)), (0.5, (-0.2, 1.2, 0.0)), (0.07, (0.05, 0.7, -0.3))]
    q = _cell(3, dust=dust)
    rho = q[4]
    rd = np.array([d[0] for d in dust])
    tau = 0.2
    u0 = np.concatenate([q[0:3] / rho] + [np.array(d[1]) for d in dust])

    def rhs(_, y):
        ug = y[0:3]
        dy = np.zeros_like(y)
        for s in range(3):
            us = y[3 + 3 * s:6 + 3 * s]
            f = (us - ug) / ts[s]
            dy[3 + 3 * s:6 + 3 * s] = -f
            dy[0:3] += rd[s] / rho * f
        return dy

    sol = solve_ivp(rhs, (0.0, tau), u0, method="Radau", rtol=1e-12, atol=1e-14)
    want = sol.y[:, -1]
    out = oracle_mod.drag_relax(cfg, r, q, tau)
    got = np.concatenate([out[0:3] / rho] + [out[5 + 4 * s:8 + 4 * s] / rd[s] for s in range(3)])
    assert np.allclose(got, want, rtol=1e-9, atol=1e-11)
    mom = lambda x: x[0:3] + sum(x[5 + 4 * s:8 + 4 * s] for s in range(3))
    assert np.allclose(mom(out), mom(q), rtol=0, atol=1e-14)
    assert _pressure(out) == pytest.approx(_pressure(q), rel=1e-13)


def test_long_time_limit_and_empty_species(oracle_mod):
    cfg = synth.C3_BIFLUID.scaled(8, 8, 4).with_(stokes=(0.05, 0.5), eps_dust=(0.01,) * 2,
                                                 hd_over_h=(0.3,) * 2)
    dust = [(0.2, (0.3, 0.9, 0.1)), (0.0, (0.0, 0.0, 0.0))]
    q = _cell(2, dust=dust)
    out = oracle_mod.drag_relax(cfg, 1.0, q, 1e4)
    ucm = (q[0:3] + q[5:8]) / (q[4] + q[8])
    assert np.allclose(out[0:3] / out[4], ucm, rtol=0, atol=1e-13)
    assert np.allclose(out[5:8] / out[8], ucm, rtol=0, atol=1e-13)
    assert np.all(out[9:13] == 0.0)   # the empty species: no momentum, no force
    assert _pressure(out) == pytest.approx(_pressure(q), rel=1e-13)


def _stiff_cfg(exact=True):
    return synth.C3_BIFLUID.scaled(12, 16, 6).with_(stokes=(0.002,), drag_exact=exact)


def test_split_step_structure(oracle_mod):
    """One step = exact relaxation over dt/2, the RK2 stages of the operator without drag,
    exact relaxation over dt/2 (Strang splitting), to roundoff."""
    cfg = _stiff_cfg()
    o = oracle_mod.Oracle(cfg, noise=synth.noise(cfg))
    geo = o.geometry()
    E0 = o.state()
    dt = o.cfl_dt()

    def relax(E, tau):
        out = E.copy()
        for k in range(cfg.nz):
            for i in range(cfg.nr):
                for j in range(cfg.nth):
                    out[:, k, i, j] = oracle_mod.drag_relax(cfg, geo["rc"][i], E[:, k, i, j], tau)
        return out

    V = geo["V"][None, None, :, None]
    E1 = relax(E0, 0.5 * dt)
    o.set_state(E1)
    Es = E1 + 0.5 * dt / V * o.eval_G()
    o.set_state(Es)
    E2 = E1 + dt / V * o.eval_G()
    expect = relax(E2, 0.5 * dt)
    o.set_state(E0)
    st, _ = o.step(1, dt=dt)
    assert st == 0
    assert np.allclose(o.state(), expect, rtol=1e-13, atol=1e-300)


def test_steps_above_the_stopping_time(oracle_mod):
    """St = 0.002: the CFL step is about ten stopping times at the inner edge.  The explicit
    stages refuse it; the split integration takes 20 steps, and the dust moves with the
    gas up to the small terminal drift (in the dust layer: far above it the dust densities
    are at roundoff and their velocities undefined)."""
    cfg = _stiff_cfg()
    o = oracle_mod.Oracle(cfg, noise=synth.noise(cfg))
    dt = o.cfl_dt()
    assert dt > 5 * o.min_stopping_time()
    st, _ = o.step(20)
    assert st == 0
    s = o.state()
    assert np.all(np.isfinite(s))
    full = s[8] > 1e-10 * s[8].max()   # the dust layer (its velocity is defined)
    vg = s[1][full] / s[4][full]
    vd = s[6][full] / s[8][full]
    assert np.max(np.abs(vd - vg)) < 1e-3 * np.max(np.abs(vg))
    e = oracle_mod.Oracle(_stiff_cfg(exact=False), noise=synth.noise(cfg))
    assert e.step(1)[0] == oracle_mod.ESTIFF


def test_split_step_second_order(oracle_mod):
    cfg = synth.C3_BIFLUID.scaled(12, 16, 6).with_(stokes=(0.05,), drag_exact=True,
                                                   vortex_amp=2e-2, noise_amp=0.0)
    dt0 = oracle_mod.Oracle(cfg).cfl_dt()
    T = 4
    o = oracle_mod.Oracle(cfg)
    o.step(T * 64, dt=dt0 / 64)
    ref = o.state()
    errs = []
    for m in (1, 2, 4):
        o = oracle_mod.Oracle(cfg)
        assert o.step(T * m, dt=dt0 / m)[0] == 0
        errs.append(np.abs(o.state() - ref)[[1, 6]].sum(axis=(1, 2, 3)))
    errs = np.array(errs)
    assert np.all(errs[:-1] / errs[1:] > 2.6), errs
