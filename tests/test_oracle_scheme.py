"""Pins of the oracle's scheme: reconstruction, equilibrium, balance, conservation,
geometry, time order, Sod early-time solution, failure codes.

Each pin is a closed form, an invariant or a brute-force check that a plausible
mistake (dropped term, wrong sign or index, transposed operand) would fail.
"""
import math

import numpy as np
import pytest

from paper_2207_04252_amd import synth

# ------------------------------------ reconstruction ------------------------------------


def test_parabola_exact_on_quadratics(oracle_mod):
    """Monotone quadratic data on a non-uniform grid: the increment to each face equals
    the quadratic's own increment (limiter inactive)."""
    rng = np.random.default_rng(1)
    for _ in range(200):
        xm, x0, xp = np.sort(rng.uniform(0, 1, 3))
        if min(x0 - xm, xp - x0) < 0.05:
            continue
        fl, fr = 0.5 * (xm + x0), 0.5 * (x0 + xp)
        a, b, c = rng.normal(), rng.uniform(1, 2), rng.normal() * 0.1
        q = lambda x: a + b * x + c * x * x
        for xf in (fl, fr):
            inc = oracle_mod.parabola_increment(q(xm), q(x0), q(xp), xm, x0, xp, xf)
            # limiter bounds: 2 d dE'(i), 2 d dE'(i+1)
            d = xf - x0
            Dm = (q(x0) - q(xm)) / (x0 - xm)
            Dp = (q(xp) - q(x0)) / (xp - x0)
            exact = q(xf) - q(x0)
            if abs(exact) <= min(abs(2 * d * Dm), abs(2 * d * Dp)):
                assert abs(inc - exact) < 1e-13 * (abs(exact) + 1), (inc, exact)


def test_uniform_weights_and_inactive_range(oracle_mod):
    """Uniform grid: unlimited face value (-E'_{i-1} + 6E'_i + 3E'_{i+1})/8, and the limiter
    is inactive iff dm/dp lies in [3/7, 7/3]."""
    for ratio in (0.43, 0.5, 1.0, 2.0, 2.33):
        em, e0 = 0.0, 1.0
        ep = e0 + (e0 - em) / ratio
        incp = oracle_mod.parabola_increment(em, e0, ep, -1, 0, 1, 0.5)
        incm = oracle_mod.parabola_increment(em, e0, ep, -1, 0, 1, -0.5)
        assert abs((e0 + incp) - (-em + 6 * e0 + 3 * ep) / 8) < 1e-14
        assert abs((e0 + incm) - (3 * em + 6 * e0 - ep) / 8) < 1e-14
    for ratio in (0.3, 0.42, 2.4, 5.0):
        em, e0 = 0.0, 1.0
        ep = e0 + (e0 - em) / ratio
        incp = oracle_mod.parabola_increment(em, e0, ep, -1, 0, 1, 0.5)
        incm = oracle_mod.parabola_increment(em, e0, ep, -1, 0, 1, -0.5)
        unl = ((-em + 6 * e0 + 3 * ep) / 8 - e0, (3 * em + 6 * e0 - ep) / 8 - e0)
        assert abs(incp - unl[0]) > 1e-6 or abs(incm - unl[1]) > 1e-6


def test_limiter_extrema_and_bounds(oracle_mod):
    rng = np.random.default_rng(2)
    for _ in range(500):
        em, e0, ep = rng.normal(size=3)
        incp = oracle_mod.parabola_increment(em, e0, ep, -1, 0, 1, 0.5)
        incm = oracle_mod.parabola_increment(em, e0, ep, -1, 0, 1, -0.5)
        if (e0 - em) * (ep - e0) <= 0:
            assert incp == 0.0 and incm == 0.0
        # face values stay between the neighbouring cell values (uniform grid)
        assert min(e0, ep) - 1e-15 <= e0 + incp <= max(e0, ep) + 1e-15
        assert min(e0, em) - 1e-15 <= e0 + incm <= max(e0, em) + 1e-15


def test_limiter_continuous(oracle_mod):
    rng = np.random.default_rng(4)
    for _ in range(300):
        v = rng.normal(size=3)
        a = oracle_mod.parabola_increment(*v, -1, 0, 1, 0.5)
        dv = rng.normal(size=3) * 1e-9
        b = oracle_mod.parabola_increment(*(v + dv), -1, 0, 1, 0.5)
        assert abs(a - b) <= 2e-9 * (1 + np.abs(dv).sum() / 1e-9)


# -------------------------------------- equilibrium --------------------------------------


def test_equilibrium_balances(oracle_mod):
    """App. A: hydrostatic dP/dz = -rho GM z/s^3 and radial balance
    rho v^2/r = rho GM r/s^3 + dP/dr, checked with finite differences of P."""
    cfg = synth.C2_DISC
    h = 1e-6
    for r, z in [(0.5, 0.1), (1.0, 0.0), (1.0, -0.12), (1.7, 0.05), (2.0, 0.149)]:
        rho, P, v = oracle_mod.equilibrium(cfg, r, z)
        s3 = (r * r + z * z) ** 1.5
        dPdz = (oracle_mod.equilibrium(cfg, r, z + h)[1] - oracle_mod.equilibrium(cfg, r, z - h)[1]) / (2 * h)
        dPdr = (oracle_mod.equilibrium(cfg, r + h, z)[1] - oracle_mod.equilibrium(cfg, r - h, z)[1]) / (2 * h)
        assert abs(dPdz + rho * z / s3) < 1e-7 * rho / r
        assert abs(rho * v * v / r - (rho * r / s3 + dPdr)) < 1e-7 * rho * v * v / r


def test_equilibrium_disc_numbers(oracle_mod):
    """c_iso = 0.05 r^(-1/4); Mach ~20/17/14 at r = 0.5/1/2; rho(0.5, 0.15)/rho_mid = 4.4e-11."""
    cfg = synth.C2_DISC
    for r, mach in [(0.5, 20), (1.0, 17), (2.0, 14)]:
        rho, P, v = oracle_mod.equilibrium(cfg, r, 0.0)
        ciso = math.sqrt(P / rho)
        assert abs(ciso - 0.05 * r ** -0.25) < 1e-15
        assert abs(v / math.sqrt(1.4 * P / rho) - mach) < 0.5
    r0 = oracle_mod.equilibrium(cfg, 0.5, 0.0)[0]
    r1 = oracle_mod.equilibrium(cfg, 0.5, 0.15)[0]
    assert 4.3e-11 < r1 / r0 < 4.5e-11
    assert abs(oracle_mod.equilibrium(cfg, 1.0, 0.0)[0] - 1.0) < 1e-15


# ---------------------------------- geometry / balance -----------------------------------


def test_geometry_closed_forms(oracle_mod):
    cfg = synth.C2_DISC.scaled(16, 8, 4)
    o = oracle_mod.Oracle(cfg)
    g = o.geometry()
    rf = 0.5 * 4.0 ** (np.arange(17) / 16)
    assert np.allclose(g["rf"], rf, rtol=1e-15)
    dth, dz = 2 * math.pi / 8, 0.3 / 4
    assert np.allclose(g["V"], 0.5 * (rf[1:] ** 2 - rf[:-1] ** 2) * dth * dz, rtol=1e-14)
    # r_c = V/(dr dtheta dz): the centre is the mean radius
    assert np.allclose(g["rc"], g["V"] / ((rf[1:] - rf[:-1]) * dth * dz), rtol=1e-14)
    assert np.allclose(g["zc"], -0.15 + (np.arange(4) + 0.5) * dz, rtol=1e-14)
    assert np.array_equal(g["zc"], -g["zc"][::-1])


def test_uniform_state_static(oracle_mod):
    """Cylindrical geometry: a uniform gas at rest without gravity stays at rest
    (the P/r source balances the radial area difference)."""
    cfg = synth.C1_SOD.with_(sod_right=(1.0, 1.0, 0.0), nr=32, nth=8, nz=4, z_half=0.5)
    o = oracle_mod.Oracle(cfg)
    s0 = o.state()
    st, dts = o.step(20)
    assert st == 0
    s = o.state()
    assert np.abs(s - s0).max() < 1e-13


def _unperturbed(cfg):
    return cfg.with_(vortex_amp=0.0, noise_amp=0.0)


def test_balanced_equilibrium_bitwise(oracle_mod):
    """Sect. 2.8: with the empty-run residual subtracted the discrete equilibrium is kept
    exactly; without it the state drifts."""
    cfg = _unperturbed(synth.C2_DISC.scaled(24, 16, 16))
    o = oracle_mod.Oracle(cfg)
    s0 = o.state()
    st, _ = o.step(200)
    assert st == 0
    assert np.array_equal(o.state(), s0)
    ob = oracle_mod.Oracle(cfg.with_(balanced=False))
    st, dts = ob.step(200, dt_list=None)
    drift = np.abs(ob.state()[4] - s0[4]) / s0[4]
    assert drift.max() > 1e-7


def test_residual_structure(oracle_mod):
    """R0 = G(E0) is non-zero only in rho u and rho w, identical along theta."""
    cfg = _unperturbed(synth.C2_DISC.scaled(24, 16, 8))
    o = oracle_mod.Oracle(cfg)
    R = o.residual()
    assert np.all(R[..., 1] == 0) and np.all(R[..., 3] == 0) and np.all(R[..., 4] == 0)
    assert np.abs(R[..., 0]).max() > 0 and np.abs(R[..., 2]).max() > 0
    G = o.eval_G(with_dust=False, subtract_R0=False)
    assert np.array_equal(G[:5], np.repeat(G[:5, ..., :1], cfg.nth, axis=-1))
    assert np.array_equal(G[:5, :, :, 0], np.moveaxis(R, -1, 0))


# ---------------------------------------- conservation -----------------------------------


def test_mass_ledger(oracle_mod):
    """M^{n+1} - M^n = -dt * (boundary outflow of the second-stage fluxes), to 1e-13."""
    cfg = synth.C3_BIFLUID.scaled(24, 32, 16)
    o = oracle_mod.Oracle(cfg, noise=synth.noise(cfg))
    m = o.mass()
    for _ in range(6):
        st, dts = o.step(1)
        assert st == 0
        m1 = o.mass()
        out = np.array(o.diag().outflow)[: 1 + cfg.n_dust]
        assert np.all(np.abs(m1 - m + dts[0] * out) <= 1e-13 * m), (m1 - m + dts[0] * out) / m
        m = m1


def test_drag_operator(oracle_mod):
    """Sect. 2.9: uniform gas and dust at rest except for w (2D, z = 0: no vertical
    gravity, no z faces): the w-components of G are the drag +-rho_d (w_d - w_g)/t_s V
    with t_s = St/Omega_K, and gas + dust momentum is exchanged exactly."""
    cfg = synth.C1_SOD.with_(sod_right=(1.0, 1.0, 0.0), nr=8, nth=4, nz=1, GM=1.0,
                             stokes=(0.3, 0.7), eps_dust=(0.0, 0.0), hd_over_h=(1.0, 1.0))
    o = oracle_mod.Oracle(cfg)
    s = o.state()
    wg, rd, wd = 0.01, (0.02, 0.05), (-0.03, 0.04)
    s[2] = 1.0 * wg
    s[3] += 0.5 * wg * wg
    for q in range(2):
        s[5 + 4 * q + 3] = rd[q]
        s[5 + 4 * q + 2] = rd[q] * wd[q]
    o.set_state(s)
    G = o.eval_G(with_dust=True, subtract_R0=False)
    g = o.geometry()
    for i in range(cfg.nr):
        omk = math.sqrt(1.0 / g["rc"][i] ** 3)
        drag = [rd[q] * (wd[q] - wg) / (cfg.stokes[q] / omk) * g["V"][i] for q in range(2)]
        assert np.allclose(G[2, 0, i, :], sum(drag), rtol=1e-13, atol=0)
        for q in range(2):
            assert np.allclose(G[5 + 4 * q + 2, 0, i, :], -drag[q], rtol=1e-13, atol=0)
        tot = G[2, 0, i, :] + G[7, 0, i, :] + G[11, 0, i, :]
        assert np.all(np.abs(tot) < 1e-16 * abs(drag[0]) * 10)
        assert np.allclose(G[3, 0, i, :], wg * sum(drag), rtol=1e-13)


# ------------------------------------------ Sod ------------------------------------------


def test_sod_annulus_theta_invariant_bitwise(oracle_mod):
    o = oracle_mod.Oracle(synth.C1_SOD)
    st, dts = o.step(100)
    assert st == 0
    s = o.state()
    assert np.array_equal(s, np.repeat(s[..., :1], synth.C1_SOD.nth, axis=-1))
    assert abs(dts[0] - 1.6475e-3) < 1e-6   # 0.5 dr / (|v| + c) of the left state


def _sod_exact(x, t, x0, g=1.4):
    """Planar Sod solution (rho) at time t from the textbook star values."""
    pS, uS, rSL, rSR = 0.30313017805064707, 0.9274526200489498, 0.42631942817849544, 0.26557371170530725
    cL = math.sqrt(g)
    sH, sT, sS = -cL, uS - cL * (pS / 1.0) ** ((g - 1) / (2 * g)), 1.7521557320301779
    xi = (x - x0) / t
    out = np.empty_like(x)
    for n, v in enumerate(xi):
        if v <= sH:
            out[n] = 1.0
        elif v <= sT:
            c = 2 / (g + 1) * (cL - 0.5 * (g - 1) * v)   # left fan, u_L = 0
            out[n] = (c / cL) ** (2 / (g - 1))
        elif v <= uS:
            out[n] = rSL
        elif v <= sS:
            out[n] = rSR
        else:
            out[n] = 0.125
    return out


def test_sod_planar_limit_converges(oracle_mod):
    """Annulus at r ~ 1000 (planar limit): L1 density error against the exact Sod
    solution decreases under refinement."""
    errs = []
    for nr in (50, 100, 200):
        cfg = synth.C1_SOD.with_(r_in=1000.0, r_out=1001.0, sod_r0=1000.5, nr=nr, nth=2,
                                 name=f"planar{nr}")
        o = oracle_mod.Oracle(cfg)
        T = 0.15
        t = 0.0
        while t < T - 1e-14:
            dt = min(o.cfl_dt(), T - t)
            st, _ = o.step(1, dt=dt)
            assert st == 0
            t += dt
        g = o.geometry()
        rho = o.state()[4, 0, :, 0]
        errs.append(np.mean(np.abs(rho - _sod_exact(g["rc"], T, 1000.5))))
    assert errs[0] > errs[1] > errs[2]
    order = math.log(errs[0] / errs[2], 4.0)
    assert order > 0.6, (errs, order)


def test_sod_annulus_early_time_waves(oracle_mod):
    """Config 1 after 100 steps: shock, contact and rarefaction head within a few cells of
    the planar positions; star plateaus within 10% (cylindrical divergence)."""
    cfg = synth.C1_SOD
    o = oracle_mod.Oracle(cfg)
    st, dts = o.step(100)
    t = dts.sum()
    g = o.geometry()
    rc = g["rc"]
    rho = o.state()[4, 0, :, 0]
    dr = rc[1] - rc[0]
    x_shock = 1.5 + 1.7521557 * t
    x_head = 1.5 - math.sqrt(1.4) * t
    # shock: last cell above the midpoint of the post-shock plateau and 0.125
    i_sh = np.max(np.nonzero(rho > 0.5 * (0.2656 + 0.125))[0])
    assert abs(rc[i_sh] - x_shock) < 3 * dr
    i_hd = np.min(np.nonzero(rho < 0.995)[0])
    assert abs(rc[i_hd] - x_head) < 3 * dr
    plateau = rho[(rc > 1.5 + 0.3 * 0.9275 * t) & (rc < 1.5 + 0.7 * 0.9275 * t)]
    assert np.all(np.abs(plateau / 0.42632 - 1) < 0.1)


def test_sod_first_stage_closed_form(oracle_mod):
    """First stage at the two diaphragm cells: the limiter is flat at the jump, so the
    faces carry the physical flux of each uniform side and the Godunov flux at the
    diaphragm; E* = E + (dt/2V)(G) with the P/r source (worked example)."""
    cfg = synth.C1_SOD
    o = oracle_mod.Oracle(cfg)
    g = o.geometry()
    dt = o.cfl_dt()
    G = o.eval_G(with_dust=False, subtract_R0=False)
    i_d = int(np.argmin(np.abs(g["rf"] - 1.5)))   # face at r = 1.5
    FG = (0.3953910704, 0.6698366622, 1.1540375169)  # mass, momentum, energy at x/t = 0
    for i, (rho, p) in ((i_d - 1, (1.0, 1.0)), (i_d, (0.125, 0.1))):
        Ap, Am, V, r = g["Ar"][i + 1], g["Ar"][i], g["V"][i], g["rc"][i]
        up = FG if i == i_d - 1 else (0.0, p, 0.0)
        um = (0.0, p, 0.0) if i == i_d - 1 else FG
        Gm = -(Ap * up[0] - Am * um[0])
        Gmom = -(Ap * up[1] - Am * um[1]) + p / r * V
        Ge = -(Ap * up[2] - Am * um[2])
        assert abs(G[4, 0, i, 0] - Gm) < 1e-8 * Ap
        assert abs(G[0, 0, i, 0] - Gmom) < 1e-8 * Ap
        assert abs(G[3, 0, i, 0] - Ge) < 1e-8 * Ap
    assert dt > 0


# ----------------------------------------- time order ------------------------------------


def test_rk2_structure_exact(oracle_mod):
    """Sect. 2.5 with a = 0, b = 1, alpha = beta = 1/2, read with V dE/dt = G:
    E^{n+1} = E^n + (dt/V) G(E^n + (dt/2V) G(E^n)), to roundoff."""
    cfg = synth.C3_BIFLUID.scaled(16, 16, 8).with_(vortex_amp=2e-2)
    o = oracle_mod.Oracle(cfg, noise=synth.noise(cfg))
    V = o.geometry()["V"][None, None, :, None]
    E0 = o.state()
    dt = 0.8 * o.cfl_dt()
    G0 = o.eval_G()
    Es = E0 + 0.5 * dt / V * G0
    o.set_state(Es)
    G1 = o.eval_G()
    expect = E0 + dt / V * G1
    o.set_state(E0)
    st, _ = o.step(1, dt=dt)
    assert st == 0
    got = o.state()
    assert np.allclose(got, expect, rtol=1e-14, atol=0)


def test_rk2_converges_second_order(oracle_mod):
    """Error against a fine-dt reference falls faster than first order (limiter kinks
    keep the measured order a little below 2)."""
    cfg = synth.C2_DISC.scaled(16, 32, 8).with_(vortex_amp=2e-2, noise_amp=0.0)
    dt0 = oracle_mod.Oracle(cfg).cfl_dt()
    T = 4
    o = oracle_mod.Oracle(cfg)
    o.step(T * 64, dt=dt0 / 64)
    ref = o.state()
    errs = []
    for m in (1, 2, 4, 8):
        o = oracle_mod.Oracle(cfg)
        st, _ = o.step(T * m, dt=dt0 / m)
        assert st == 0
        errs.append(np.abs(o.state() - ref)[:5].sum(axis=(1, 2, 3)))
    errs = np.array(errs)
    assert np.all(errs[0] / errs[3] > 25.0), errs[0] / errs[3]
    assert np.all(errs[:-1] / errs[1:] > 2.6)


# ---------------------------------------- failure codes ----------------------------------


def test_negative_pressure_detected(oracle_mod):
    cfg = synth.C2_DISC.scaled(12, 8, 8)
    o = oracle_mod.Oracle(cfg)
    s = o.state()
    k, i, j = 3, 5, 2
    s[3, k, i, j] = 0.5 * (s[0, k, i, j] ** 2 + s[1, k, i, j] ** 2) / s[4, k, i, j] * 0.2
    o.set_state(s)
    st, _ = o.step(2)
    assert st == oracle_mod.ENEGATIVE
    d = o.diag()
    assert d.first_bad_step == 0 and d.first_bad_cell >= 0


def test_stiff_drag_detected(oracle_mod):
    cfg = synth.C3_BIFLUID.scaled(12, 8, 8).with_(stokes=(1e-4,))
    o = oracle_mod.Oracle(cfg)
    st, _ = o.step(1)
    assert st == oracle_mod.ESTIFF


def test_vacuum_flagged(oracle_mod):
    cfg = synth.C1_SOD.with_(nr=16, nth=4, sod_left=(1.0, 0.01, -5.0), sod_right=(1.0, 0.01, 5.0),
                             sod_r0=1.5)
    o = oracle_mod.Oracle(cfg)
    st, _ = o.step(1, dt=1e-5)
    assert st == oracle_mod.EVACUUM
    assert o.diag().vacuum_faces > 0


def test_newton_cap_detected(oracle_mod):
    """A Newton iteration cap of one stops the Sod annulus at its first step with the
    no-convergence error (the diaphragm problem needs several iterations); the default
    cap of 50 converges."""
    cfg = synth.C1_SOD.with_(nr=32, nth=4, newton_max_iter=1)
    o = oracle_mod.Oracle(cfg)
    st, _ = o.step(2)
    assert st == oracle_mod.ENOCONV and o.diag().step == 0
    assert oracle_mod.Oracle(cfg.with_(newton_max_iter=0)).step(2)[0] == 0
