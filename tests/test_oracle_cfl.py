"""Pins of the oracle's CFL time step (Sect. 2.5: N_CFL V / ((|V| + c_s) max |dA|) per cell,
global minimum), through invariances the definition implies rather than the formula
itself: which face area binds (the z face of flat cells makes the step proportional to the
cell height, the radial face of tall cells makes it independent of it, 2D cells have no
z face), the adiabatic sound speed (fixed c when p and rho scale together, c doubling when p
quadruples), and the dust speed (a fast dust cell halves the step when its speed doubles,
an empty dust cell's momentum does not count)."""
import numpy as np
import pytest

from paper_2207_04252_amd import synth


def _uniform_annulus(nz, z_half, rho=1.0, p=1.0, u=0.3):
    return synth.C1_SOD.with_(nr=16, nth=8, nz=nz, z_half=z_half, sod_left=(rho, p, u),
                              sod_right=(rho, p, u))


def test_binding_face_area(oracle_mod):
    # flat cells: the z face is the largest, dt = N V / (s A_z) = N dz / s, so halving the
    # height halves the step
    a = oracle_mod.Oracle(_uniform_annulus(4, 0.05)).cfl_dt()
    b = oracle_mod.Oracle(_uniform_annulus(4, 0.025)).cfl_dt()
    assert b == pytest.approx(0.5 * a, rel=1e-14)
    # tall cells: the outer radial face binds, V / A_r does not depend on the height
    c = oracle_mod.Oracle(_uniform_annulus(4, 2.0)).cfl_dt()
    d = oracle_mod.Oracle(_uniform_annulus(4, 4.0)).cfl_dt()
    assert d == pytest.approx(c, rel=1e-14) and c > 2 * a
    # 2D: no z faces and a nominal unit height, whatever z_half says
    e = oracle_mod.Oracle(_uniform_annulus(1, 0.05)).cfl_dt()
    f = oracle_mod.Oracle(_uniform_annulus(1, 3.0)).cfl_dt()
    assert e == f


def test_adiabatic_sound_speed(oracle_mod):
    at_rest = dict(u=0.0)
    a = oracle_mod.Oracle(_uniform_annulus(4, 0.5, rho=1.0, p=1.0, **at_rest)).cfl_dt()
    b = oracle_mod.Oracle(_uniform_annulus(4, 0.5, rho=2.0, p=2.0, **at_rest)).cfl_dt()
    c = oracle_mod.Oracle(_uniform_annulus(4, 0.5, rho=1.0, p=4.0, **at_rest)).cfl_dt()
    assert b == pytest.approx(a, rel=1e-14)
    assert c == pytest.approx(0.5 * a, rel=1e-14)
    # gamma enters through c = sqrt(gamma p / rho)
    d = oracle_mod.Oracle(_uniform_annulus(4, 0.5, **at_rest).with_(gamma=5.0 / 3.0)).cfl_dt()
    assert d == pytest.approx(a * np.sqrt(1.4 / (5.0 / 3.0)), rel=1e-14)


def test_dust_speed_term(oracle_mod):
    cfg = synth.C3_BIFLUID.scaled(12, 16, 8).with_(noise_amp=0.0)
    o = oracle_mod.Oracle(cfg)
    s0 = o.state()
    dt0 = o.cfl_dt()
    k, i, j = 3, 5, 7
    for fac in (1.0, 2.0):
        s = s0.copy()
        rd = s[8, k, i, j]
        s[5:8, k, i, j] = fac * 400.0 * rd * np.array([1.0, 1.0, 1.0])   # |v_d| ~ 700 c_s
        o.set_state(s)
        if fac == 1.0:
            dt1 = o.cfl_dt()
            assert dt1 < 0.05 * dt0
        else:
            assert o.cfl_dt() == pytest.approx(0.5 * dt1, rel=1e-14)
    # the same momenta in a cell without dust do not count
    s = s0.copy()
    s[8, k, i, j] = 0.0
    s[5:8, k, i, j] = 400.0
    o.set_state(s)
    assert o.cfl_dt() == pytest.approx(dt0, rel=1e-14)
