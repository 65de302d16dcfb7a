"""The exact gas solver's edge branches and the error paths on the GPU, against the
oracle (Sect. 2.6 solver; Sod annulus variants, FP64).

The Sod annulus itself, and variants whose diaphragm problem takes the solver's rarer
branches: both states shifted outwards by 0.75 of the left sound speed, so that x/t = 0 lies inside
the left rarefaction fan (transonic); a pressure ratio of 1e5 (strong shock and strong
rarefaction); colliding and receding streams at u = -+5 (vacuum: reported as RB_EVACUUM
while the run continues).  Every cell against the oracle after 10 steps.  Error paths:
a NaN and a negative density set into the state, and a Newton iteration cap of one
(RB_ENOCONV), each with the step and the first bad cell of the oracle.  Diagnostics: the
Newton-iteration histogram of the variants and the count of negative dust densities of a
forced divergent dust stream, against the oracle's."""
import sys

import numpy as np
import pytest

import oracle
from paper_2207_04252_amd import synth
from tests.parity import field_errors, worst

pytestmark = pytest.mark.gpu

CL = float(np.sqrt(1.4))     # left sound speed of the Sod states (rho = p = 1)
BASE = synth.C1_SOD.with_(nr=96, nth=8)
VARIANTS = [
    ("sod", BASE, None),
    ("transonic", BASE.with_(sod_left=(1.0, 1.0, 0.75 * CL), sod_right=(0.125, 0.1, 0.75 * CL)), None),
    ("strong_shock", BASE.with_(sod_left=(1.0, 1000.0, 0.0), sod_right=(1.0, 0.01, 0.0)), None),
    ("vacuum", BASE.with_(sod_left=(1.0, 0.01, -5.0), sod_right=(1.0, 0.01, 5.0)), 2e-4),
]


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


@pytest.mark.parametrize("name,cfg,dt", VARIANTS, ids=[v[0] for v in VARIANTS])
def test_sod_variant_parity(rb, name, cfg, dt):
    say(f"[riemann edge] {name}")
    n = 10
    sim = rb.Sim(cfg)
    o = oracle.Oracle(cfg)
    if dt is None:
        st, dts = sim.step(n)
        st2, dts2 = o.step(n)
        assert np.allclose(dts, dts2, rtol=1e-12, atol=0)
    else:
        st, dts = sim.step(n, dt=dt)
        st2, dts2 = o.step(n, dt=dt)
    expect = oracle.EVACUUM if name == "vacuum" else 0
    assert st2 == expect and st == expect, (st, st2)
    d1, d2 = sim.diagnostics(), o.diag()
    assert (d1.vacuum_faces > 0) == (d2.vacuum_faces > 0) == (name == "vacuum")
    errs = field_errors(sim.fields(), o.state(), cfg.gamma, 0)
    say(f"[riemann edge] {name}: worst {worst(errs)}, Newton max {d1.max_newton} / {d2.max_newton}")
    for k, v in errs.items():
        assert v <= 1e-10, (k, v)
    check_histogram(d1, d2)
    sim.close()


def check_histogram(d_gpu, d_or):
    """Both sides count every gas face once per evaluation.  The GPU takes supersonic
    faces without a Newton solve (bin 0) where the oracle iterates, so faces may only move
    from the oracle's Newton bins to the GPU's bin 0; where no face took that path the
    histograms agree (up to faces whose last relative change lies within rounding of the
    1e-12 stopping threshold)."""
    hg, ho = np.array(d_gpu.newton_hist), np.array(d_or.newton_hist)
    say(f"[newton histogram] gpu {hg.tolist()} oracle {ho.tolist()}")
    assert hg.sum() == ho.sum() > 0
    moved = hg[0] - ho[0]
    assert moved >= 0
    slack = max(2, int(1e-5 * ho.sum()))
    assert np.abs(hg[1:] - ho[1:]).sum() <= moved + slack
    if moved == 0:
        assert np.abs(hg - ho).max() <= slack


@pytest.mark.parametrize("what", ["nan", "negative_density"])
def test_bad_state_reported(rb, what):
    cfg = synth.C2_DISC.scaled(24, 64, 16)
    say(f"[error path] {what}")
    sim = rb.Sim(cfg, noise=synth.noise(cfg))
    s = sim.fields()
    k, i, j = 5, 7, 33
    s[4, k, i, j] = np.nan if what == "nan" else -1e-3
    sim.set_fields(s)
    st, _ = sim.step(1)
    assert st == rb.RB_ENEGATIVE
    d = sim.diagnostics()
    cell = (k * cfg.nr + i) * cfg.nth + j
    assert d.first_bad_cell == cell and d.step == 0
    o = oracle.Oracle(cfg)
    o.set_state(s)
    assert o.step(1)[0] == oracle.ENEGATIVE
    assert o.diag().first_bad_cell == cell
    sim.close()


def test_newton_cap_reported(rb):
    """With a cap of one Newton iteration every face that needs a second one fails: the
    first step stops with RB_ENOCONV on both sides; the default cap converges."""
    cfg = BASE.with_(newton_max_iter=1)
    say("[error path] newton cap")
    sim = rb.Sim(cfg)
    st, _ = sim.step(3)
    assert st == rb.RB_ENOCONV
    d = sim.diagnostics()
    assert d.first_bad_step == 0 and d.step == 0
    o = oracle.Oracle(cfg)
    assert o.step(3)[0] == oracle.ENOCONV and o.diag().step == 0
    sim.close()
    sim = rb.Sim(BASE)
    assert sim.step(3)[0] == rb.RB_OK
    sim.close()


def test_negative_dust_count(rb):
    """A dust stream split at one radius (inwards below it, outwards above it, at 12 in
    code units) empties cells next to the split faster than their content allows within
    one CFL step, so their dust densities end the step negative: the count and every cell
    match the oracle over two steps."""
    cfg = synth.C3_BIFLUID.scaled(16, 32, 8).with_(noise_amp=0.0)
    say("[diagnostics] negative dust")
    o = oracle.Oracle(cfg)
    s = o.state()
    dt = o.cfl_dt()
    k, i0, j, U = 1, 8, 5, 12.0
    rd = s[8].copy()
    s[5, k, i0:, j] = rd[k, i0:, j] * U
    s[5, k, :i0, j] = -rd[k, :i0, j] * U
    o.set_state(s)
    sim = rb.Sim(cfg)
    sim.set_fields(s)
    for n in (1, 2):
        assert o.step(1, dt=dt)[0] == 0
        assert sim.step(1, dt=dt)[0] == rb.RB_OK
        d1, d2 = sim.diagnostics(), o.diag()
        say(f"[diagnostics] step {n}: negative dust {d1.negative_dust} / {d2.negative_dust}")
        assert d1.negative_dust == d2.negative_dust >= n
        errs = field_errors(sim.fields(), o.state(), cfg.gamma, cfg.n_dust)
        for key, v in errs.items():
            assert v <= 1e-10, (key, v)
    sim.close()
