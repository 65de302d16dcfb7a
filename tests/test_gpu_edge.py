"""Edge cases through the C ABI: the smallest grids the library accepts (one partial tile
in every direction), a zero-step call, a single radial ring of tiles with a ragged theta
count, and the first and last z planes of a chunked column; each against the oracle."""
import sys

import numpy as np
import pytest

import oracle
from paper_2207_04252_amd import synth
from tests.parity import field_errors, worst

pytestmark = pytest.mark.gpu


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


CASES = [
    ("min_2d_disc", synth.C2_DISC.scaled(3, 4, 1)),
    ("min_3d_disc", synth.C2_DISC.scaled(3, 4, 4)),
    ("min_3d_bifluid", synth.C3_BIFLUID.scaled(3, 4, 4)),
    ("ragged_theta_67", synth.C2_DISC.scaled(9, 67, 5)),
    ("min_sod", synth.C1_SOD.scaled(3, 4, 1)),
]


@pytest.mark.parametrize("name,cfg", CASES, ids=[c[0] for c in CASES])
def test_small_grid_steps(rb, name, cfg):
    """The step map on the smallest and most ragged grids: the GPU's first CFL step from
    the initial state, and one step from the oracle's states at steps 5 and 9, every cell
    against the oracle (vortex discs amplify rounding differences over free-running steps,
    so later states come from the oracle)."""
    say(f"[edge] {name}")
    xi = synth.noise(cfg)
    sim = rb.Sim(cfg, noise=xi)
    o = oracle.Oracle(cfg, noise=xi)
    done = 0
    for c in (0, 5, 9):
        if c > done:
            assert o.step(c - done)[0] == 0
            done = c
        if c:
            sim.set_fields(o.state())
        dt = o.cfl_dt()
        st, dts = sim.step(1)
        assert st == rb.RB_OK, sim.error()
        assert abs(dts[0] / dt - 1) < 1e-12
        assert o.step(1, dt=dts[0])[0] == 0
        done += 1
        errs = field_errors(sim.fields(), o.state(), cfg.gamma, cfg.n_dust)
        say(f"[edge] {name} step {c}: worst {worst(errs)}")
        for k, v in errs.items():
            assert v <= 1e-10, (c, k, v)
    sim.close()
    o.close()


def test_zero_steps(rb):
    """n = 0 advances nothing, changes no field and returns status OK."""
    cfg = synth.C3_BIFLUID.scaled(12, 64, 8)
    sim = rb.Sim(cfg, noise=synth.noise(cfg))
    s0 = sim.fields()
    st, dts = sim.step(0)
    assert st == rb.RB_OK and len(dts) == 0
    d = sim.diagnostics()
    assert d.step == 0 and d.t == 0.0
    assert np.array_equal(sim.fields(), s0)
    sim.close()


@pytest.mark.parametrize("tk", [1, 3, 7])
def test_z_chunk_boundaries(rb, tk, monkeypatch):
    """Chunked z march with chunk lengths that do not divide nz: the column set-up of each
    chunk (ring, lower z face) and the last partial chunk give the same state as the
    oracle."""
    monkeypatch.setenv("RB_TK", str(tk))
    cfg = synth.C3_BIFLUID.scaled(12, 64, 10)
    say(f"[edge] z chunks of {tk}")
    xi = synth.noise(cfg)
    sim = rb.Sim(cfg, noise=xi)
    o = oracle.Oracle(cfg, noise=xi)
    st, dts = sim.step(3)
    assert st == rb.RB_OK, sim.error()
    assert o.step(3, dt_list=dts)[0] == 0
    errs = field_errors(sim.fields(), o.state(), cfg.gamma, cfg.n_dust)
    say(f"[edge] z chunks of {tk}: worst {worst(errs)}")
    for k, v in errs.items():
        assert v <= 1e-10, (k, v)
    sim.close()
    o.close()
