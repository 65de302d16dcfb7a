"""rb_cfl_dt_static, the allocation-free variant of rb_cfl_dt (static device scratch, no
host synchronisation), through the C ABI against rb_cfl_dt: two calls in a row, the
second on a smaller grid; both must give rb_cfl_dt's step bit for bit (same kernels, same
partition)."""
import ctypes
import sys

import numpy as np
import pytest

from paper_2207_04252_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rb():
    import torch
    assert torch.cuda.is_available(), "GPU test on a machine without a GPU"
    from paper_2207_04252_amd import rossbi
    L = rossbi.load()
    L.rb_cfl_dt_static.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    L.rb_cfl_dt_static.restype = ctypes.c_int
    return rossbi


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def static_dt(rb, sim, state_ptr):
    import torch
    out = torch.full((1,), -1.0, dtype=torch.float64, device=sim.state.device)
    st = sim.lib.rb_cfl_dt_static(sim.ctx, ctypes.c_void_p(state_ptr),
                                  ctypes.c_void_p(out.data_ptr()))
    assert st == rb.RB_OK, sim.error()
    sim.stream.synchronize()
    return float(out.cpu()[0])


@pytest.mark.parametrize("precision", ["fp64", "fp32p"])
def test_static_cfl_matches_cfl_dt(rb, precision):
    prec = rb.RB_FP64 if precision == "fp64" else rb.RB_FP32_PERT
    big = synth.C3_BIFLUID.scaled(96, 200, 48)
    small = synth.C3_BIFLUID.scaled(12, 64, 8)
    for cfg in (big, small):
        say(f"[no-alloc cfl] {cfg.name} {precision}")
        sim = rb.Sim(cfg, precision=prec, noise=synth.noise(cfg))
        sim.step(3)
        want = sim.cfl_dt()
        got = static_dt(rb, sim, sim.state.data_ptr())
        say(f"[no-alloc cfl] rb_cfl_dt {want!r} rb_cfl_dt_static {got!r}")
        assert got == want
        # a state with a non-positive pressure gives 0.0 (and leaves the context alone)
        s = sim.fields()
        s[3, 1, 2, 3] = 0.0
        sim.set_fields(s)
        assert static_dt(rb, sim, sim.state.data_ptr()) == 0.0
        sim.close()


def test_static_cfl_rejects_null(rb):
    cfg = synth.C2_DISC.scaled(12, 64, 8)
    sim = rb.Sim(cfg)
    assert sim.lib.rb_cfl_dt_static(sim.ctx, None, None) == rb.RB_EINVAL
    sim.close()
