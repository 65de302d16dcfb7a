"""Pins of the oracle's diagnostics counters: the Newton-iteration histogram counts every
gas face once per evaluation of the operator, and a face between identical states needs
exactly one iteration (the primitive-variable guess is then the exact star pressure,
Sect. 2.6); the negative-dust count after a step is the number of negative dust
densities of the new state."""
import numpy as np

import oracle
from paper_2207_04252_amd import synth


def test_histogram_uniform_state():
    cfg = synth.C1_SOD.with_(nr=24, nth=8, sod_left=(1.0, 1.0, 0.0), sod_right=(1.0, 1.0, 0.0))
    o = oracle.Oracle(cfg)
    h0 = np.array(o.diag().newton_hist)
    o.step(3)
    h = np.array(o.diag().newton_hist) - h0
    faces = (cfg.nr + 1) * cfg.nth + cfg.nr * cfg.nth
    assert h[1] == 3 * 2 * faces and h.sum() == h[1]


def test_histogram_counts_every_face_of_a_3d_disc():
    cfg = synth.C3_BIFLUID.scaled(8, 16, 6)
    o = oracle.Oracle(cfg, noise=synth.noise(cfg))
    h0 = np.array(o.diag().newton_hist)
    o.step(2)
    h = np.array(o.diag().newton_hist) - h0
    nr, nth, nz = cfg.nr, cfg.nth, cfg.nz
    faces = (nr + 1) * nth * nz + nr * nth * nz + nr * nth * (nz + 1)
    assert h.sum() == 2 * 2 * faces
    assert h[0] == 0  # no vacuum


def test_negative_dust_count_is_the_new_state_count():
    cfg = synth.C3_BIFLUID.scaled(16, 32, 8).with_(noise_amp=0.0)
    o = oracle.Oracle(cfg)
    s = o.state()
    dt = o.cfl_dt()
    rd = s[8].copy()
    s[5, 1, 8:, 5] = rd[1, 8:, 5] * 12.0
    s[5, 1, :8, 5] = -rd[1, :8, 5] * 12.0
    o.set_state(s)
    assert o.diag().negative_dust == 0
    o.step(1, dt=dt)
    n1 = int((o.state()[8] < 0).sum())
    assert o.diag().negative_dust == n1 >= 1
    o.step(1, dt=dt)
    assert o.diag().negative_dust == n1 + int((o.state()[8] < 0).sum())
