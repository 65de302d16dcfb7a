"""Discrete adjoint on the GPU (rb_record / rb_adjoint / rb_amp_gradient) against the
FP64 oracle's forward-mode derivatives and against finite differences.

Dot-product tests: for a final-state cotangent lam and a direction (v, st_dot),
<lam, dE_n> from the oracle's dual-number run equals <dJ/dE_0, v> + <dJ/dSt, st_dot>
from the GPU adjoint of the same recorded steps.  Both differentiate the branches the
primal solves took (limiter, Riemann wave pattern, fallbacks), so they agree to
rounding on any state, kinks included."""
import sys

import numpy as np
import pytest

import oracle
from paper_2207_04252_amd import synth

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


def steps_for(cfg, n):
    """CFL steps of the oracle, capped below half the smallest stopping time."""
    o = oracle.Oracle(cfg, noise=synth.noise(cfg) if cfg.noise_amp else None)
    dts = []
    for _ in range(n):
        dt = o.cfl_dt()
        if cfg.n_dust:
            dt = min(dt, 0.5 * o.min_stopping_time())
        assert o.step(1, dt=dt)[0] == 0
        dts.append(dt)
    return np.array(dts)


def perturbed_state(cfg, seed):
    """The configuration's initial state with a seeded per-cell perturbation of relative
    size 1e-3 (density, internal energy, momenta on the scale rho c_s; dust alike).

    Branch decisions of the scheme (limiter arguments, the sign of a star velocity or of
    a delta-shock speed) taken on rounding-level data -- exactly uniform regions, exactly
    mirror-symmetric columns -- go either way between two FP64 implementations, and so
    does the branch a derivative is frozen on.  The perturbation puts every decision
    well above rounding."""
    xi = synth.noise(cfg) if cfg.noise_amp else None
    x = oracle.Oracle(cfg, noise=xi).state()
    rng = np.random.default_rng(seed)
    g = cfg.gamma
    rho = x[4]
    pres = (g - 1) * (x[3] - 0.5 * (x[0] ** 2 + x[1] ** 2 + x[2] ** 2) / rho)
    cs = np.sqrt(g * pres / rho)
    u = lambda: rng.uniform(-1, 1, size=rho.shape)  # noqa: E731
    for f in range(3):
        x[f] += 1e-3 * rho * cs * u()
    x[4] = rho * (1 + 1e-3 * u())
    x[3] = 0.5 * (x[0] ** 2 + x[1] ** 2 + x[2] ** 2) / x[4] + pres * (1 + 1e-3 * u()) / (g - 1)
    for s in range(cfg.n_dust):
        o = 5 + 4 * s
        for c in range(3):
            x[o + c] += 1e-3 * x[o + 3] * cs * u()
        x[o + 3] *= 1 + 1e-3 * u()
    return x


def steps_from(cfg, x0, n):
    """CFL steps of the oracle from x0, capped below half the smallest stopping time."""
    o = oracle.Oracle(cfg)
    o.set_state(x0)
    dts = []
    for _ in range(n):
        dt = o.cfl_dt()
        if cfg.n_dust:
            dt = min(dt, 0.5 * o.min_stopping_time())
        assert o.step(1, dt=dt)[0] == 0
        dts.append(dt)
    return np.array(dts)


CASES = [
    ("adjoint_disc", synth.C5_ADJOINT.scaled(20, 72, 16), 3, 2),
    ("gas_disc", synth.C2_DISC.scaled(20, 72, 16), 3, 2),
    ("bifluid3", synth.C4_LARGE.scaled(20, 72, 8), 2, 1),
    ("sod_2d", synth.C1_SOD.scaled(40, 16, 1), 3, 3),
    ("sod_3d", synth.C1_SOD.scaled(24, 16, 4), 2, 1),
]


def local_scale(cfg, x):
    """Per-cell scale of every field: rho c_s for the momenta, the internal energy,
    the density; the dust alike with the gas sound speed."""
    g = cfg.gamma
    rho = x[4]
    p = (g - 1) * (x[3] - 0.5 * (x[0] ** 2 + x[1] ** 2 + x[2] ** 2) / rho)
    cs = np.sqrt(g * p / rho)
    sc = np.empty_like(x)
    for f in range(3):
        sc[f] = rho * cs
    sc[3] = p / (g - 1)
    sc[4] = rho
    for s in range(cfg.n_dust):
        o = 5 + 4 * s
        for c in range(3):
            sc[o + c] = x[o + 3] * cs
        sc[o + 3] = x[o + 3]
    return sc


@pytest.mark.parametrize("name,cfg,n,k", CASES, ids=[c[0] for c in CASES])
def test_adjoint_dot_product(rb, name, cfg, n, k):
    """The cotangent and the directions are random on each cell's own scale, on the
    cells holding gas (dust) above 1% of their column's peak: the thin gas at the top
    and bottom of the inner disc, and the dust far above its layer, are ill-conditioned
    (rounding-level changes of the state move their tangents by many orders more).  The tolerance is calibrated on the oracle
    itself: ten times the change of the same dot product when the base state is moved
    by 1e-14 relative, the size of the rounding difference between two FP64
    trajectories after a few steps (and at least 1e-10)."""
    say(f"[adjoint dot] {name} {cfg.name} n={n} ckpt={k}")
    x0 = perturbed_state(cfg, seed=7)
    dts = steps_from(cfg, x0, n)
    sim = rb.Sim(cfg)
    sim.set_fields(x0)
    got = sim.record(n, k, dt_list=dts)
    assert np.array_equal(got, dts)
    rng = np.random.default_rng(2207)
    sc = local_scale(cfg, x0)
    live = np.empty(x0.shape, dtype=bool)
    for o, dens in [(0, 4)] + [(5 + 4 * s, 8 + 4 * s) for s in range(cfg.n_dust)]:
        m = x0[dens] >= 1e-2 * x0[dens].max(axis=0, keepdims=True)
        for f in range(o, o + (5 if o == 0 else 4)):
            live[f] = m
    lam = rng.uniform(-1, 1, size=x0.shape) / sc * live
    g0, gst = sim.adjoint(lam)
    g0 = g0.cpu().numpy()
    sim.close()
    x1 = x0 * (1 + 1e-14 * np.random.default_rng(5).uniform(-1, 1, size=x0.shape))
    groups = [("gas", list(range(5)))] + [
        (f"dust{s}", list(range(5 + 4 * s, 9 + 4 * s))) for s in range(cfg.n_dust)]
    dirs = []
    for gname, fields in groups:
        v = np.zeros_like(x0)
        for f in fields:
            v[f] = rng.uniform(-1, 1, size=x0[f].shape) * sc[f] * live[f]
        dirs.append((gname, v, None))
    for s in range(cfg.n_dust):
        sd = [0.0] * cfg.n_dust
        sd[s] = 1.0
        dirs.append((f"stokes{s}", np.zeros_like(x0), sd))
    bad = {}
    for dname, v, sd in dirs:
        st, _, dxn = oracle.tangent_state(cfg, x0, v, sd, dts)
        assert st == 0
        st, _, dxn1 = oracle.tangent_state(cfg, x1, v, sd, dts)
        assert st == 0
        lhs = float(np.sum(lam * dxn))
        mag = float(np.sum(np.abs(lam * dxn)))
        rhs = float(np.sum(g0 * v)) + (0.0 if sd is None else float(np.dot(gst, sd)))
        err = abs(lhs - rhs) / mag
        tol = max(1e-10, 10.0 * abs(float(np.sum(lam * dxn1)) - lhs) / mag)
        say(f"[adjoint dot] {name} {dname}: oracle {lhs:.15e} gpu {rhs:.15e} rel {err:.2e} "
            f"(tol {tol:.1e})")
        if err > tol:
            bad[dname] = (err, tol)
    assert not bad, bad


def test_adjoint_amplitude_and_stokes_vs_oracle(rb):
    """Gradient of the vortex-core dust mass after n steps with respect to the vortex
    amplitude field and the Stokes number, against the oracle's tangent."""
    cfg = synth.C5_ADJOINT.scaled(20, 72, 16)
    n = 6
    say(f"[adjoint amp] {cfg.name} n={n}")
    xi = synth.noise(cfg)
    amp = synth.amplitude_field(cfg)
    dts = steps_for(cfg, n)
    sim = rb.Sim(cfg, noise=xi, amp=amp)
    sim.record(n, 4, dt_list=dts)
    lam = core_mass_cotangent(rb, cfg)
    g0, gst = sim.adjoint(lam)
    gamp = sim.amp_gradient(g0, noise=xi, amp=amp).cpu().numpy()
    sim.close()
    d = synth.random_direction(cfg, seed=3) * cfg.vortex_amp
    st, J, dJ = oracle.tangent(cfg, xi, amp, d, None, dts)
    assert st == 0
    got = float(np.sum(gamp * d))
    say(f"[adjoint amp] oracle {dJ:.15e} gpu {got:.15e}")
    assert got == pytest.approx(dJ, rel=1e-9)
    st, J, dJs = oracle.tangent(cfg, xi, amp, None, [1.0], dts)
    say(f"[adjoint amp] stokes oracle {dJs:.15e} gpu {gst[0]:.15e}")
    assert gst[0] == pytest.approx(dJs, rel=1e-9)


def core_mass_cotangent(rb, cfg):
    """dJ/dE of J = dust mass in the vortex core (r in the core band, |theta - theta_v|
    below the core half-width): the cell volume on each dust density in the core.  The
    oracle's mesh, checked against the library's (rb_get_geometry)."""
    geo = oracle.Oracle(cfg).geometry()
    V, rc = geo["V"], geo["rc"]
    sim = rb.Sim(cfg)
    g = sim.geometry()
    sim.close()
    assert np.allclose(V, g["V"], rtol=1e-13) and np.allclose(rc, g["rc"], rtol=1e-14)
    assert np.allclose(geo["rf"], g["rf"], rtol=1e-14) and np.allclose(geo["zc"], g["zc"], atol=1e-15)
    th = (np.arange(cfg.nth) + 0.5) * 2 * np.pi / cfg.nth
    mask = ((rc >= synth.CORE_R[0]) & (rc <= synth.CORE_R[1]))[:, None] & \
           (np.abs(th - cfg.vortex_th0) < synth.CORE_DTH)[None, :]
    lam = np.zeros((cfg.n_fields, cfg.nz, cfg.nr, cfg.nth))
    for s in range(cfg.n_dust):
        lam[5 + 4 * s + 3] = (V[:, None] * mask)[None, :, :]
    return lam


def test_autograd_matches_finite_differences(rb):
    """torch.autograd through the disc run (rb_record forward, rb_adjoint backward):
    the gradient of the core dust mass with respect to the vortex amplitude (along the
    uniform direction) and the Stokes number, against central differences of the GPU
    forward run with the same time steps.

    The limited scheme is only piecewise smooth: a perturbation that breaks the vortex's
    mirror symmetry about the mesh face it is centred on lands exactly on limiter kinks,
    and longer runs cross more kinks within any finite step.  Finite differences confirm
    the gradient where the run is smooth at the step size: a uniform amplitude change
    and the Stokes number over a few steps.  An odd number of z layers puts the
    midplane at a cell centre (an even number makes it a face where settling dust meets
    in a standing delta shock whose side is set by rounding-level asymmetry)."""
    import torch
    cfg = synth.C5_ADJOINT.scaled(20, 72, 15)
    n = 5
    say(f"[autograd] {cfg.name} n={n}")
    xi = synth.noise(cfg)
    dts = steps_for(cfg, n)
    lam = torch.as_tensor(core_mass_cotangent(rb, cfg), device="cuda")
    amp = torch.full((cfg.nz, cfg.nr, cfg.nth), cfg.vortex_amp, dtype=torch.float64,
                     device="cuda", requires_grad=True)
    st = torch.tensor(cfg.stokes, dtype=torch.float64, requires_grad=True)
    final = rb.disc_run(amp, st, cfg, n, dts, ckpt_every=2, noise=xi)
    J = (final * lam).sum()
    J.backward()
    got_amp = float(amp.grad.sum()) * cfg.vortex_amp
    got_st = float(st.grad[0])

    def J_of(a, s):
        sim = rb.Sim(cfg.with_(stokes=(s,)), noise=xi, amp=np.full(cfg.n_cells, a))
        sim.step(n, dt_list=dts, check=True)
        out = float(np.sum(sim.fields() * lam.cpu().numpy()))
        sim.close()
        return out

    A, S = cfg.vortex_amp, cfg.stokes[0]
    h = 1e-4
    fd_amp = (J_of(A * (1 + h), S) - J_of(A * (1 - h), S)) / (2 * h)
    hs = 1e-5
    fd_st = (J_of(A, S + hs) - J_of(A, S - hs)) / (2 * hs)
    say(f"[autograd] amp: adjoint {got_amp:.12e} fd {fd_amp:.12e}; "
        f"stokes: adjoint {got_st:.12e} fd {fd_st:.12e}")
    assert got_amp == pytest.approx(fd_amp, rel=1e-5)
    assert got_st == pytest.approx(fd_st, rel=1e-6)


def test_adjoint_workload_200_steps_vs_finite_differences(rb):
    """The adjoint workload at its full size (128 x 256 x 32, one dust species), 200 CFL
    steps with checkpoints every 20: the gradient of the vortex-core dust mass with respect
    to a uniform change of the vortex amplitude and to the Stokes number, against central
    differences of the GPU forward run over the same time steps.  The differences follow
    the expected error curve -- truncation falling as h^2 from h = 1e-4 to 1e-5, rounding
    growing as 1/h below -- and meet the adjoint at their best step to 5e-6 (measured
    0.7e-6 to 2e-6: at h = 1e-5 the differences' own rounding floor, a relative rounding
    of J times J / (2 h dJ), is of that size and moves with the last bits of J)."""
    import torch
    cfg = synth.C5_ADJOINT
    n, k = 200, 20
    say(f"[adjoint 200] {cfg.name} n={n} checkpoints every {k}")
    xi = synth.noise(cfg)
    sim = rb.Sim(cfg, noise=xi)
    st, dts = sim.step(n)
    assert st == rb.RB_OK
    sim.close()
    lam_np = core_mass_cotangent(rb, cfg)
    lam = torch.as_tensor(lam_np, device="cuda")
    amp = torch.full((cfg.nz, cfg.nr, cfg.nth), cfg.vortex_amp, dtype=torch.float64,
                     device="cuda", requires_grad=True)
    stt = torch.tensor(cfg.stokes, dtype=torch.float64, requires_grad=True)
    final = rb.disc_run(amp, stt, cfg, n, dts, ckpt_every=k, noise=xi)
    (final * lam).sum().backward()
    g_amp = float(amp.grad.sum()) * cfg.vortex_amp
    g_st = float(stt.grad[0])

    def J_of(a, s):
        sm = rb.Sim(cfg.with_(stokes=(s,)), noise=xi, amp=np.full(cfg.n_cells, a))
        sm.step(n, dt_list=dts, check=True)
        out = float(np.sum(sm.fields() * lam_np))
        sm.close()
        return out

    A, S = cfg.vortex_amp, cfg.stokes[0]
    rel_a, rel_s = {}, {}
    for h in (1e-4, 1e-5, 1e-6):
        fa = (J_of(A * (1 + h), S) - J_of(A * (1 - h), S)) / (2 * h)
        fs = (J_of(A, S * (1 + h)) - J_of(A, S * (1 - h))) / (2 * h * S)
        rel_a[h], rel_s[h] = abs(fa / g_amp - 1), abs(fs / g_st - 1)
        say(f"[adjoint 200] h={h:.0e}: amplitude fd {fa:.10e} adjoint {g_amp:.10e} "
            f"(rel {rel_a[h]:.1e}); Stokes fd {fs:.10e} adjoint {g_st:.10e} (rel {rel_s[h]:.1e})")
    assert min(rel_a.values()) <= 5e-6 and min(rel_s.values()) <= 5e-6
    assert rel_a[1e-5] < rel_a[1e-4] / 10
