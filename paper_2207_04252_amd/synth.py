"""Seeded synthetic inputs for the bi-fluid disc step.

This module holds the named workload configurations and the seeded noise
generator.  It is the only module that both the HIP library binding and the
CPU oracle read: it contains parameters and random numbers, and none of the
method's arithmetic (no mesh, no equilibrium, no flux).

Noise: SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014), keyed by ``seed XOR (fluid*ncells + global cell index)``
with the global index ``(k*nr + i)*ntheta + j`` and fluid 0 the gas, 1 + s dust
species s; the top 53 bits give a uniform double in [0, 1) which is mapped to
[-1, 1).  Every fluid's density carries its own noise.
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field, replace
from typing import Tuple

import numpy as np

INIT_SOD = 0
INIT_DISC = 1

DEFAULT_SEED = 220704252


@dataclass(frozen=True)
class Config:
    """One workload: grid, physics constants, initial-state recipe."""
    name: str
    nr: int
    nth: int
    nz: int
    log_r: bool
    r_in: float
    r_out: float
    z_half: float
    init_kind: int
    gamma: float = 1.4
    GM: float = 1.0
    cfl: float = 0.5
    balanced: bool = True
    # Sod annulus (init_kind == INIT_SOD): (rho, p, u_r) left/right of sod_r0
    sod_r0: float = 1.5
    sod_left: Tuple[float, float, float] = (1.0, 1.0, 0.0)
    sod_right: Tuple[float, float, float] = (0.125, 0.1, 0.0)
    # disc (init_kind == INIT_DISC): H/r = h0 at r = 1, T ~ r^beta_T,
    # midplane density rho_mid0 * r^beta_rho
    h0: float = 0.05
    beta_T: float = -0.5
    rho_mid0: float = 1.0
    beta_rho: float = -1.5
    # column Gaussian vortex (streamfunction), amplitude = -Rossby number
    vortex_amp: float = 0.0
    vortex_r0: float = 1.0
    vortex_th0: float = math.pi
    vortex_sig_r: float = 0.05
    vortex_sig_a: float = 0.15
    noise_amp: float = 0.0
    seed: int = DEFAULT_SEED
    stokes: Tuple[float, ...] = ()
    eps_dust: Tuple[float, ...] = ()
    hd_over_h: Tuple[float, ...] = ()
    steps: int = 100
    indirect: bool = False      # indirect gravity of the star's displacement (Sect. 2.10)
    # drag law (Sect. 2.9): 0 constant Stokes number (t_s = St / Omega_K); 1 Epstein /
    # Stokes regimes from the grain radius and material density, with the gas mean free
    # path lambda = mfp_coef / rho_g (code units)
    drag_law: int = 0
    # drag integration: False, explicit in the RK2 stages (the step must stay below the
    # smallest stopping time); True, the drag is split off and integrated exactly over
    # half steps before and after the stages (Strang), so any step is allowed
    drag_exact: bool = False
    grain_size: Tuple[float, ...] = ()
    grain_density: Tuple[float, ...] = ()
    mfp_coef: float = 0.0
    # boundary conditions (Sect. 2.4).  bc_r: 0 ghosts hold the stationary (sheared) flow;
    # 1 adds wave-killing zones r < damp_r_in r_in and r > damp_r_out r_out.  bc_z: 0
    # stationary ghosts; 1 outflow (ghosts repeat the boundary cell's deviation); 2 sheared
    # damped zones |z| > damp_z z_half.  Damping relaxes the gas deviation at rate R / tau,
    # R rising quadratically from 0 at the zone edge to 1 at the boundary, tau = damp_tau
    # orbital periods (at the boundary radius; at the cell radius for the z zones).
    bc_r: int = 0
    bc_z: int = 0
    damp_r_in: float = 1.25
    damp_r_out: float = 0.84
    damp_z: float = 0.8
    damp_tau: float = 1.0
    # Rossby-wave-instability seed (Sect. 4.3): density bump 1 + rwi_delta exp(-(r -
    # rwi_r0)^2 / (2 rwi_dr^2)) at unchanged temperature with v_theta rebalanced, and a
    # radial velocity rwi_eps v_theta0 sin(rwi_m theta) with the same Gaussian profile
    rwi_m: int = 0
    rwi_delta: float = 0.0
    rwi_dr: float = 0.05
    rwi_r0: float = 1.0
    rwi_eps: float = 0.0
    # cap on the Newton iterations of the exact gas solver (0: the default 50); a face that
    # needs more stops the run with the no-convergence error
    newton_max_iter: int = 0

    @property
    def n_dust(self) -> int:
        return len(self.stokes)

    @property
    def n_fields(self) -> int:
        return 5 + 4 * self.n_dust

    @property
    def n_cells(self) -> int:
        return self.nr * self.nth * self.nz

    def scaled(self, nr: int, nth: int, nz: int, name: str | None = None) -> "Config":
        """Same physics on another grid (for tests that the oracle finishes in seconds)."""
        return replace(self, nr=nr, nth=nth, nz=nz,
                       name=name or f"{self.name}@{nr}x{nth}x{nz}")

    def with_(self, **kw) -> "Config":
        return replace(self, **kw)


def _disc(name, nr, nth, nz, **kw) -> Config:
    base = dict(log_r=True, r_in=0.5, r_out=2.0, z_half=0.15, init_kind=INIT_DISC,
                GM=1.0, balanced=True, vortex_amp=1e-3, noise_amp=1e-6)
    base.update(kw)
    return Config(name=name, nr=nr, nth=nth, nz=nz, **base)


# The five workloads (grid sizes and physics as the paper's test outlines,
# at the resolutions used for measurement).
C1_SOD = Config(name="sod_annulus_256x64x1", nr=256, nth=64, nz=1, log_r=False,
                r_in=1.0, r_out=2.0, z_half=0.5, init_kind=INIT_SOD, GM=0.0,
                balanced=False, steps=100)
C2_DISC = _disc("gas_disc_128x256x64", 128, 256, 64, steps=200)
C3_BIFLUID = _disc("bifluid_disc_256x512x64", 256, 512, 64, stokes=(0.1,),
                   eps_dust=(0.01,), hd_over_h=(0.3,), steps=500)
C4_LARGE = _disc("bifluid3_disc_512x1024x128", 512, 1024, 128, vortex_amp=1e-2,
                 stokes=(0.01, 0.1, 1.0), eps_dust=(0.0033, 0.0033, 0.0033),
                 hd_over_h=(0.3, 0.3, 0.3), steps=1000)
C5_ADJOINT = _disc("adjoint_disc_128x256x32", 128, 256, 32, stokes=(0.1,),
                   eps_dust=(0.01,), hd_over_h=(0.3,), steps=200)

# Rossby-wave-instability test (Sect. 4.3): gas disc of the second workload with a density
# bump (amplitude 0.2 and width 0.05 at r = 1: readings, the paper gives neither) and the
# m = 4 radial-velocity seed of amplitude 1e-4; no vortex
C6_RWI = _disc("rwi_disc_128x256x64", 128, 256, 64, vortex_amp=0.0, rwi_m=4, rwi_delta=0.2,
               rwi_dr=0.05, rwi_r0=1.0, rwi_eps=1e-4, steps=200)

CONFIGS = {c.name: c for c in (C1_SOD, C2_DISC, C3_BIFLUID, C4_LARGE, C5_ADJOINT, C6_RWI)}


def epstein_grains(cfg: Config, rho_switch: float = 0.5, rho_s: float = 1.0) -> Config:
    """The disc cfg with the Epstein / Stokes drag law (Sect. 2.9) in place of constant
    Stokes numbers: each species gets the grain radius whose Epstein stopping time at
    r = 1, z = 0 of the stationary disc is its configured Stokes number (material density
    rho_s), and the mean-free-path constant puts the regime switch r_p = 9 lambda / 4 of
    the middle species at gas density rho_switch, so that grains of that size are in the
    Stokes regime in the dense inner midplane and in the Epstein regime elsewhere."""
    assert cfg.init_kind == INIT_DISC and cfg.n_dust > 0
    c1 = cfg.h0 * math.sqrt(cfg.GM)          # isothermal sound speed at r = 1
    om1 = math.sqrt(cfg.GM)
    sizes = tuple(st * cfg.rho_mid0 * c1 / (om1 * rho_s) for st in cfg.stokes)
    mid = sizes[len(sizes) // 2]
    return cfg.with_(drag_law=1, grain_size=sizes, grain_density=(rho_s,) * len(sizes),
                     mfp_coef=4.0 * rho_switch * mid / 9.0,
                     name=cfg.name.replace("_disc", "_epstein_disc", 1))

# vortex core region used by the adjoint objective (dust mass in the core)
CORE_R = (0.9, 1.1)
CORE_DTH = 0.3

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def splitmix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 output function applied elementwise to uint64 keys."""
    with np.errstate(over="ignore"):
        z = (x + np.uint64(0x9E3779B97F4A7C15)) & _M64
        z = ((z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)) & _M64
        z = ((z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)) & _M64
        return z ^ (z >> np.uint64(31))


def noise(cfg: Config) -> np.ndarray:
    """Uniform noise xi in [-1, 1) for the density of every fluid (gas, then each dust
    species), shape (1 + n_dust, nz, nr, nth), float64, C order."""
    n = cfg.n_cells * (1 + cfg.n_dust)
    idx = np.arange(n, dtype=np.uint64)
    z = splitmix64(np.uint64(cfg.seed) ^ idx)
    u = (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    return (2.0 * u - 1.0).reshape(1 + cfg.n_dust, cfg.nz, cfg.nr, cfg.nth)


def amplitude_field(cfg: Config, amp: float | None = None) -> np.ndarray:
    """Per-cell vortex amplitude field (uniform at the config's amplitude)."""
    a = cfg.vortex_amp if amp is None else amp
    return np.full((cfg.nz, cfg.nr, cfg.nth), a, dtype=np.float64)


def random_direction(cfg: Config, seed: int = 7) -> np.ndarray:
    """Seeded random field in [-1, 1) used as a tangent direction in gradient checks."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=(cfg.nz, cfg.nr, cfg.nth))


def config_dict(cfg: Config) -> dict:
    return dataclasses.asdict(cfg)
