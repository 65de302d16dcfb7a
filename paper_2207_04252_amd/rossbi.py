"""Python binding of the MI355X bi-fluid finite-volume library (ctypes, marshalling only).

Every step of the computation runs in the HIP kernels of ``librossbi_mi355x.so``;
PyTorch provides the device buffers and the stream.  The function names follow the
C ABI of ``include/rossbi_mi355x.h``.  Loading fails loudly when the library has not
been built: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import synth

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librossbi_mi355x.so")

RB_OK, RB_EINVAL, RB_ENOMEM, RB_EDEVICE = 0, -1, -2, -3
RB_ENEGATIVE, RB_EVACUUM, RB_ENOCONV, RB_ESTIFF, RB_ESTATE = -4, -5, -6, -7, -8
RB_FP64, RB_FP32_PERT = 0, 1
RB_DT_CFL, RB_DT_FIXED, RB_DT_LIST = 0, 1, 2
STATUS_NAMES = {0: "RB_OK", -1: "RB_EINVAL", -2: "RB_ENOMEM", -3: "RB_EDEVICE",
                -4: "RB_ENEGATIVE", -5: "RB_EVACUUM", -6: "RB_ENOCONV", -7: "RB_ESTIFF",
                -8: "RB_ESTATE"}

_D = ctypes.POINTER(ctypes.c_double)


class rb_config(ctypes.Structure):
    _fields_ = [
        ("nr", ctypes.c_int32), ("ntheta", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("log_r", ctypes.c_int32), ("init_kind", ctypes.c_int32), ("balanced", ctypes.c_int32),
        ("n_dust", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("r_in", ctypes.c_double), ("r_out", ctypes.c_double), ("z_half", ctypes.c_double),
        ("gamma", ctypes.c_double), ("GM", ctypes.c_double), ("cfl", ctypes.c_double),
        ("sod_r0", ctypes.c_double), ("sod_left", ctypes.c_double * 3),
        ("sod_right", ctypes.c_double * 3),
        ("h0", ctypes.c_double), ("beta_T", ctypes.c_double), ("rho_mid0", ctypes.c_double),
        ("beta_rho", ctypes.c_double),
        ("vortex_amp", ctypes.c_double), ("vortex_r0", ctypes.c_double),
        ("vortex_th0", ctypes.c_double), ("vortex_sig_r", ctypes.c_double),
        ("vortex_sig_a", ctypes.c_double), ("noise_amp", ctypes.c_double),
        ("stokes", ctypes.c_double * 4), ("eps_dust", ctypes.c_double * 4),
        ("hd_over_h", ctypes.c_double * 4),
        ("indirect", ctypes.c_int32), ("drag_law", ctypes.c_int32),
        ("grain_size", ctypes.c_double * 4), ("grain_density", ctypes.c_double * 4),
        ("mfp_coef", ctypes.c_double),
        ("bc_r", ctypes.c_int32), ("bc_z", ctypes.c_int32),
        ("damp_r_in", ctypes.c_double), ("damp_r_out", ctypes.c_double),
        ("damp_z", ctypes.c_double), ("damp_tau", ctypes.c_double),
        ("rwi_m", ctypes.c_int32), ("newton_max_iter", ctypes.c_int32),
        ("rwi_delta", ctypes.c_double), ("rwi_dr", ctypes.c_double),
        ("rwi_r0", ctypes.c_double), ("rwi_eps", ctypes.c_double),
        ("drag_exact", ctypes.c_int32), ("pad_end", ctypes.c_int32),
    ]


class rb_buffers(ctypes.Structure):
    _fields_ = [("state", ctypes.c_void_p), ("stage", ctypes.c_void_p), ("work", ctypes.c_void_p),
                ("state_bytes", ctypes.c_size_t), ("stage_bytes", ctypes.c_size_t),
                ("work_bytes", ctypes.c_size_t)]


class rb_dt_policy(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("pad", ctypes.c_int32), ("dt", ctypes.c_double),
                ("dt_list", _D)]


class rb_diag(ctypes.Structure):
    _fields_ = [
        ("t", ctypes.c_double), ("step", ctypes.c_int64), ("flags", ctypes.c_int32),
        ("first_bad_step", ctypes.c_int32), ("first_bad_cell", ctypes.c_int64),
        ("fallbacks", ctypes.c_int64), ("vacuum_faces", ctypes.c_int64),
        ("max_newton", ctypes.c_int32), ("pad", ctypes.c_int32),
        ("mass", ctypes.c_double * 5), ("outflow", ctypes.c_double * 5),
        ("dt_last", ctypes.c_double), ("fp64_resolves", ctypes.c_int64),
        ("newton_hist", ctypes.c_int64 * 8), ("negative_dust", ctypes.c_int64),
    ]


# names exported by the library, in the order of include/rossbi_mi355x.h
EXPORTS = ("rb_query_sizes", "rb_init_state", "rb_step", "rb_get_fields", "rb_set_fields",
           "rb_eval_operator", "rb_get_residual", "rb_get_geometry", "rb_cfl_dt",
           "rb_cfl_dt_static", "rb_diagnostics", "rb_profile",
           "rb_profile_read", "rb_adjoint_workspace", "rb_record", "rb_adjoint",
           "rb_amp_gradient", "rb_last_error", "rb_destroy")

_lib = None


def load() -> ctypes.CDLL:
    """Load the built library (no build, no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library {LIB_PATH} is not built; run "
                           "`python -c 'import __graft_entry__ as g; g.build()'`")
    # torch brings its own copy of the HIP runtime; it must be the one loaded when the
    # library is, so that buffers and streams from torch belong to the library's runtime
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    L.rb_query_sizes.argtypes = [ctypes.POINTER(rb_config), ctypes.POINTER(rb_buffers)]
    L.rb_init_state.argtypes = [ctypes.POINTER(rb_config), ctypes.POINTER(rb_buffers), _D, _D,
                                ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]
    L.rb_step.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(rb_dt_policy), _D]
    L.rb_get_fields.argtypes = [ctypes.c_void_p, _D, ctypes.c_size_t]
    L.rb_set_fields.argtypes = [ctypes.c_void_p, _D, ctypes.c_size_t]
    L.rb_eval_operator.argtypes = [ctypes.c_void_p, _D, ctypes.c_size_t]
    L.rb_get_residual.argtypes = [ctypes.c_void_p, _D, ctypes.c_size_t]
    L.rb_get_geometry.argtypes = [ctypes.c_void_p, _D, _D, _D, _D]
    L.rb_cfl_dt.argtypes = [ctypes.c_void_p, _D]
    L.rb_cfl_dt_static.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    L.rb_diagnostics.argtypes = [ctypes.c_void_p, ctypes.POINTER(rb_diag)]
    L.rb_profile.argtypes = [ctypes.c_void_p, ctypes.c_int]
    L.rb_profile_read.argtypes = [ctypes.c_void_p, _D, ctypes.POINTER(ctypes.c_int64)]
    L.rb_adjoint_workspace.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                       ctypes.POINTER(ctypes.c_size_t)]
    L.rb_record.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                            ctypes.POINTER(rb_dt_policy), _D, ctypes.c_void_p, ctypes.c_size_t]
    L.rb_adjoint.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, _D,
                             ctypes.c_void_p, ctypes.c_size_t]
    L.rb_amp_gradient.argtypes = [ctypes.c_void_p, _D, _D, ctypes.c_void_p, ctypes.c_void_p]
    L.rb_last_error.argtypes = [ctypes.c_void_p]
    L.rb_last_error.restype = ctypes.c_char_p
    L.rb_destroy.argtypes = [ctypes.c_void_p]
    L.rb_destroy.restype = None
    for name in EXPORTS[:-2]:
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def to_config(cfg: synth.Config, precision: int = RB_FP64) -> rb_config:
    c = rb_config()
    c.nr, c.ntheta, c.nz = cfg.nr, cfg.nth, cfg.nz
    c.log_r = int(cfg.log_r)
    c.init_kind = cfg.init_kind
    c.balanced = int(cfg.balanced)
    c.n_dust = cfg.n_dust
    c.precision = precision
    c.r_in, c.r_out, c.z_half = cfg.r_in, cfg.r_out, cfg.z_half
    c.gamma, c.GM, c.cfl = cfg.gamma, cfg.GM, cfg.cfl
    c.sod_r0 = cfg.sod_r0
    for q in range(3):
        c.sod_left[q] = cfg.sod_left[q]
        c.sod_right[q] = cfg.sod_right[q]
    c.h0, c.beta_T, c.rho_mid0, c.beta_rho = cfg.h0, cfg.beta_T, cfg.rho_mid0, cfg.beta_rho
    c.vortex_amp, c.vortex_r0, c.vortex_th0 = cfg.vortex_amp, cfg.vortex_r0, cfg.vortex_th0
    c.vortex_sig_r, c.vortex_sig_a, c.noise_amp = cfg.vortex_sig_r, cfg.vortex_sig_a, cfg.noise_amp
    for q in range(cfg.n_dust):
        c.stokes[q] = cfg.stokes[q]
        c.eps_dust[q] = cfg.eps_dust[q]
        c.hd_over_h[q] = cfg.hd_over_h[q]
    c.indirect = int(cfg.indirect)
    c.drag_law = int(cfg.drag_law)
    if cfg.drag_law:
        for q in range(cfg.n_dust):
            c.grain_size[q] = cfg.grain_size[q]
            c.grain_density[q] = cfg.grain_density[q]
        c.mfp_coef = cfg.mfp_coef
    c.bc_r, c.bc_z = int(cfg.bc_r), int(cfg.bc_z)
    c.damp_r_in, c.damp_r_out, c.damp_z, c.damp_tau = (cfg.damp_r_in, cfg.damp_r_out,
                                                       cfg.damp_z, cfg.damp_tau)
    c.rwi_m = int(cfg.rwi_m)
    c.newton_max_iter = int(cfg.newton_max_iter)
    c.drag_exact = int(cfg.drag_exact)
    c.rwi_delta, c.rwi_dr, c.rwi_r0, c.rwi_eps = (cfg.rwi_delta, cfg.rwi_dr, cfg.rwi_r0,
                                                  cfg.rwi_eps)
    return c


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_D)


class RbError(RuntimeError):
    def __init__(self, status, msg=""):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Sim:
    """One simulation on the GPU: caller-owned torch buffers and stream, one rb_ctx."""

    def __init__(self, cfg: synth.Config, precision: int = RB_FP64, noise: np.ndarray | None = None,
                 amp: np.ndarray | None = None, device: str = "cuda:0", stream=None):
        import torch
        self.cfg = cfg
        self.lib = load()
        self.c = to_config(cfg, precision)
        sizes = rb_buffers()
        st = self.lib.rb_query_sizes(ctypes.byref(self.c), ctypes.byref(sizes))
        if st != RB_OK:
            raise RbError(st, "rb_query_sizes rejected the configuration")
        dev = torch.device(device)
        self.state = torch.empty(sizes.state_bytes, dtype=torch.uint8, device=dev)
        self.stage = torch.empty(sizes.stage_bytes, dtype=torch.uint8, device=dev)
        self.work = torch.empty(sizes.work_bytes, dtype=torch.uint8, device=dev)
        for t in (self.state, self.stage, self.work):
            if t.data_ptr() % 256:
                raise RuntimeError("device buffer not 256-byte aligned")
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        bufs = rb_buffers(self.state.data_ptr(), self.stage.data_ptr(), self.work.data_ptr(),
                          sizes.state_bytes, sizes.stage_bytes, sizes.work_bytes)
        self._noise = None if noise is None else np.ascontiguousarray(noise, dtype=np.float64)
        self._amp = None if amp is None else np.ascontiguousarray(amp, dtype=np.float64)
        if self._noise is not None and self._noise.size != cfg.n_cells * (1 + cfg.n_dust):
            raise ValueError("noise must have one value per cell and fluid")
        if self._amp is not None and self._amp.size != cfg.n_cells:
            raise ValueError("amp must have one value per cell")
        ctx = ctypes.c_void_p()
        st = self.lib.rb_init_state(ctypes.byref(self.c), ctypes.byref(bufs), _ptr(self._noise),
                                    _ptr(self._amp), ctypes.c_void_p(self.stream.cuda_stream),
                                    ctypes.byref(ctx))
        if st != RB_OK:
            raise RbError(st, "rb_init_state failed")
        self.ctx = ctx
        self.nf = cfg.n_fields
        self.shape = (self.nf, cfg.nz, cfg.nr, cfg.nth)

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.rb_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def error(self) -> str:
        return self.lib.rb_last_error(self.ctx).decode()

    @staticmethod
    def _policy(dt, dt_list):
        pol = rb_dt_policy()
        lst = None
        if dt_list is not None:
            lst = np.ascontiguousarray(dt_list, dtype=np.float64)
            pol.kind, pol.dt_list = RB_DT_LIST, _ptr(lst)
        elif dt is not None:
            pol.kind, pol.dt = RB_DT_FIXED, float(dt)
        else:
            pol.kind = RB_DT_CFL
        return pol, lst

    def step(self, n: int, dt: float | None = None, dt_list=None, check: bool = False):
        """rb_step: n steps (CFL default, fixed dt, or dt list). Returns (status, dts)."""
        pol, lst = self._policy(dt, dt_list)
        dts = np.zeros(max(n, 1))
        st = self.lib.rb_step(self.ctx, n, ctypes.byref(pol), _ptr(dts))
        if check and st != RB_OK:
            raise RbError(st, self.error())
        return st, dts[:n]

    def fields(self) -> np.ndarray:
        out = np.empty(self.shape)
        st = self.lib.rb_get_fields(self.ctx, _ptr(out), out.size)
        if st != RB_OK:
            raise RbError(st, self.error())
        return out

    def set_fields(self, arr: np.ndarray):
        a = np.ascontiguousarray(arr, dtype=np.float64)
        st = self.lib.rb_set_fields(self.ctx, _ptr(a), a.size)
        if st != RB_OK:
            raise RbError(st, self.error())

    def operator(self) -> np.ndarray:
        out = np.empty(self.shape)
        st = self.lib.rb_eval_operator(self.ctx, _ptr(out), out.size)
        if st != RB_OK:
            raise RbError(st, self.error())
        return out

    def residual(self) -> np.ndarray:
        out = np.empty((self.cfg.nz, self.cfg.nr, 5))
        st = self.lib.rb_get_residual(self.ctx, _ptr(out), out.size)
        if st != RB_OK:
            raise RbError(st, self.error())
        return out

    def geometry(self) -> dict:
        """rb_get_geometry: r faces, r centres, cell volume per radial row, z centres."""
        c = self.cfg
        g = dict(rf=np.empty(c.nr + 1), rc=np.empty(c.nr), V=np.empty(c.nr), zc=np.empty(c.nz))
        st = self.lib.rb_get_geometry(self.ctx, _ptr(g["rf"]), _ptr(g["rc"]), _ptr(g["V"]),
                                      _ptr(g["zc"]))
        if st != RB_OK:
            raise RbError(st, self.error())
        return g

    def cfl_dt(self) -> float:
        d = ctypes.c_double()
        st = self.lib.rb_cfl_dt(self.ctx, ctypes.byref(d))
        if st != RB_OK:
            raise RbError(st, self.error())
        return d.value

    def diagnostics(self) -> rb_diag:
        d = rb_diag()
        st = self.lib.rb_diagnostics(self.ctx, ctypes.byref(d))
        if st != RB_OK:
            raise RbError(st, self.error())
        return d

    def profile(self, enable: bool = True):
        st = self.lib.rb_profile(self.ctx, int(enable))
        if st != RB_OK:
            raise RbError(st, self.error())

    def profile_read(self):
        """Per kernel kind (gas stage, dust stage, reductions): (total ms, launches)."""
        ms = np.zeros(3)
        n = (ctypes.c_int64 * 3)()
        st = self.lib.rb_profile_read(self.ctx, _ptr(ms), n)
        if st != RB_OK:
            raise RbError(st, self.error())
        return ms, np.array(list(n))

    def mass(self) -> np.ndarray:
        return np.array(self.diagnostics().mass)[: 1 + self.cfg.n_dust]

    # ---- discrete adjoint
    def record(self, n: int, ckpt_every: int = 20, dt: float | None = None, dt_list=None):
        """rb_record: n steps with checkpoints every ckpt_every steps (workspace held by
        this object until the next record).  Returns the time steps."""
        import torch
        size = ctypes.c_size_t()
        st = self.lib.rb_adjoint_workspace(self.ctx, n, ckpt_every, ctypes.byref(size))
        if st != RB_OK:
            raise RbError(st, "rb_adjoint_workspace")
        self._ws = torch.empty(size.value, dtype=torch.uint8, device=self.state.device)
        pol, lst = self._policy(dt, dt_list)
        dts = np.zeros(n)
        st = self.lib.rb_record(self.ctx, n, ckpt_every, ctypes.byref(pol), _ptr(dts),
                                ctypes.c_void_p(self._ws.data_ptr()), size.value)
        if st != RB_OK:
            raise RbError(st, self.error())
        return dts

    def adjoint(self, lam_final):
        """rb_adjoint: lam_final = dJ/dE after the recorded steps (array or torch tensor of
        the fields' shape).  Returns (dJ/dE before them as a float64 device tensor,
        dJ/dSt per dust species)."""
        import torch
        lam = torch.as_tensor(lam_final, dtype=torch.float64, device=self.state.device)
        lam = lam.reshape(self.shape).contiguous()
        grad = torch.empty_like(lam)
        gst = np.zeros(max(self.cfg.n_dust, 1))
        st = self.lib.rb_adjoint(self.ctx, ctypes.c_void_p(lam.data_ptr()),
                                 ctypes.c_void_p(grad.data_ptr()), _ptr(gst),
                                 ctypes.c_void_p(self._ws.data_ptr()), self._ws.numel())
        if st != RB_OK:
            raise RbError(st, self.error())
        return grad, gst[: self.cfg.n_dust]

    def amp_gradient(self, grad_state0, noise=None, amp=None):
        """rb_amp_gradient: dJ/dA per cell from dJ/dE of the initial state (noise and amp
        as given at initialisation).  Returns a float64 device tensor (nz, nr, ntheta)."""
        import torch
        lam = torch.as_tensor(grad_state0, dtype=torch.float64, device=self.state.device)
        lam = lam.reshape(self.shape).contiguous()
        out = torch.empty(self.shape[1:], dtype=torch.float64, device=self.state.device)
        nz = None if noise is None else np.ascontiguousarray(noise, dtype=np.float64)
        am = None if amp is None else np.ascontiguousarray(amp, dtype=np.float64)
        st = self.lib.rb_amp_gradient(self.ctx, _ptr(nz), _ptr(am), ctypes.c_void_p(lam.data_ptr()),
                                      ctypes.c_void_p(out.data_ptr()))
        if st != RB_OK:
            raise RbError(st, self.error())
        return out


def _make_disc_run():
    import torch

    class DiscRun(torch.autograd.Function):
        """n RK2 steps of the disc from its initial state with the given time steps,
        differentiable with respect to the per-cell vortex amplitude field and the Stokes
        numbers.  Forward: rb_record (checkpoints every ckpt_every steps); backward:
        rb_adjoint + rb_amp_gradient.  Returns the final fields (float64, on the device);
        the gradients come back on the devices of amp and stokes."""

        @staticmethod
        def forward(ctx, amp, stokes, cfg, n, ckpt_every, noise, dt_list):
            st_vals = tuple(float(v) for v in stokes.detach().cpu().numpy())
            c2 = cfg.with_(stokes=st_vals) if cfg.n_dust else cfg
            amp_np = amp.detach().cpu().numpy().astype(np.float64).reshape(cfg.nz, cfg.nr, cfg.nth)
            sim = Sim(c2, noise=noise, amp=amp_np, device=amp.device if amp.is_cuda else "cuda")
            dts = sim.record(n, ckpt_every, dt_list=dt_list)
            out = torch.as_tensor(sim.fields(), device=sim.state.device)
            ctx.sim, ctx.noise, ctx.amp_np, ctx.dts = sim, noise, amp_np, dts
            ctx.amp_shape, ctx.amp_device, ctx.st_device = amp.shape, amp.device, stokes.device
            return out

        @staticmethod
        def backward(ctx, grad_out):
            sim = ctx.sim
            g0, gst = sim.adjoint(grad_out.detach())
            gamp = sim.amp_gradient(g0, noise=ctx.noise, amp=ctx.amp_np)
            sim.close()
            ctx.sim = None
            gamp = gamp.reshape(ctx.amp_shape).to(ctx.amp_device)
            gst_t = torch.as_tensor(gst, dtype=torch.float64, device=ctx.st_device)
            return gamp, gst_t, None, None, None, None, None

    return DiscRun


_disc_run = None


def disc_run(amp, stokes, cfg: synth.Config, n: int, dt_list, ckpt_every: int = 20, noise=None):
    """Differentiable n-step disc run (torch.autograd): see DiscRun.  The time steps are
    given (dt_list, n entries): the adjoint differentiates the step map at fixed steps, so
    a run with Courant steps, which depend on the amplitude and the Stokes numbers, has no
    gradient here."""
    if dt_list is None or len(dt_list) != n:
        raise ValueError("disc_run needs the n time steps (dt_list): the gradient is taken at "
                         "fixed steps")
    global _disc_run
    if _disc_run is None:
        _disc_run = _make_disc_run()
    return _disc_run.apply(amp, stokes, cfg, n, ckpt_every, noise, dt_list)
