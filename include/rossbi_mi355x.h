/*
 * rossbi_mi355x.h -- C ABI of the MI355X (gfx950) library for one time step of the
 * RoSSBi3D bi-fluid finite-volume scheme (Rendon Restrepo & Barge, arXiv 2207.04252).
 *
 * The library advances a compressible inviscid ideal gas and up to four pressureless
 * dust fluids on a cylindrical (r, theta, z) grid: parabolic reconstruction of the
 * deviation from the stationary flow with a MinMod limiter (Sect. 2.7), an exact
 * Riemann problem at every interface (Sect. 2.6; pressureless for the dust, Sect. 2.9),
 * flux divergence with geometric, gravity and drag sources (Sect. 2.1, App. B), the
 * empty-run residual of the balanced scheme (Sect. 2.8), the RK2 midpoint step and the
 * CFL time step (Sect. 2.5).
 *
 * Conventions for every call:
 *   - return value: rb_status, 0 on success, negative on error;
 *   - device memory for the state, the stage buffer and the work area is allocated by
 *     the caller (for instance as torch tensors) and passed as raw device pointers; the
 *     library allocates no device memory;
 *   - all work is issued on the caller's HIP stream; calls that return host data
 *     synchronise that stream;
 *   - a context is thread-compatible, not thread-safe: calls on one context must not
 *     overlap;
 *   - fields are stored field-major, then z, then r, then theta:
 *     index = ((f * nz + k) * nr + i) * ntheta + j, theta contiguous.  Field order:
 *     gas (rho u, rho v, rho w, E, rho) with u, v, w the r, theta, z velocities
 *     (App. B), then for each dust species (rho_d u, rho_d v, rho_d w, rho_d).
 */
#ifndef ROSSBI_MI355X_H
#define ROSSBI_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RB_OK = 0,
  RB_EINVAL = -1,    /* bad argument or configuration                              */
  RB_ENOMEM = -2,    /* a caller buffer is smaller than rb_query_sizes asked for   */
  RB_EDEVICE = -3,   /* a HIP call failed                                          */
  RB_ENEGATIVE = -4, /* a cell has rho <= 0 or p <= 0 (or NaN)                     */
  RB_EVACUUM = -5,   /* a Riemann problem generated vacuum (run completed)         */
  RB_ENOCONV = -6,   /* Newton on p* did not converge in 50 iterations             */
  RB_ESTIFF = -7,    /* dt >= the smallest dust stopping time                      */
  RB_ESTATE = -8     /* call made in the wrong state (e.g. after a hard error)    */
} rb_status;

typedef enum { RB_FP64 = 0, RB_FP32_PERT = 1 } rb_precision;

typedef enum { RB_DT_CFL = 0, RB_DT_FIXED = 1, RB_DT_LIST = 2 } rb_dt_kind;

enum { RB_INIT_SOD = 0, RB_INIT_DISC = 1 };

/* Time-step policy.  CFL: dt = min over cells of cfl V / ((|v| + c_s) max|dA|), the
 * dust adding its own speed (Sect. 2.5); FIXED: dt; LIST: dt_list[q] for step q of the
 * call (host pointer, n entries). */
typedef struct {
  int32_t kind;
  int32_t pad;
  double dt;
  const double* dt_list;
} rb_dt_policy;

/* Problem statement (Sect. 2.1-2.5, App. A).  Code units: GM and r = 1 set the unit of
 * length and time; the disc has H/r = h0 at r = 1, temperature ~ r^beta_T and midplane
 * density rho_mid0 r^beta_rho; z in [-z_half, z_half] (nz == 1: 2D, no z faces). */
typedef struct {
  int32_t nr, ntheta, nz;     /* interior cells                                     */
  int32_t log_r;              /* 1: logarithmic radial faces (Sect. 2.3), 0: uniform  */
  int32_t init_kind;          /* RB_INIT_SOD or RB_INIT_DISC                         */
  int32_t balanced;           /* subtract the empty-run residual (Sect. 2.8)         */
  int32_t n_dust;             /* 0..4 pressureless dust species                      */
  int32_t precision;          /* rb_precision                                        */
  double r_in, r_out, z_half;
  double gamma, GM, cfl;
  /* Sod annulus: (rho, p, u_r) for r < sod_r0 and r >= sod_r0                        */
  double sod_r0, sod_left[3], sod_right[3];
  /* disc                                                                              */
  double h0, beta_T, rho_mid0, beta_rho;
  /* column Gaussian vortex of the initial state (amplitude = -Rossby number), and the
   * relative amplitude of the density noise                                           */
  double vortex_amp, vortex_r0, vortex_th0, vortex_sig_r, vortex_sig_a, noise_amp;
  /* dust: Stokes number (t_s = St / Omega_K), dust-to-gas column ratio, H_d / H       */
  double stokes[4], eps_dust[4], hd_over_h[4];
  /* 1: indirect gravity (Sect. 2.10) -- every fluid element feels minus the star's
   * acceleration by the disc, G sum m r_vec/|r_vec|^3 over gas and dust (G = GM, unit star
   * mass); recomputed from each stage's input.  Disc only; not with rb_record.          */
  int32_t indirect;
  /* drag law (Sect. 2.9).  0: constant Stokes number, t_s = stokes[s] / Omega_K(r).
   * 1: Epstein / Stokes regimes from the gas state of each cell: with c_s = sqrt(p/rho)
   * (the isothermal sound speed of App. A) and the mean free path lambda = mfp_coef/rho
   * (mu m_u / sigma_eff folded into one code-unit constant), t^E = grain_density
   * grain_size / (rho c_s) while grain_size <= 9 lambda / 4, else (4/9)(grain_size /
   * lambda) t^E.  The stiffness check (RB_ESTIFF) then takes the minimum over cells of
   * the state at the start of each step.  stokes[] is unused by law 1; not with
   * rb_record.                                                                         */
  int32_t drag_law;
  double grain_size[4], grain_density[4], mfp_coef;
  /* boundary conditions (Sect. 2.4; disc only).  bc_r 0: r ghosts hold the stationary
   * sheared flow; 1: in addition, wave-killing zones r < damp_r_in r_in and
   * r > damp_r_out r_out.  bc_z 0: z ghosts hold the stationary flow; 1: outflow, the
   * two z ghosts carry the boundary cell's gas deviation scaled by the ratio of the
   * stationary densities (zero gradient of E'/rho0) and repeat its dust variables; 2:
   * sheared damped zones |z| > damp_z z_half.  A damping zone relaxes the gas deviation from the
   * stationary flow at the rate R / tau added to the operator (V dE'/dt = ... - V R E'/tau),
   * R = x^2 with x rising linearly from 0 at the zone edge to 1 at the boundary and
   * tau = damp_tau orbital periods 2 pi / Omega_K at the boundary radius (radial zones)
   * or at the cell radius (vertical zones).  Not with rb_record.                       */
  int32_t bc_r, bc_z;
  double damp_r_in, damp_r_out, damp_z, damp_tau;
  /* Rossby-wave-instability seed of the initial disc (Sect. 4.3; 0 amplitudes: none):
   * density and pressure times B = 1 + rwi_delta exp(-(r - rwi_r0)^2 / (2 rwi_dr^2))
   * (temperature unchanged), v_theta^2 = v_theta0^2 + r c_iso^2 B'/B (radial balance), and
   * v_r = rwi_eps v_theta0 sin(rwi_m theta) exp(-(r - rwi_r0)^2 / (2 rwi_dr^2)).
   * rb_amp_gradient refuses a seeded disc.                                              */
  int32_t rwi_m;
  /* Cap on the Newton iterations of the exact gas solver (Sect. 2.6); 0 means 50.  A face
   * that does not converge within it stops the run with RB_ENOCONV.                     */
  int32_t newton_max_iter;
  double rwi_delta, rwi_dr, rwi_r0, rwi_eps;
  /* Drag integration (Sect. 2.9 forces).  0: explicit, inside the RK2 stages; a step at or
   * above the smallest stopping time stops the run with RB_ESTIFF.  1: split off and
   * integrated exactly (Strang): each step is the drag alone over dt/2, the two RK2
   * stages of the operator without drag, the drag alone over dt/2.  The drag alone
   * keeps the densities and stopping times of each cell and the total momentum; the
   * dust-gas velocity differences relax as exp(tau B), B = -diag(1/t_s) - 1 (eps/t)^T
   * (eps_s = rho_s/rho_g; dust cells with rho_s <= 0 take no part); the gas energy changes
   * by the gas kinetic-energy change.  Any step is allowed; rb_eval_operator then
   * returns the operator without drag.  Not with rb_record.                            */
  int32_t drag_exact;
  int32_t pad_end;
} rb_config;

/* Caller-owned device buffers.  Sizes come from rb_query_sizes; pointers must be
 * 256-byte aligned device addresses that stay valid until rb_destroy. */
/* State layout.  FP64: all fields in FP64, field-major.  FP32-perturbation: the gas
 * deviation E' (5 fields) and the dust velocity deviations from the stationary flow's
 * (3 per species: radial, azimuthal minus the gas equilibrium's, vertical), in FP32,
 * padded to a multiple of 64 floats, then the dust densities in FP64.
 * rb_get_fields / rb_set_fields always exchange FP64 full values. */
typedef struct {
  void* state;   /* the state (layout above)                                          */
  void* stage;   /* midpoint state of the RK2 step, same layout and type             */
  void* work;    /* geometry, background, residual tables and reduction partials     */
  size_t state_bytes, stage_bytes, work_bytes;
} rb_buffers;

typedef struct {
  double t;               /* simulated time                                          */
  int64_t step;           /* completed steps                                         */
  int32_t flags;          /* bit 0 negative, 1 vacuum, 2 no convergence, 3 stiff    */
  int32_t first_bad_step; /* step at which a hard error was first seen, or -1        */
  int64_t first_bad_cell; /* lowest global cell index (k*nr + i)*ntheta + j, or -1   */
  int64_t fallbacks;      /* face states replaced by the cell-centre state           */
  int64_t vacuum_faces;   /* Riemann problems that generated vacuum                  */
  int32_t max_newton;     /* largest Newton iteration count seen                     */
  int32_t pad;
  double mass[5];         /* total gas mass, then each dust species                  */
  double outflow[5];      /* boundary mass outflow rate of the last second stage     */
  double dt_last;         /* last time step                                          */
  int64_t fp64_resolves;  /* FP32-perturbation faces re-solved by the FP64 solver    */
  int64_t newton_hist[8]; /* gas face solves by the Newton iteration count of the     */
                          /* solve whose flux was kept (Sect. 2.6): bin 0 none needed */
                          /* (supersonic face, vacuum), bins 1-6 that many, bin 7     */
                          /* seven or more; every face of the mesh once per stage     */
                          /* evaluation                                               */
  int64_t negative_dust;  /* cells and species whose dust density was negative at the */
                          /* end of a step, summed over steps                         */
} rb_diag;

typedef struct rb_ctx rb_ctx;

/* Fills the three *_bytes fields for cfg (pointers untouched).  EINVAL on a bad cfg. */
rb_status rb_query_sizes(const rb_config* cfg, rb_buffers* sizes);

/* Builds the geometry, the stationary flow at cell and face centres (App. A), the
 * empty-run residual R0 = G(E0) (Sect. 2.8, computed by the step kernel itself) and
 * the initial state, all on the device.  noise: host array of (1 + n_dust) x ncells
 * doubles in [-1, 1), one field per fluid (gas, then each dust species), each
 * multiplying noise_amp in that fluid's initial density (NULL: no noise); amp: host
 * array of ncells vortex amplitudes (NULL: vortex_amp everywhere).  Both are read before
 * the call returns.
 * stream: hipStream_t (NULL: default stream).  *out receives the context. */
rb_status rb_init_state(const rb_config* cfg, const rb_buffers* bufs, const double* noise,
                        const double* amp, void* stream, rb_ctx** out);

/* Advances n RK2 steps (Sect. 2.5) entirely on the device, with no host
 * synchronisation between steps.  dt_out (host, n entries, may be NULL) receives the
 * time steps.  Hard errors (ENEGATIVE, ENOCONV, ESTIFF) stop the evolution at the
 * step where they occur and are sticky until rb_set_fields; EVACUUM is reported after
 * the n steps complete. */
rb_status rb_step(rb_ctx* ctx, int n, const rb_dt_policy* policy, double* dt_out);

/* Copies the full conservative state E0 + E' (gas) and the dust variables to host
 * memory, FP64, in the field layout above; n_doubles must be nfields * ncells. */
rb_status rb_get_fields(rb_ctx* ctx, double* host_out, size_t n_doubles);

/* Replaces the state from host memory (same layout as rb_get_fields) and clears the
 * error flags. */
rb_status rb_set_fields(rb_ctx* ctx, const double* host_in, size_t n_doubles);

/* Writes the spatial operator of the current state to host memory: G(E) - R0 for the
 * gas (R0 subtracted when balanced) and G for the dust, FP64, field layout above
 * (Sect. 2.2: V dE/dt = G). */
rb_status rb_eval_operator(rb_ctx* ctx, double* host_out, size_t n_doubles);

/* Copies the empty-run residual R0 to host memory, [nz][nr][5]. */
rb_status rb_get_residual(rb_ctx* ctx, double* host_out, size_t n_doubles);

/* The mesh of the context as the kernels use it (Sect. 2.3): r_faces[nr + 1] (logarithmic
 * or uniform in r), r_centres[nr] (mid-points of the radial faces), volumes[nr] (the
 * volume of a cell of each radial row, (r+^2 - r-^2)/2 dtheta dz), z_centres[nz] (zero
 * in 2D).  Host arrays, each may be NULL; EINVAL on a null context. */
rb_status rb_get_geometry(rb_ctx* ctx, double* r_faces, double* r_centres, double* volumes,
                          double* z_centres);

/* CFL time step of the current state (Sect. 2.5), computed on the device. */
rb_status rb_cfl_dt(rb_ctx* ctx, double* dt);

/* For callers that cannot allocate device memory or synchronise with the host (code
 * under stream capture, tight serving loops): the CFL time step of any state of the
 * context's layout (device pointer `state`, not modified) into the device double *dt_dev,
 * or 0.0 there when the state has a cell with a non-positive density or pressure.  The
 * same kernels as rb_cfl_dt; their partials live in a static device array of 4,136
 * doubles (33 KB: the control block, the step, 2 x 2,048 block partials) that each device
 * holds until the process ends.  The CFL kernel strides over the cells with at most 2,048
 * blocks, so every grid fits; a context whose launch would need more partials is refused
 * with RB_EINVAL.  No allocation and no host synchronisation: the result is ready when the
 * context's stream reaches it; errors of the launches themselves return RB_EDEVICE.  The
 * array keeps the last call's contents and its control block is cleared at the start of
 * every call.  Every call on a device shares that device's array: calls that overlap on
 * one device (two streams, two threads) race. */
rb_status rb_cfl_dt_static(rb_ctx* ctx, const void* state, double* dt_dev);

/* Counters, time, masses (fixed-tree FP64 sums) and the last boundary outflow. */
rb_status rb_diagnostics(rb_ctx* ctx, rb_diag* out);

/* Kernel timers.  With enable != 0, rb_step brackets every launch of the stage
 * kernels (gas, dust) and of the reductions with HIP events recorded on the context's
 * stream and accumulates their elapsed times.  rb_profile_read fills, per kernel kind
 * (0 gas stage kernel, 1 dust stage kernel, 2 reductions and CFL), the total
 * milliseconds and the number of launches since profiling was enabled (3 entries
 * each).  Enabling resets the totals. */
rb_status rb_profile(rb_ctx* ctx, int enable);
rb_status rb_profile_read(rb_ctx* ctx, double* total_ms, int64_t* launches);

/* ---- discrete adjoint (FP64 precision only) --------------------------------------
 *
 * The adjoint of n RK2 steps is taken in two calls.  rb_record advances n steps like
 * rb_step (same dt policies) and keeps a checkpoint of the state every ckpt_every steps
 * and the time steps used.  rb_adjoint then sweeps backwards: for each checkpoint
 * segment it recomputes the segment's states E^m and midpoints E* with the stage
 * kernels and applies the transposed stage Jacobians (Sect. 2.5: E* = E^m + dt/(2V)
 * (G(E^m) - R0), E^{m+1} = E^m + dt/V (G(E*) - R0)), the face fluxes differentiated on
 * the branches the primal solves took (Riemann wave pattern, limiter, fallbacks) and
 * p* by implicit differentiation of the pressure-function equation (Sect. 2.6).  The
 * time steps are held fixed (the recorded ones).
 *
 * Workspace: caller-owned device memory of the size rb_adjoint_workspace returns
 * (two state-sized vectors, ceil(n / ckpt_every) checkpoints, 2 ckpt_every - 1 segment
 * states, Stokes partials); it must stay untouched between rb_record and rb_adjoint.
 * Device vectors lambda_final and grad_state0 are FP64 fields in the layout of
 * rb_get_fields ([field][k][i][j]); a gradient with respect to the full state equals
 * the one with respect to the stored deviation.  Errors: RB_EINVAL for the FP32
 * form, n < 1, ckpt_every < 1, a workspace that is too small, or rb_adjoint without a
 * matching rb_record; device errors as rb_step. */
rb_status rb_adjoint_workspace(const rb_ctx* ctx, int n, int ckpt_every, size_t* bytes);

/* Advances n steps from the current state (as rb_step) and records checkpoints and time
 * steps in the workspace.  dt_out (host, n entries, may be NULL) receives the steps. */
rb_status rb_record(rb_ctx* ctx, int n, int ckpt_every, const rb_dt_policy* policy,
                    double* dt_out, void* workspace, size_t workspace_bytes);

/* Reverse sweep over the recorded steps.  lambda_final: dJ/dE after the n steps;
 * grad_state0 receives dJ/dE before them; grad_stokes (host, n_dust entries, may be
 * NULL) receives dJ/dSt of each dust species (constant-Stokes drag, Sect. 2.9).  The
 * context's state is left at the end of the recorded steps. */
rb_status rb_adjoint(rb_ctx* ctx, const void* lambda_final, void* grad_state0,
                     double* grad_stokes, void* workspace, size_t workspace_bytes);

/* Contracts a state cotangent lam (device, layout of rb_get_fields) with the derivative
 * of the initial disc state with respect to the per-cell vortex amplitude: out[cell] =
 * sum_f lam[f][cell] dE_f/dA(cell).  noise ((1 + n_dust) x ncells) and amp (ncells),
 * host arrays that may be NULL, must be those given to rb_init_state; out is a device
 * array of ncells doubles. */
rb_status rb_amp_gradient(rb_ctx* ctx, const double* noise, const double* amp, const void* lam,
                          void* out);

/* Message describing the last error on ctx; valid until the next call on ctx. */
const char* rb_last_error(const rb_ctx* ctx);

/* Releases the host-side context (the caller frees its device buffers). */
void rb_destroy(rb_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* ROSSBI_MI355X_H */
