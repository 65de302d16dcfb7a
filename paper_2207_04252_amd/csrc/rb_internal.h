// Internal definitions shared by the device kernels and the host runtime of the
// bi-fluid finite-volume library (work-area layout, kernel argument blocks, flags).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "rossbi_mi355x.h"

namespace rb {

// Tiles: 64 cells along theta (one wavefront per radial row) x TI rows in r, marching
// through a chunk of z planes; TM rows for the stage kernel (RB_TM at build time), TI for
// the in-plane adjoint kernel.
constexpr int TJ = 64;
constexpr int TI = 8;
constexpr int NT = TJ * TI;
#ifndef RB_TM
#define RB_TM 8
#endif
constexpr int TM = RB_TM;
#ifndef RB_WPE
#define RB_WPE 2
#endif
constexpr int WPE = RB_WPE;  // stage-kernel waves per SIMD the register budget is set for
constexpr int NTM = TJ * TM;
static_assert(TM == 4 || TM == 8, "stage-kernel tiles of 4 or 8 rows");
constexpr int MAXF = 21;
constexpr int DTLOG = 4096;  // device dt log entries per rb_step chunk

enum : int { FL_NEG = 1, FL_VAC = 2, FL_NOCONV = 4, FL_STIFF = 8 };
constexpr int FL_HARD = FL_NEG | FL_NOCONV | FL_STIFF;

// per-radial-row table entries (interior rows)
enum { RT_V = 0, RT_INVV, RT_ATH, RT_AZ, RT_INVRC, RT_OMK, RT_MAXA, RT_RC, RT_N };
// reconstruction coefficients of a cell along r: increment to the upper face is
// minmod(wpm*dm + wpp*dp, lpm*dm, lpp*dp), to the lower face
// minmod(wmm*dm + wmp*dp, lmm*dm, lmp*dp), dm/dp the backward/forward differences.
enum { RC_WPM = 0, RC_WPP, RC_LPM, RC_LPP, RC_WMM, RC_WMP, RC_LMM, RC_LMP, RC_N };
// primitive variables of the stationary flow at a cell centre or face centre (the
// reference of the reconstructed gas deviation W' = W(E) - W(E0)): velocity (r, theta, z),
// pressure and density in the slots of the gas fields, then the adiabatic sound speed,
// the total enthalpy per volume E + P and 1/rho.  All zero where the split has no
// reference (the Sod annulus).
enum { WB_U = 0, WB_V, WB_W, WB_P, WB_RHO, WB_C, WB_H, WB_IRHO, WB_N };

// Device control block at the start of the work area.
struct Ctrl {
  int status;
  int bad_step;
  int maxit;
  int pad0;
  unsigned long long first_bad;
  unsigned long long nfall;
  unsigned long long nvac;
  unsigned long long nresolve;  // FP32-perturbation faces re-solved in FP64
  double min_ts;          // smallest dust stopping time (init)
  double outflow[5];      // boundary mass outflow of the last second stage
  unsigned long long newton_hist[8];  // gas Newton solves by iteration count (7: >= 7)
  unsigned long long nnegd;           // dust densities negative at the end of a step
};

// Offsets (in doubles) of the tables inside the work area.
struct Layout {
  size_t ctrl, rt, ar, rco, rcell, rface, zc, bgc, bgr, bgz, wc, wr, wz, r0, grav, ghr, ghrw, ghz, ghzw;
  size_t trig, indw, indab, indp, damp, ozr, dtlog, cflp, outp, tsp, red, total;
  int nind;      // blocks of the indirect-gravity sums
  int nblocks;   // stage-kernel blocks
  int ntj, nti, nkc, tk;
  int ntm;       // stage-kernel tiles in r (TM rows each)
  int nblocks_adj;  // in-plane adjoint kernel blocks (TI-row tiles)
  int ncfl;      // blocks of the standalone CFL / conversion kernels
};

struct Geo {
  int nr, nth, nz, twod, nd, nf;
  int p32;       // state stored as FP32 perturbation (gas) / FP32 dust velocities
  int indirect;  // indirect gravity of the displaced star
  int drag_law;  // 0 constant Stokes number, 1 Epstein / Stokes regimes
  int bc_z;      // 0 stationary z ghosts, 1 outflow (ghosts repeat the boundary cell), 2 damped
  int damp;      // boundary damping zones present (rate table)
  int newton_max;  // Newton iteration cap of the exact gas solver
  int drag_exact;  // drag split off the stages and integrated exactly (dust present)
  size_t N;
  double gamma, GM, cfl;
  double inv_st[4];
  double inv_mp[4];  // 1 / (grain density x grain radius)   (drag law 1)
  double rp94[4];    // 4 grain radius / 9                    (drag law 1)
  double mfp;        // mean-free-path constant: lambda = mfp / rho_gas
};

struct Tables {
  const double* rt;
  const double* ar;
  const double* rco;
  const double* bgc;
  const double* bgr;
  const double* bgz;
  const double* wc;    // stationary-flow primitives [k][i][WB_N] at cell centres
  const double* wr;    //   at r faces [k][i + 1/2][WB_N]
  const double* wz;    //   at z faces [k + 1/2][i][WB_N]
  const double* r0;
  const double* grav;
  const double* ghr;   // reconstructed variables of the r ghosts [side][layer][k][nf]
  const double* ghrw;  // their stationary-flow primitives [side][layer][k][WB_N]
  const double* ghz;   // reconstructed variables of the z ghosts [side][layer][i][nf]
  const double* ghzw;  // their stationary-flow primitives [side][layer][i][WB_N]
  const double* trig;  // cos, sin of the theta cell centres [2][ntheta]
  const double* indw;  // V r / (r^2 + z^2)^(3/2) per (k, i) (indirect-gravity sums)
  const double* indab; // the indirect-gravity sums A, B of the current stage input
  const double* damp;  // boundary-zone relaxation rate R / tau per (k, i), 0 outside
  const double* ozr;   // outflow z ghosts: rho0(ghost) / rho0(boundary cell) [side][layer][i]
};

struct Ctl {
  Ctrl* ctrl;
  double* dtlog;
  double* cflp;
  double* outp;
  double* tsp;   // per-block smallest stopping time of a state (drag law 1)
  double* r0w;   // writable residual table (empty run)
};

enum : int { MODE_UPDATE = 0, MODE_RESID = 1, MODE_OPER = 2 };

struct StageArgs {
  Geo g;
  Tables t;
  Ctl c;
  const void* in;       // state whose operator is evaluated (stencil source)
  const void* base;     // E^n, base of the update
  void* out;            // updated state (or operator output, FP64)
  double coef;          // 1/2 for the first stage, 1 for the second
  int dt_idx;           // dtlog entry holding this step's dt
  int mode;
  int gas_only;         // empty run: gas without drag
  int second;           // second stage: CFL partials, ledger, checks
  int step;             // global step index (error reporting)
  int tk, ntj, nti, nkc;
  int ntm;              // stage-kernel tiles in r (rows of TM)
};

struct InitArgs {
  Geo g;
  rb_config cfg;
  double* work;
  Layout L;
  const double* noise;  // device, may be null
  const double* amp;    // device, may be null
  void* state;
};

// Vector-Jacobian product of one stage update E_out = base + c dt V^-1 (G(E) - R0):
// out = base1 + base2 + (dE_out/dE)^T-part of G, i.e. out = base1 + base2 + J_G(E)^T w with
// w = cw V^-1 cot (cot the cotangent of E_out).  FP64 state layout.
struct AdjArgs {
  StageArgs s;          // geometry and tables; s.in = E, the state the operator is taken at
  const double* cot;    // cotangent of the stage output
  const double* base1;  // added to out, may be null
  const double* base2;  // added to out, may be null
  double* out;
  double cw;            // stage coefficient x dt
  double* stpart;       // per-block Stokes-number partials (dust groups)
  int tk, nkc;          // z chunking of the adjoint launch
};

// launchers (rb_kernels.hip)
hipError_t launch_tables(const InitArgs& a, hipStream_t s);
hipError_t launch_init_state(const InitArgs& a, hipStream_t s);
hipError_t launch_stage(const StageArgs& a, int blocks, hipStream_t s);
// one group of a stage: 0 the gas, 1 + s dust species s
hipError_t launch_stage_group(const StageArgs& a, int blocks, int group, hipStream_t s);
hipError_t launch_cfl(const StageArgs& a, const void* state, int blocks, int dt_idx, hipStream_t s);
hipError_t launch_drag(const StageArgs& a, void* state, double frac, int blocks, hipStream_t s);
hipError_t launch_reduce(const StageArgs& a, int nparts, int dt_idx_next, int want_dt,
                         int want_ledger, hipStream_t s);
hipError_t launch_fill(double* p, size_t n, double v, hipStream_t s);
hipError_t launch_ctrl_init(Ctrl* c, hipStream_t s);
hipError_t launch_cfl_out(const Ctrl* c, const double* dt, double* out, hipStream_t s);
hipError_t launch_to_full(const StageArgs& a, const void* state, double* out, int f,
                          hipStream_t s);
hipError_t launch_from_full(const StageArgs& a, const double* in, void* state, int f,
                            hipStream_t s);
hipError_t launch_mass(const StageArgs& a, const void* state, double* partials, int f,
                       int blocks, hipStream_t s);
hipError_t launch_sum(const double* partials, int n, double* out, hipStream_t s);
// indirect-gravity sums A, B of a state into the table (fixed-order partial sums)
hipError_t launch_indirect(const StageArgs& a, const void* state, double* partials, int blocks,
                           double* ab, hipStream_t s);
// d(initial state)/d(vortex amplitude) contracted with a state cotangent, per cell
hipError_t launch_amp_grad(const InitArgs& a, const double* lam, double* out, hipStream_t s);

// launchers (rb_adjoint.hip)
hipError_t launch_adj_group(const AdjArgs& a, int blocks, int group, hipStream_t s);
// acc[species] += sum of the per-block Stokes partials (one block, fixed order)
hipError_t launch_st_accum(const double* parts, int nblocks, double* acc, hipStream_t s);

}  // namespace rb
