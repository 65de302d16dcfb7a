// Host runtime behind the C ABI of include/rossbi_mi355x.h: validation, work-area
// layout, the initialisation sequence (tables, empty run, initial state) and the step
// loop.  Every computation runs in the device kernels of rb_kernels.hip; this file
// only sequences launches on the caller's stream and moves data at the boundary.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "rb_internal.h"

using namespace rb;

struct rb_ctx {
  rb_config cfg;
  Geo g;
  Layout L;
  hipStream_t stream;
  void* state;
  void* stage;
  double* work;
  double t;
  int64_t step;
  double dt_last;
  int hard;       // sticky rb_status of a hard error, 0 if none
  std::string err;
  // kernel timers (rb_profile): events bracketing launches within one rb_step chunk
  int prof = 0;
  std::vector<hipEvent_t> ev;
  std::vector<int> ev_kind;
  size_t ev_used = 0;
  double prof_ms[3] = {0, 0, 0};
  int64_t prof_n[3] = {0, 0, 0};
  // recorded run for the adjoint (rb_record)
  int rec_n = 0, rec_k = 0;
  std::vector<double> rec_dts;
  void* rec_ws = nullptr;
  int device = 0;  // the device current at rb_init_state
};

namespace {

size_t up32(size_t x) { return (x + 31) / 32 * 32; }

// Scratch of rb_cfl_dt_static: a control block, the reduced step and the per-block CFL and
// stopping-time partials (at most SCRATCH_PARTS blocks), in one file-scope device array.
// Each device holds its own copy until the process ends; every call on a device shares it.
constexpr size_t SCRATCH_CTRL = 32, SCRATCH_DT = 8, SCRATCH_PARTS = 2048;
constexpr size_t SCRATCH_DOUBLES = SCRATCH_CTRL + SCRATCH_DT + 2 * SCRATCH_PARTS;
static_assert(sizeof(Ctrl) <= SCRATCH_CTRL * sizeof(double), "control block fits the scratch");
__device__ __align__(256) double scratch[SCRATCH_DOUBLES];
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[MAX_DEVICES] = {};

// The device address of `scratch` on the current device (the array's name in host code is
// a host-side stand-in, not that address), taken once per device.
bool scratch_setup(int dev) {
  if (dev < 0 || dev >= MAX_DEVICES) return false;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_dev[dev]) return true;
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return false;
  g_scratch_dev[dev] = (double*)p;
  return true;
}
double* scratch_of(int dev) {
  if (dev < 0 || dev >= MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_dev[dev];
}

bool validate(const rb_config* c, std::string* why) {
  auto bad = [&](const char* m) { if (why) *why = m; return false; };
  if (!c) return bad("null config");
  if (c->nr < 3 || c->ntheta < 4 || c->nz < 1) return bad("grid too small (nr >= 3, ntheta >= 4)");
  if (c->nz == 2 || c->nz == 3) return bad("nz must be 1 (2D) or >= 4");
  if ((double)c->nr * c->ntheta * c->nz > 4.0e9) return bad("grid too large");
  if (c->n_dust < 0 || c->n_dust > 4) return bad("n_dust must be 0..4");
  if (!(c->gamma > 1.0)) return bad("gamma must exceed 1");
  if (!(c->cfl > 0.0 && c->cfl <= 1.0)) return bad("cfl must be in (0, 1]");
  if (c->newton_max_iter < 0) return bad("newton_max_iter must be >= 0 (0: the default 50)");
  if (c->drag_exact != 0 && c->drag_exact != 1) return bad("drag_exact must be 0 or 1");
  if (!(c->r_in > 0.0 && c->r_out > c->r_in)) return bad("need 0 < r_in < r_out");
  if (c->nz > 1 && !(c->z_half > 0.0)) return bad("z_half must be positive in 3D");
  if (c->init_kind != RB_INIT_SOD && c->init_kind != RB_INIT_DISC) return bad("unknown init_kind");
  if (c->init_kind == RB_INIT_DISC && !(c->GM > 0.0)) return bad("disc needs GM > 0");
  if (c->init_kind == RB_INIT_SOD && c->n_dust > 0) return bad("Sod annulus carries no dust");
  if (c->drag_law != 0 && c->drag_law != 1) return bad("drag_law must be 0 or 1");
  if (c->n_dust > 0 && c->drag_law == 0 && !(c->GM > 0.0))
    return bad("dust drag needs GM > 0 (t_s = St/Omega_K)");
  if (c->n_dust > 0 && c->drag_law == 1) {
    if (!(c->mfp_coef > 0.0)) return bad("drag law 1 needs mfp_coef > 0");
    for (int s = 0; s < c->n_dust; ++s)
      if (!(c->grain_size[s] > 0.0) || !(c->grain_density[s] > 0.0))
        return bad("drag law 1 needs positive grain sizes and densities");
  }
  if (c->indirect && c->init_kind != RB_INIT_DISC) return bad("indirect gravity needs a disc");
  if (c->bc_r < 0 || c->bc_r > 1 || c->bc_z < 0 || c->bc_z > 2) return bad("bc_r must be 0..1, bc_z 0..2");
  if ((c->rwi_delta != 0.0 || c->rwi_eps != 0.0) &&
      (c->init_kind != RB_INIT_DISC || !(c->rwi_dr > 0.0) || !(c->rwi_delta > -1.0) || c->rwi_m < 0))
    return bad("the RWI seed needs a disc, rwi_dr > 0, rwi_delta > -1 and rwi_m >= 0");
  if ((c->bc_r || c->bc_z) && c->init_kind != RB_INIT_DISC) return bad("boundary options need a disc");
  if ((c->bc_r == 1 || c->bc_z == 2) &&
      (!(c->damp_tau > 0.0) || !(c->damp_r_in > 1.0) || !(c->damp_r_out > 0.0 && c->damp_r_out < 1.0) ||
       !(c->damp_z > 0.0 && c->damp_z < 1.0)))
    return bad("damping zones need damp_tau > 0, damp_r_in > 1, 0 < damp_r_out < 1, 0 < damp_z < 1");
  for (int s = 0; s < c->n_dust; ++s)
    if ((c->drag_law == 0 && !(c->stokes[s] > 0.0)) || !(c->hd_over_h[s] > 0.0) ||
        !(c->eps_dust[s] >= 0.0))
      return bad("dust parameters must be positive");
  if (c->precision != RB_FP64 && c->precision != RB_FP32_PERT) return bad("unknown precision");
  if (c->precision == RB_FP32_PERT && c->init_kind != RB_INIT_DISC)
    return bad("the FP32-perturbation form needs a disc background");
  if (c->precision == RB_FP32_PERT && c->gamma != 1.4)
    return bad("the FP32-perturbation form is specialised to gamma = 7/5");
  return true;
}

Layout make_layout(const rb_config& c) {
  Layout L;
  const size_t nr = c.nr, nth = c.ntheta, nz = c.nz, nf = 5 + 4 * c.n_dust;
  const size_t N = nr * nth * nz;
  L.ntj = (int)((nth + TJ - 1) / TJ);
  L.nti = (int)((nr + TI - 1) / TI);
  L.ntm = (int)((nr + TM - 1) / TM);
  if (nz == 1) {
    L.tk = 1;
  } else {
    int tk = 2;
    const char* env = std::getenv("RB_TK");
    if (env && std::atoi(env) > 0) {
      tk = std::min(std::atoi(env), 4096);  // the Newton histogram's 16-bit bins
    } else {
      // A stage-kernel workgroup of 64 x TM threads holds at most 256 VGPRs per lane (two
      // waves per SIMD), so 8 / TM workgroups fill a CU and a launch runs in
      // ceil(blocks / (256 * 8 / TM)) rounds on the 256 CUs of an MI355X; a block marches
      // tk planes plus about 1.5 planes of set-up (initial ring, first z face).  Take the
      // chunk length with the fewest plane-times.
      const size_t tiles = (size_t)L.ntj * L.ntm;
      const size_t conc = 256 * (8 / TM);
      const int cand[7] = {128, 64, 32, 16, 8, 4, 2};
      double best = 1e300;
      for (int q = 0; q < 7; ++q) {
        const size_t c = std::min<size_t>(cand[q], nz);
        const size_t blocks = tiles * ((nz + c - 1) / c);
        const double t = (double)((blocks + conc - 1) / conc) * ((double)c + 1.5);
        if (t < best) { best = t; tk = (int)c; }
      }
    }
    L.tk = (int)std::min<size_t>(tk, nz);
  }
  L.nkc = (int)((nz + L.tk - 1) / L.tk);
  L.nblocks = L.ntj * L.ntm * L.nkc;
  L.nblocks_adj = L.ntj * L.nti * L.nkc;
  L.ncfl = (int)std::min<size_t>((N + 255) / 256, 2048);
  size_t o = 0;
  auto take = [&](size_t n) { size_t at = o; o += up32(n); return at; };
  L.ctrl = take((sizeof(Ctrl) + 7) / 8);
  L.rt = take(nr * RT_N);
  L.ar = take(nr + 1);
  L.rco = take((nr + 2) * RC_N);
  L.rcell = take(nr + 4);
  L.rface = take(nr + 1);
  L.zc = take(nz);
  L.bgc = take(nz * nr * 5);
  L.bgr = take(nz * (nr + 1) * 5);
  L.bgz = take((nz + 1) * nr * 5);
  L.wc = take(nz * nr * WB_N);
  L.wr = take(nz * (nr + 1) * WB_N);
  L.wz = take((nz + 1) * nr * WB_N);
  L.r0 = take(nz * nr * 5);
  L.grav = take(nz * nr * 2);
  L.ghr = take(4 * nz * nf);
  L.ghrw = take(4 * nz * WB_N);
  L.ghz = take(4 * nr * nf);
  L.ghzw = take(4 * nr * WB_N);
  L.trig = take(2 * nth);
  L.indw = take(nz * nr);
  L.indab = take(2);
  L.nind = (int)std::min<size_t>((N + 255) / 256, 1024);
  L.indp = take((size_t)L.nind * 2);
  L.damp = take(nz * nr);
  L.ozr = take(4 * nr);
  L.dtlog = take(DTLOG + 2);
  L.cflp = take(std::max((size_t)L.nblocks * 5, (size_t)L.ncfl));
  L.outp = take((size_t)L.nblocks * 5);
  L.tsp = take(std::max((size_t)L.nblocks, (size_t)L.ncfl));
  L.red = take(2048 + 16);
  L.total = o;
  return L;
}

Geo make_geo(const rb_config& c) {
  Geo g;
  g.nr = c.nr; g.nth = c.ntheta; g.nz = c.nz;
  g.twod = c.nz == 1;
  g.nd = c.n_dust;
  g.nf = 5 + 4 * c.n_dust;
  g.N = (size_t)c.nr * c.ntheta * c.nz;
  g.gamma = c.gamma; g.GM = c.GM; g.cfl = c.cfl;
  g.p32 = c.precision == RB_FP32_PERT;
  g.indirect = c.indirect != 0;
  g.drag_law = c.drag_law;
  g.newton_max = c.newton_max_iter > 0 ? c.newton_max_iter : 50;
  g.drag_exact = (c.drag_exact && c.n_dust > 0) ? 1 : 0;
  g.bc_z = c.nz > 1 ? c.bc_z : 0;
  g.damp = c.bc_r == 1 || (c.bc_z == 2 && c.nz > 1);
  g.mfp = c.drag_law ? c.mfp_coef : 0.0;
  for (int s = 0; s < 4; ++s) {
    const bool on = s < c.n_dust;
    g.inv_st[s] = on && c.drag_law == 0 ? 1.0 / c.stokes[s] : 0.0;
    g.inv_mp[s] = on && c.drag_law ? 1.0 / (c.grain_density[s] * c.grain_size[s]) : 0.0;
    g.rp94[s] = on && c.drag_law ? 4.0 * c.grain_size[s] / 9.0 : 0.0;
  }
  return g;
}

StageArgs base_args(rb_ctx* x) {
  StageArgs a;
  std::memset(&a, 0, sizeof(a));
  a.g = x->g;
  const Layout& L = x->L;
  double* w = x->work;
  a.t.rt = w + L.rt; a.t.ar = w + L.ar; a.t.rco = w + L.rco; a.t.bgc = w + L.bgc;
  a.t.bgr = w + L.bgr; a.t.bgz = w + L.bgz; a.t.r0 = w + L.r0; a.t.grav = w + L.grav;
  a.t.wc = w + L.wc; a.t.wr = w + L.wr; a.t.wz = w + L.wz;
  a.t.ghr = w + L.ghr; a.t.ghrw = w + L.ghrw; a.t.ghz = w + L.ghz; a.t.ghzw = w + L.ghzw;
  a.t.trig = w + L.trig; a.t.indw = w + L.indw; a.t.indab = w + L.indab;
  a.t.damp = w + L.damp;
  a.t.ozr = w + L.ozr;
  a.c.ctrl = reinterpret_cast<Ctrl*>(w + L.ctrl);
  a.c.dtlog = w + L.dtlog; a.c.cflp = w + L.cflp; a.c.outp = w + L.outp; a.c.r0w = w + L.r0;
  a.c.tsp = w + L.tsp;
  a.tk = L.tk; a.ntj = L.ntj; a.nti = L.nti; a.nkc = L.nkc; a.ntm = L.ntm;
  a.dt_idx = -1;
  return a;
}

rb_status fail(rb_ctx* x, rb_status s, const std::string& m) {
  if (x) x->err = m;
  return s;
}

rb_status hip_fail(rb_ctx* x, hipError_t e, const char* where) {
  std::string m = std::string(where) + ": " + hipGetErrorString(e);
  return fail(x, RB_EDEVICE, m);
}

#define HIPCHK(x, expr, where)                       \
  do {                                              \
    hipError_t e_ = (expr);                         \
    if (e_ != hipSuccess) return hip_fail(x, e_, where); \
  } while (0)

rb_status reset_ctrl(rb_ctx* x) {
  Ctrl c;
  std::memset(&c, 0, sizeof(c));
  c.bad_step = -1;
  c.first_bad = ~0ull;
  // keep the stopping time computed by the table kernel
  Ctrl old;
  HIPCHK(x, hipMemcpyAsync(&old, x->work + x->L.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, x->stream),
         "read control block");
  HIPCHK(x, hipStreamSynchronize(x->stream), "sync");
  c.min_ts = old.min_ts;
  HIPCHK(x, hipMemcpyAsync(x->work + x->L.ctrl, &c, sizeof(Ctrl), hipMemcpyHostToDevice, x->stream),
         "write control block");
  HIPCHK(x, hipStreamSynchronize(x->stream), "sync");
  return RB_OK;
}

// event pair around one launch of kernel kind `kind` (no-op unless profiling)
struct ProfScope {
  rb_ctx* x;
  int kind;
  size_t slot;
  ProfScope(rb_ctx* x_, int kind_) : x(x_), kind(kind_), slot(0) {
    if (!x->prof) return;
    if (x->ev_used + 2 > x->ev.size()) {
      for (int q = 0; q < 64; ++q) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return;
        x->ev.push_back(e);
      }
      x->ev_kind.resize(x->ev.size() / 2);
    }
    slot = x->ev_used;
    x->ev_used += 2;
    x->ev_kind[slot / 2] = kind;
    (void)hipEventRecord(x->ev[slot], x->stream);
  }
  ~ProfScope() {
    if (x->prof && slot + 1 < x->ev.size()) (void)hipEventRecord(x->ev[slot + 1], x->stream);
  }
};

// accumulate the recorded event pairs (stream already synchronised)
void prof_collect(rb_ctx* x) {
  if (!x->prof) return;
  for (size_t p = 0; p + 1 < x->ev_used; p += 2) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, x->ev[p], x->ev[p + 1]) == hipSuccess) {
      int k = x->ev_kind[p / 2];
      x->prof_ms[k] += ms;
      x->prof_n[k] += 1;
    }
  }
  x->ev_used = 0;
}

// indirect-gravity sums of the stage input (before any group kernel of the stage)
hipError_t prep_stage(rb_ctx* x, const StageArgs& a) {
  if (!x->g.indirect || a.mode == MODE_RESID) return hipSuccess;
  ProfScope ps(x, 2);
  return launch_indirect(a, a.in, x->work + x->L.indp, x->L.nind, x->work + x->L.indab, x->stream);
}

hipError_t run_stage(rb_ctx* x, const StageArgs& a) {
  hipError_t e = prep_stage(x, a);
  if (e != hipSuccess) return e;
  {
    ProfScope ps(x, 0);
    e = launch_stage_group(a, x->L.nblocks, 0, x->stream);
  }
  if (e != hipSuccess || a.gas_only) return e;
  for (int s = 0; s < x->g.nd; ++s) {
    ProfScope ps(x, 1);
    e = launch_stage_group(a, x->L.nblocks, 1 + s, x->stream);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

rb_status status_of_flags(int flags) {
  if (flags & FL_NEG) return RB_ENEGATIVE;
  if (flags & FL_NOCONV) return RB_ENOCONV;
  if (flags & FL_STIFF) return RB_ESTIFF;
  if (flags & FL_VAC) return RB_EVACUUM;
  return RB_OK;
}

}  // namespace

extern "C" {

rb_status rb_query_sizes(const rb_config* cfg, rb_buffers* sizes) {
  if (!cfg || !sizes) return RB_EINVAL;
  std::string why;
  if (!validate(cfg, &why)) return RB_EINVAL;
  const size_t N = (size_t)cfg->nr * cfg->ntheta * cfg->nz;
  const size_t nf = 5 + 4 * cfg->n_dust;
  Layout L = make_layout(*cfg);
  size_t bytes = nf * N * 8;
  if (cfg->precision == RB_FP32_PERT) {
    // gas deviation + dust momenta in FP32 (padded to 256 B), dust densities in FP64
    const size_t nf32 = 5 + 3 * (size_t)cfg->n_dust;
    bytes = (nf32 * N + 63) / 64 * 64 * 4 + (size_t)cfg->n_dust * N * 8;
  }
  sizes->state_bytes = bytes;
  sizes->stage_bytes = bytes;
  sizes->work_bytes = L.total * sizeof(double);
  return RB_OK;
}

rb_status rb_init_state(const rb_config* cfg, const rb_buffers* bufs, const double* noise,
                        const double* amp, void* stream, rb_ctx** out) {
  if (!out) return RB_EINVAL;
  *out = nullptr;
  if (!cfg || !bufs) return RB_EINVAL;
  std::string why;
  if (!validate(cfg, &why)) {
    std::fprintf(stderr, "rb_init_state: %s\n", why.c_str());
    return RB_EINVAL;
  }
  rb_buffers need;
  rb_query_sizes(cfg, &need);
  if (!bufs->state || !bufs->stage || !bufs->work) return RB_EINVAL;
  if (bufs->state_bytes < need.state_bytes || bufs->stage_bytes < need.stage_bytes ||
      bufs->work_bytes < need.work_bytes)
    return RB_ENOMEM;
  if (((uintptr_t)bufs->state | (uintptr_t)bufs->stage | (uintptr_t)bufs->work) & 255)
    return RB_EINVAL;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || !scratch_setup(dev)) return RB_EDEVICE;
  rb_ctx* x = new rb_ctx();
  x->device = dev;
  x->cfg = *cfg;
  x->g = make_geo(*cfg);
  x->L = make_layout(*cfg);
  x->stream = (hipStream_t)stream;
  x->state = bufs->state;
  x->stage = bufs->stage;
  x->work = (double*)bufs->work;
  x->t = 0.0;
  x->step = 0;
  x->dt_last = 0.0;
  x->hard = 0;
  auto bail = [&](rb_status s) { delete x; return s; };
  if (launch_fill(x->work, x->L.total, 0.0, x->stream) != hipSuccess) return bail(RB_EDEVICE);
  if (reset_ctrl(x) != RB_OK) return bail(RB_EDEVICE);

  InitArgs ia;
  std::memset(&ia, 0, sizeof(ia));
  ia.g = x->g;
  ia.cfg = *cfg;
  ia.work = x->work;
  ia.L = x->L;
  ia.state = x->state;
  if (launch_tables(ia, x->stream) != hipSuccess) return bail(RB_EDEVICE);

  // empty run (Sect. 2.8): the spatial operator of the stationary flow, by the step
  // kernel itself, written to the residual table.  The FP32-perturbation form forms
  // G(E) - G(E0) directly and needs no residual.
  if (cfg->balanced && !x->g.p32) {
    if (launch_fill((double*)x->stage, x->g.N * x->g.nf, 0.0, x->stream) != hipSuccess)
      return bail(RB_EDEVICE);
    StageArgs a = base_args(x);
    a.in = x->stage;
    a.base = x->stage;
    a.out = nullptr;
    a.mode = MODE_RESID;
    a.gas_only = 1;
    if (launch_stage(a, x->L.nblocks, x->stream) != hipSuccess) return bail(RB_EDEVICE);
  }
  // initial state: noise (one field per fluid) and amplitude fields staged through the
  // stage buffer, which holds at least (2 + n_dust) N doubles in either storage form
  const size_t N = x->g.N, NN = (size_t)(1 + x->g.nd) * N;
  if (noise) {
    if (hipMemcpyAsync(x->stage, noise, NN * sizeof(double), hipMemcpyHostToDevice, x->stream) !=
        hipSuccess)
      return bail(RB_EDEVICE);
    ia.noise = (const double*)x->stage;
  }
  if (amp) {
    if (hipMemcpyAsync((double*)x->stage + NN, amp, N * sizeof(double), hipMemcpyHostToDevice,
                       x->stream) != hipSuccess)
      return bail(RB_EDEVICE);
    ia.amp = (const double*)x->stage + NN;
  }
  if (launch_init_state(ia, x->stream) != hipSuccess) return bail(RB_EDEVICE);
  if (hipStreamSynchronize(x->stream) != hipSuccess) return bail(RB_EDEVICE);
  if (hipGetLastError() != hipSuccess) return bail(RB_EDEVICE);
  *out = x;
  return RB_OK;
}

rb_status rb_step(rb_ctx* x, int n, const rb_dt_policy* policy, double* dt_out) {
  if (!x || !policy || n < 0) return RB_EINVAL;
  if (x->hard) return fail(x, (rb_status)x->hard, "a hard error is pending; call rb_set_fields");
  if (policy->kind == RB_DT_FIXED && !(policy->dt > 0.0)) return fail(x, RB_EINVAL, "dt must be > 0");
  if (policy->kind == RB_DT_LIST && !policy->dt_list) return fail(x, RB_EINVAL, "dt_list is null");
  if (policy->kind < 0 || policy->kind > 2) return fail(x, RB_EINVAL, "unknown dt policy");
  const bool cfl = policy->kind == RB_DT_CFL;
  StageArgs a = base_args(x);
  double* dtlog = x->work + x->L.dtlog;
  std::vector<double> hd;
  int done = 0;
  while (done < n || (n == 0 && done == 0)) {
    const int m = std::min(n - done, DTLOG);
    if (!cfl) {
      hd.assign(m + 1, policy->dt);
      if (policy->kind == RB_DT_LIST) {
        for (int q = 0; q < m; ++q) {
          hd[q] = policy->dt_list[done + q];
          if (!(hd[q] > 0.0)) return fail(x, RB_EINVAL, "dt_list entries must be > 0");
        }
        hd[m] = m > 0 ? hd[m - 1] : policy->dt;
      }
      HIPCHK(x, hipMemcpyAsync(dtlog, hd.data(), (m + 1) * sizeof(double), hipMemcpyHostToDevice,
                               x->stream), "upload dt");
    }
    // start of the chunk: positivity check and CFL of the current state
    a.step = (int)(x->step);
    {
      ProfScope ps(x, 2);
      HIPCHK(x, launch_cfl(a, x->state, x->L.ncfl, 0, x->stream), "cfl");
      HIPCHK(x, launch_reduce(a, x->L.ncfl, 0, cfl ? 1 : 0, 0, x->stream), "reduce");
    }
    for (int q = 0; q < m; ++q) {
      a.step = (int)(x->step + q);
      a.dt_idx = q;
      a.mode = MODE_UPDATE;
      a.gas_only = 0;
      const bool split = x->g.drag_exact != 0;
      // split drag: the drag alone over dt/2 before the stages
      if (split) HIPCHK(x, launch_drag(a, x->state, 0.5, x->L.ncfl, x->stream), "drag");
      // first stage: E* = E^n + (dt/2V) (G(E^n) - R0)
      a.in = x->state; a.base = x->state; a.out = x->stage; a.coef = 0.5; a.second = 0;
      HIPCHK(x, run_stage(x, a), "stage 1");
      // second stage: E^{n+1} = E^n + (dt/V) (G(E*) - R0), in place
      a.in = x->stage; a.base = x->state; a.out = x->state; a.coef = 1.0; a.second = 1;
      HIPCHK(x, run_stage(x, a), "stage 2");
      if (split) {
        // boundary ledger of the stages, then the drag alone over dt/2 and the CFL step of
        // the relaxed state (which replaces the one the second stage formed)
        ProfScope ps(x, 2);
        HIPCHK(x, launch_reduce(a, x->L.nblocks, q + 1, 0, 1, x->stream), "ledger");
        HIPCHK(x, launch_drag(a, x->state, 0.5, x->L.ncfl, x->stream), "drag");
        a.step = (int)(x->step + q + 1);
        HIPCHK(x, launch_cfl(a, x->state, x->L.ncfl, 0, x->stream), "cfl");
        HIPCHK(x, launch_reduce(a, x->L.ncfl, q + 1, cfl ? 1 : 0, 0, x->stream), "reduce");
        a.step = (int)(x->step + q);
      } else {
        ProfScope ps(x, 2);
        HIPCHK(x, launch_reduce(a, x->L.nblocks, q + 1, cfl ? 1 : 0, 1, x->stream), "reduce");
      }
    }
    std::vector<double> got(m + 1);
    HIPCHK(x, hipMemcpyAsync(got.data(), dtlog, (m + 1) * sizeof(double), hipMemcpyDeviceToHost,
                             x->stream), "read dt");
    Ctrl c;
    HIPCHK(x, hipMemcpyAsync(&c, x->work + x->L.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, x->stream),
           "read control");
    HIPCHK(x, hipStreamSynchronize(x->stream), "sync");
    prof_collect(x);
    int completed = m;
    if (c.status & FL_HARD) {
      completed = std::max(0, std::min(m, c.bad_step - (int)x->step));
    }
    for (int q = 0; q < completed; ++q) {
      x->t += got[q];
      if (dt_out) dt_out[done + q] = got[q];
    }
    if (completed > 0) x->dt_last = got[completed - 1];
    x->step += completed;
    done += m;
    if (c.status & FL_HARD) {
      x->hard = status_of_flags(c.status & FL_HARD);
      char buf[160];
      std::snprintf(buf, sizeof(buf), "hard error flags 0x%x at step %d, first bad cell %llu",
                    c.status, c.bad_step, (unsigned long long)c.first_bad);
      return fail(x, (rb_status)x->hard, buf);
    }
    if (n == 0) break;
  }
  Ctrl c;
  HIPCHK(x, hipMemcpy(&c, x->work + x->L.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost), "read control");
  if (c.status & FL_VAC) return fail(x, RB_EVACUUM, "vacuum generated in a Riemann problem");
  return RB_OK;
}

rb_status rb_get_fields(rb_ctx* x, double* host_out, size_t n_doubles) {
  if (!x || !host_out) return RB_EINVAL;
  const size_t N = x->g.N;
  if (n_doubles != N * x->g.nf) return fail(x, RB_EINVAL, "n_doubles must be nfields * ncells");
  StageArgs a = base_args(x);
  for (int f = 0; f < x->g.nf; ++f) {
    HIPCHK(x, launch_to_full(a, x->state, (double*)x->stage, f, x->stream), "to_full");
    HIPCHK(x, hipMemcpyAsync(host_out + (size_t)f * N, x->stage, N * sizeof(double),
                             hipMemcpyDeviceToHost, x->stream), "copy out");
  }
  HIPCHK(x, hipStreamSynchronize(x->stream), "sync");
  return RB_OK;
}

rb_status rb_set_fields(rb_ctx* x, const double* host_in, size_t n_doubles) {
  if (!x || !host_in) return RB_EINVAL;
  const size_t N = x->g.N;
  if (n_doubles != N * x->g.nf) return fail(x, RB_EINVAL, "n_doubles must be nfields * ncells");
  StageArgs a = base_args(x);
  // each dust density before its momenta (the FP32 layout stores velocities against it)
  std::vector<int> order;
  for (int f = 0; f < 5; ++f) order.push_back(f);
  for (int s = 0; s < x->g.nd; ++s)
    for (int c : {3, 0, 1, 2}) order.push_back(5 + 4 * s + c);
  for (int f : order) {
    HIPCHK(x, hipMemcpyAsync(x->stage, host_in + (size_t)f * N, N * sizeof(double),
                             hipMemcpyHostToDevice, x->stream), "copy in");
    HIPCHK(x, launch_from_full(a, (const double*)x->stage, x->state, f, x->stream), "from_full");
  }
  HIPCHK(x, hipStreamSynchronize(x->stream), "sync");
  x->hard = 0;
  return reset_ctrl(x);
}

rb_status rb_eval_operator(rb_ctx* x, double* host_out, size_t n_doubles) {
  if (!x || !host_out) return RB_EINVAL;
  const size_t N = x->g.N;
  if (n_doubles != N * x->g.nf) return fail(x, RB_EINVAL, "n_doubles must be nfields * ncells");
  StageArgs a = base_args(x);
  a.in = x->state; a.base = x->state; a.out = x->stage; a.mode = MODE_OPER; a.gas_only = 0;
  HIPCHK(x, prep_stage(x, a), "indirect sums");
  HIPCHK(x, launch_stage(a, x->L.nblocks, x->stream), "operator");
  if (x->g.p32) {
    // FP32 form: the kernels write FP32; widened at the boundary
    std::vector<float> tmp(N * x->g.nf);
    HIPCHK(x, hipMemcpyAsync(tmp.data(), x->stage, tmp.size() * sizeof(float),
                             hipMemcpyDeviceToHost, x->stream), "copy out");
    HIPCHK(x, hipStreamSynchronize(x->stream), "sync");
    for (size_t q = 0; q < tmp.size(); ++q) host_out[q] = tmp[q];
    return RB_OK;
  }
  HIPCHK(x, hipMemcpyAsync(host_out, x->stage, N * x->g.nf * sizeof(double), hipMemcpyDeviceToHost,
                           x->stream), "copy out");
  HIPCHK(x, hipStreamSynchronize(x->stream), "sync");
  return RB_OK;
}

rb_status rb_get_residual(rb_ctx* x, double* host_out, size_t n_doubles) {
  if (!x || !host_out) return RB_EINVAL;
  const size_t n = (size_t)x->g.nz * x->g.nr * 5;
  if (n_doubles != n) return fail(x, RB_EINVAL, "n_doubles must be nz * nr * 5");
  if (x->g.p32) return fail(x, RB_EINVAL, "the FP32-perturbation form has no residual table");
  HIPCHK(x, hipMemcpyAsync(host_out, x->work + x->L.r0, n * sizeof(double), hipMemcpyDeviceToHost,
                           x->stream), "copy out");
  HIPCHK(x, hipStreamSynchronize(x->stream), "sync");
  return RB_OK;
}

rb_status rb_get_geometry(rb_ctx* x, double* r_faces, double* r_centres, double* volumes,
                          double* z_centres) {
  if (!x) return RB_EINVAL;
  const int nr = x->cfg.nr, nz = x->cfg.nz;
  std::vector<double> rt((size_t)nr * RT_N);
  HIPCHK(x, hipMemcpyAsync(rt.data(), x->work + x->L.rt, rt.size() * sizeof(double),
                           hipMemcpyDeviceToHost, x->stream), "copy radial table");
  if (r_faces)
    HIPCHK(x, hipMemcpyAsync(r_faces, x->work + x->L.rface, (nr + 1) * sizeof(double),
                             hipMemcpyDeviceToHost, x->stream), "copy faces");
  if (z_centres)
    HIPCHK(x, hipMemcpyAsync(z_centres, x->work + x->L.zc, nz * sizeof(double),
                             hipMemcpyDeviceToHost, x->stream), "copy z centres");
  HIPCHK(x, hipStreamSynchronize(x->stream), "sync");
  for (int i = 0; i < nr; ++i) {
    if (r_centres) r_centres[i] = rt[(size_t)i * RT_N + RT_RC];
    if (volumes) volumes[i] = rt[(size_t)i * RT_N + RT_V];
  }
  return RB_OK;
}

rb_status rb_cfl_dt_static(rb_ctx* x, const void* state, double* dt_dev) {
  if (!x || !state || !dt_dev) return RB_EINVAL;
  if ((size_t)x->L.ncfl > SCRATCH_PARTS)
    return fail(x, RB_EINVAL, "the state needs more CFL partials than the static scratch holds");
  double* s = scratch_of(x->device);
  if (!s) return fail(x, RB_EDEVICE, "no static scratch on the context's device");
  StageArgs a = base_args(x);
  a.step = 0;
  a.c.ctrl = reinterpret_cast<Ctrl*>(s);
  a.c.dtlog = s + SCRATCH_CTRL;
  a.c.cflp = s + SCRATCH_CTRL + SCRATCH_DT;
  a.c.tsp = a.c.cflp + SCRATCH_PARTS;
  HIPCHK(x, launch_ctrl_init(a.c.ctrl, x->stream), "scratch control block");
  HIPCHK(x, launch_cfl(a, state, x->L.ncfl, 0, x->stream), "cfl");
  HIPCHK(x, launch_reduce(a, x->L.ncfl, 0, 1, 0, x->stream), "reduce");
  HIPCHK(x, launch_cfl_out(a.c.ctrl, a.c.dtlog, dt_dev, x->stream), "cfl out");
  return RB_OK;
}

rb_status rb_cfl_dt(rb_ctx* x, double* dt) {
  if (!x || !dt) return RB_EINVAL;
  if (x->hard) return fail(x, (rb_status)x->hard, "a hard error is pending");
  StageArgs a = base_args(x);
  a.step = (int)x->step;
  HIPCHK(x, launch_cfl(a, x->state, x->L.ncfl, 0, x->stream), "cfl");
  HIPCHK(x, launch_reduce(a, x->L.ncfl, DTLOG + 1, 1, 0, x->stream), "reduce");
  HIPCHK(x, hipMemcpyAsync(dt, x->work + x->L.dtlog + DTLOG + 1, sizeof(double),
                           hipMemcpyDeviceToHost, x->stream), "copy out");
  Ctrl c;
  HIPCHK(x, hipMemcpyAsync(&c, x->work + x->L.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, x->stream),
         "read control");
  HIPCHK(x, hipStreamSynchronize(x->stream), "sync");
  if (c.status & FL_NEG) {
    x->hard = RB_ENEGATIVE;
    return fail(x, RB_ENEGATIVE, "negative density or pressure in the state");
  }
  return RB_OK;
}

rb_status rb_diagnostics(rb_ctx* x, rb_diag* out) {
  if (!x || !out) return RB_EINVAL;
  std::memset(out, 0, sizeof(*out));
  StageArgs a = base_args(x);
  double* red = x->work + x->L.red;
  const int nb = 2048;
  for (int s = 0; s <= x->g.nd; ++s) {
    const int f = s == 0 ? 4 : 5 + 4 * (s - 1) + 3;
    HIPCHK(x, launch_mass(a, x->state, red, f, nb, x->stream), "mass");
    HIPCHK(x, launch_sum(red, nb, red + nb + s, x->stream), "sum");
  }
  double ms[5] = {0, 0, 0, 0, 0};
  HIPCHK(x, hipMemcpyAsync(ms, red + nb, (x->g.nd + 1) * sizeof(double), hipMemcpyDeviceToHost,
                           x->stream), "copy");
  Ctrl c;
  HIPCHK(x, hipMemcpyAsync(&c, x->work + x->L.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, x->stream),
         "read control");
  HIPCHK(x, hipStreamSynchronize(x->stream), "sync");
  out->t = x->t;
  out->step = x->step;
  out->flags = c.status;
  out->first_bad_step = c.bad_step;
  out->first_bad_cell = c.first_bad == ~0ull ? -1 : (int64_t)c.first_bad;
  out->fallbacks = (int64_t)c.nfall;
  out->vacuum_faces = (int64_t)c.nvac;
  out->max_newton = c.maxit;
  for (int s = 0; s < 5; ++s) {
    out->mass[s] = ms[s];
    out->outflow[s] = c.outflow[s];
  }
  out->dt_last = x->dt_last;
  out->fp64_resolves = (int64_t)c.nresolve;
  for (int b = 0; b < 8; ++b) out->newton_hist[b] = (int64_t)c.newton_hist[b];
  out->negative_dust = (int64_t)c.nnegd;
  return RB_OK;
}

rb_status rb_profile(rb_ctx* x, int enable) {
  if (!x) return RB_EINVAL;
  x->prof = enable ? 1 : 0;
  x->ev_used = 0;
  for (int k = 0; k < 3; ++k) { x->prof_ms[k] = 0.0; x->prof_n[k] = 0; }
  return RB_OK;
}

rb_status rb_profile_read(rb_ctx* x, double* total_ms, int64_t* launches) {
  if (!x || !total_ms || !launches) return RB_EINVAL;
  for (int k = 0; k < 3; ++k) { total_ms[k] = x->prof_ms[k]; launches[k] = x->prof_n[k]; }
  return RB_OK;
}

}  // extern "C"

// ---- discrete adjoint ------------------------------------------------------------

namespace {

// workspace layout, in doubles, each part 256-byte aligned
struct AdjLayout {
  size_t S, lam, nu, ck, segE, segS, stp, sta, total;
  int nseg, nblocks, tk, nkc;
};

AdjLayout adj_layout(const rb_ctx* x, int n, int k) {
  AdjLayout A;
  const Layout& L = x->L;
  // the in-plane adjoint kernel uses the forward stage kernel's tiles and z chunks
  A.tk = L.tk;
  A.nkc = L.nkc;
  A.nblocks = L.nblocks_adj;
  A.S = (size_t)x->g.nf * x->g.N;
  A.nseg = (n + k - 1) / k;
  size_t o = 0;
  auto take = [&](size_t m) { size_t at = o; o += up32(m); return at; };
  A.lam = take(A.S);
  A.nu = take(A.S);
  A.ck = o; o += (size_t)A.nseg * up32(A.S);
  A.segE = o; o += (size_t)std::max(k - 1, 0) * up32(A.S);
  A.segS = o; o += (size_t)k * up32(A.S);
  A.stp = take(A.nblocks);
  A.sta = take(4);
  A.total = o;
  return A;
}

}  // namespace

extern "C" {

rb_status rb_adjoint_workspace(const rb_ctx* x, int n, int ckpt_every, size_t* bytes) {
  if (!x || !bytes || n < 1 || ckpt_every < 1) return RB_EINVAL;
  if (x->g.p32) return RB_EINVAL;
  *bytes = adj_layout(x, n, std::min(ckpt_every, n)).total * sizeof(double);
  return RB_OK;
}

rb_status rb_record(rb_ctx* x, int n, int ckpt_every, const rb_dt_policy* policy, double* dt_out,
                    void* ws, size_t ws_bytes) {
  if (!x || !policy || !ws || n < 1 || ckpt_every < 1) return RB_EINVAL;
  if (x->g.p32) return fail(x, RB_EINVAL, "the adjoint is FP64 only");
  if (x->g.indirect) return fail(x, RB_EINVAL, "the adjoint does not cover indirect gravity");
  if (x->g.drag_law) return fail(x, RB_EINVAL, "the adjoint covers the constant-Stokes drag only");
  if (x->g.drag_exact) return fail(x, RB_EINVAL, "the adjoint covers the explicit drag only");
  if (x->g.bc_z || x->g.damp) return fail(x, RB_EINVAL, "the adjoint covers the stationary ghosts only");
  const int k = std::min(ckpt_every, n);
  const AdjLayout A = adj_layout(x, n, k);
  if (ws_bytes < A.total * sizeof(double)) return fail(x, RB_EINVAL, "workspace too small");
  if (policy->kind == RB_DT_LIST && !policy->dt_list) return fail(x, RB_EINVAL, "dt_list is null");
  x->rec_n = 0;
  x->rec_ws = nullptr;
  x->rec_dts.assign(n, 0.0);
  double* w = (double*)ws;
  const size_t bytes = A.S * sizeof(double);
  for (int seg = 0; seg < A.nseg; ++seg) {
    const int m0 = seg * k, len = std::min(k, n - m0);
    HIPCHK(x, hipMemcpyAsync(w + A.ck + (size_t)seg * up32(A.S), x->state, bytes,
                             hipMemcpyDeviceToDevice, x->stream), "checkpoint");
    rb_dt_policy p = *policy;
    if (p.kind == RB_DT_LIST) p.dt_list = policy->dt_list + m0;
    const rb_status st = rb_step(x, len, &p, x->rec_dts.data() + m0);
    if (st != RB_OK) return st;
  }
  if (dt_out) std::memcpy(dt_out, x->rec_dts.data(), n * sizeof(double));
  x->rec_n = n;
  x->rec_k = k;
  x->rec_ws = ws;
  return RB_OK;
}

rb_status rb_adjoint(rb_ctx* x, const void* lambda_final, void* grad_state0, double* grad_stokes,
                     void* ws, size_t ws_bytes) {
  if (!x || !lambda_final || !grad_state0 || !ws) return RB_EINVAL;
  if (x->g.p32) return fail(x, RB_EINVAL, "the adjoint is FP64 only");
  if (x->rec_n < 1 || x->rec_ws != ws) return fail(x, RB_EINVAL, "no matching rb_record");
  const int n = x->rec_n, k = x->rec_k;
  const AdjLayout A = adj_layout(x, n, k);
  if (ws_bytes < A.total * sizeof(double)) return fail(x, RB_EINVAL, "workspace too small");
  double* w = (double*)ws;
  double* lam = w + A.lam;
  double* nu = w + A.nu;
  const size_t bytes = A.S * sizeof(double);
  HIPCHK(x, hipMemcpyAsync(lam, lambda_final, bytes, hipMemcpyDeviceToDevice, x->stream), "lambda");
  HIPCHK(x, launch_fill(w + A.sta, 4, 0.0, x->stream), "clear");
  StageArgs a = base_args(x);
  double* dtlog = x->work + x->L.dtlog;
  AdjArgs J;
  std::memset(&J, 0, sizeof(J));
  J.tk = A.tk;
  J.nkc = A.nkc;
  J.stpart = w + A.stp;
  auto vjp = [&](const double* E, double cw, const double* cot, const double* b1, const double* b2,
                 double* out) -> hipError_t {
    J.s = a;
    J.s.in = E;
    J.cot = cot; J.base1 = b1; J.base2 = b2; J.out = out; J.cw = cw;
    for (int grp = 0; grp <= x->g.nd; ++grp) {
      hipError_t e = launch_adj_group(J, A.nblocks, grp, x->stream);
      if (e != hipSuccess) return e;
      if (grp > 0) {
        e = launch_st_accum(J.stpart, A.nblocks, w + A.sta + (grp - 1), x->stream);
        if (e != hipSuccess) return e;
      }
    }
    return hipSuccess;
  };
  std::vector<double> hd(k + 1);
  for (int seg = A.nseg - 1; seg >= 0; --seg) {
    const int m0 = seg * k, len = std::min(k, n - m0);
    for (int q = 0; q < len; ++q) hd[q] = x->rec_dts[m0 + q];
    hd[len] = hd[len - 1];
    HIPCHK(x, hipMemcpyAsync(dtlog, hd.data(), (len + 1) * sizeof(double), hipMemcpyHostToDevice,
                             x->stream), "upload dt");
    // states of the segment: E_0 the checkpoint, E_q (q >= 1) and midpoints S_q
    auto Eq = [&](int q) {
      return q == 0 ? w + A.ck + (size_t)seg * up32(A.S) : w + A.segE + (size_t)(q - 1) * up32(A.S);
    };
    auto Sq = [&](int q) { return w + A.segS + (size_t)q * up32(A.S); };
    for (int q = 0; q < len; ++q) {
      a.step = (int)(m0 + q);
      a.dt_idx = q;
      a.mode = MODE_UPDATE;
      a.gas_only = 0;
      a.in = Eq(q); a.base = Eq(q); a.out = Sq(q); a.coef = 0.5; a.second = 0;
      HIPCHK(x, run_stage(x, a), "recompute stage 1");
      if (q + 1 < len) {
        a.in = Sq(q); a.base = Eq(q); a.out = Eq(q + 1); a.coef = 1.0; a.second = 1;
        HIPCHK(x, run_stage(x, a), "recompute stage 2");
      }
    }
    // reverse: nu = J_G(S)^T (dt/V lambda); lambda <- lambda + nu + J_G(E)^T (dt/(2V) nu)
    for (int q = len - 1; q >= 0; --q) {
      const double dt = x->rec_dts[m0 + q];
      HIPCHK(x, vjp(Sq(q), dt, lam, nullptr, nullptr, nu), "adjoint stage 2");
      HIPCHK(x, vjp(Eq(q), 0.5 * dt, nu, lam, nu, lam), "adjoint stage 1");
    }
  }
  HIPCHK(x, hipMemcpyAsync(grad_state0, lam, bytes, hipMemcpyDeviceToDevice, x->stream), "gradient");
  double sta[4] = {0, 0, 0, 0};
  HIPCHK(x, hipMemcpyAsync(sta, w + A.sta, 4 * sizeof(double), hipMemcpyDeviceToHost, x->stream),
         "stokes");
  Ctrl c;
  HIPCHK(x, hipMemcpyAsync(&c, x->work + x->L.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, x->stream),
         "read control");
  HIPCHK(x, hipStreamSynchronize(x->stream), "sync");
  if (grad_stokes)
    for (int s = 0; s < x->g.nd; ++s) grad_stokes[s] = sta[s];
  if (c.status & FL_HARD) {
    x->hard = status_of_flags(c.status & FL_HARD);
    return fail(x, (rb_status)x->hard, "hard error while recomputing a recorded segment");
  }
  return RB_OK;
}

rb_status rb_amp_gradient(rb_ctx* x, const double* noise, const double* amp, const void* lam,
                          void* out) {
  if (!x || !lam || !out) return RB_EINVAL;
  if (x->cfg.init_kind != RB_INIT_DISC) return fail(x, RB_EINVAL, "no vortex in this initial state");
  if (x->cfg.rwi_delta != 0.0 || x->cfg.rwi_eps != 0.0)
    return fail(x, RB_EINVAL, "the amplitude gradient covers the vortex-only initial state");
  const size_t N = x->g.N;
  InitArgs ia;
  std::memset(&ia, 0, sizeof(ia));
  ia.g = x->g;
  ia.cfg = x->cfg;
  ia.work = x->work;
  ia.L = x->L;
  ia.state = x->state;
  const size_t NN = (size_t)(1 + x->g.nd) * N;
  if (noise) {
    HIPCHK(x, hipMemcpyAsync(x->stage, noise, NN * sizeof(double), hipMemcpyHostToDevice,
                             x->stream), "noise");
    ia.noise = (const double*)x->stage;
  }
  if (amp) {
    HIPCHK(x, hipMemcpyAsync((double*)x->stage + NN, amp, N * sizeof(double), hipMemcpyHostToDevice,
                             x->stream), "amp");
    ia.amp = (const double*)x->stage + NN;
  }
  HIPCHK(x, launch_amp_grad(ia, (const double*)lam, (double*)out, x->stream), "amp gradient");
  HIPCHK(x, hipStreamSynchronize(x->stream), "sync");
  return RB_OK;
}

const char* rb_last_error(const rb_ctx* x) { return x ? x->err.c_str() : "null context"; }

void rb_destroy(rb_ctx* x) {
  if (!x) return;
  for (hipEvent_t e : x->ev) (void)hipEventDestroy(e);
  delete x;
}

}  // extern "C"
