/*
 * Oracle for one time step of the RoSSBi3D bi-fluid finite-volume scheme
 * (Rendon Restrepo & Barge, arXiv 2207.04252).
 *
 * TEST INFRASTRUCTURE ONLY.  A plain, slow, scalar CPU implementation in FP64,
 * written from the paper to check the HIP library against.  Only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark load it;
 * the product path never does.  It shares no code with the HIP library.
 *
 * Passages followed:
 *   gas conservation laws, ideal gas energy, star gravity   Sect. 2.1, Eq. (1)
 *   cell-centred finite volumes, V dE/dt = G = S V - sum A F  Sect. 2.2
 *   log-spaced r, uniform theta and z                       Sect. 2.3
 *   two ghost cells tied to the stationary flow, periodic   Sect. 2.4
 *   explicit RK2 with a=0, b=1, alpha=beta=1/2; CFL, N=1/2  Sect. 2.5
 *   exact Riemann solver, F* = F(E*)                        Sect. 2.6
 *   E = E0 + E', three-point parabola on E', MinMod         Sect. 2.7
 *   empty-run residual subtracted every stage               Sect. 2.8
 *   pressureless dust, drag rho_d dv / t_stop, back-reaction Sect. 2.9, Table 1
 *   stationary solution                                     App. A
 *   conservative variables, fluxes, sources                 App. B
 *
 * Readings where the paper is silent (each stated again at its function):
 *   - the exact solver is the standard two-rarefaction/two-shock pressure
 *     function solved by Newton from the primitive-variable guess, relative
 *     change <= 1e-12, at most 50 iterations, sampled at x/t = 0;
 *   - the parabola of Sect. 2.7 is taken on the primitive form of the Euler
 *     variables: velocity, pressure and density of the gas as deviations from the
 *     stationary flow's (W' = W(E) - W(E0)), and velocity and density of each dust
 *     fluid whole; the face states are W0(face) + W'(i) + increment, and only
 *     F* = F(E*) is formed from them.  Limiting the conservative variables one by one
 *     was measured to be unstable at the disc's Mach numbers (a clipped increment of
 *     one of rho u, E, rho is a pressure error times Mach^2);
 *   - the MinMod limiter acts on the parabolic face increment, bounded by
 *     twice the one-sided slopes times the face distance (continuous form);
 *   - a face state with rho <= 0 or p <= 0 (dust: rho_d < 0) is replaced by
 *     the cell-centre state;
 *   - the dust Riemann problem is the exact pressureless one (vacuum or
 *     delta shock, the tie s = 0 takes the mean of both fluxes);
 *   - the empty run evaluates the whole spatial operator once on the gas
 *     equilibrium, without dust, and is subtracted from the gas components in
 *     both stages;
 *   - boundary conditions (Sect. 2.4 names them without formulas): bc_r 1 adds
 *     wave-killing zones next to the radial boundaries and bc_z 2 sheared damped zones
 *     next to the vertical ones, both relaxing the gas deviation from the stationary
 *     flow to zero at the rate R / tau (R a quadratic ramp from 0 at the zone's edge to 1
 *     at the boundary, tau = damp_tau orbital periods at the boundary radius, or at the
 *     cell's radius for the vertical zones; the form of de Val-Borro et al. 2006); bc_z 1
 *     is the outflow condition: z ghosts carry the boundary cell's gas deviation scaled
 *     by the ratio of the stationary densities (zero gradient of E'/rho0, so that the
 *     ghost keeps the boundary cell's relative perturbation) and repeat its dust
 *     variables;
 *   - the Rossby-wave-instability initial state (Sect. 4.3) keeps the temperature of the
 *     stationary flow under the density bump and rebalances v_theta radially (the
 *     bump's amplitude, width and centre are configuration values);
 *   - drag uses a constant Stokes number, t_s = St / Omega_K(r), or (drag_law 1) the
 *     Epstein / Stokes law of Sect. 2.9 with c_s the isothermal sound speed sqrt(p/rho)
 *     of the cell's gas (the c_s of App. A) and lambda = mfp_coef / rho_g;
 *   - the drag is explicit inside the RK2 stages (a step at or above the smallest
 *     stopping time is refused), or (drag_exact) split off: the drag alone over dt/2,
 *     the two stages without it, the drag alone over dt/2, each drag part solved exactly
 *     for the cell's held densities and stopping times;
 *   - the density noise of the initial state is one seeded field per fluid.
 * Parity unpinned (no external value exists for them): the limiter variant and the
 * dust tie rule.
 */
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

extern "C" {

typedef struct {
  int32_t nr, nth, nz, log_r, init_kind, balanced, n_dust, indirect;
  double r_in, r_out, z_half, gamma, GM, cfl;
  double sod_r0, sod_left[3], sod_right[3];
  double h0, beta_T, rho_mid0, beta_rho;
  double vortex_amp, vortex_r0, vortex_th0, vortex_sig_r, vortex_sig_a, noise_amp;
  double stokes[4], eps_dust[4], hd_over_h[4];
  int32_t drag_law, drag_exact;
  double grain_size[4], grain_density[4], mfp_coef;
  int32_t bc_r, bc_z;
  double damp_r_in, damp_r_out, damp_z, damp_tau;
  int32_t rwi_m, newton_max_iter;
  double rwi_delta, rwi_dr, rwi_r0, rwi_eps;
} OrConfig;

typedef struct {
  double t;
  int64_t step;
  int32_t flags;
  int32_t first_bad_step;
  int64_t first_bad_cell;
  int64_t fallbacks;
  int64_t vacuum_faces;
  int32_t max_newton;
  int32_t pad;
  double mass[5];     /* gas, dust species 0..3, after the last step          */
  double outflow[5];  /* boundary mass outflow rate of the last second stage   */
  double dt_last;
  int64_t newton_hist[8]; /* gas face solves by Newton iteration count (0: vacuum;   */
                          /* 7: seven or more), every face once per evaluation        */
  int64_t negative_dust;  /* dust densities negative at the end of a step, summed    */
} OrDiag;

}  // extern "C"

namespace {

enum { OR_OK = 0, OR_EINVAL = -1, OR_ENEGATIVE = -4, OR_EVACUUM = -5, OR_ENOCONV = -6,
       OR_ESTIFF = -7 };
enum { F_NEG = 1, F_VAC = 2, F_NOCONV = 4, F_STIFF = 8 };
enum { INIT_SOD = 0, INIT_DISC = 1 };

/* ---------------- scalar types: double, and a forward-mode dual number --------------- */

struct Dual {
  double v, d;
  Dual(double x = 0.0) : v(x), d(0.0) {}
  Dual(double x, double dx) : v(x), d(dx) {}
};
inline Dual operator+(const Dual& a, const Dual& b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(const Dual& a, const Dual& b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator-(const Dual& a) { return Dual(-a.v, -a.d); }
inline Dual operator*(const Dual& a, const Dual& b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(const Dual& a, const Dual& b) {
  double q = a.v / b.v;
  return Dual(q, (a.d - q * b.d) / b.v);
}
inline Dual operator+(const Dual& a, double b) { return Dual(a.v + b, a.d); }
inline Dual operator+(double a, const Dual& b) { return Dual(a + b.v, b.d); }
inline Dual operator-(const Dual& a, double b) { return Dual(a.v - b, a.d); }
inline Dual operator-(double a, const Dual& b) { return Dual(a - b.v, -b.d); }
inline Dual operator*(const Dual& a, double b) { return Dual(a.v * b, a.d * b); }
inline Dual operator*(double a, const Dual& b) { return Dual(a * b.v, a * b.d); }
inline Dual operator/(const Dual& a, double b) { return Dual(a.v / b, a.d / b); }
inline Dual operator/(double a, const Dual& b) {
  double q = a / b.v;
  return Dual(q, -q * b.d / b.v);
}

/* FP64 operation counter: a double that counts its own arithmetic (+ - * / sqrt pow),
 * used to state the algorithmic work of the scheme per cell (comparisons are free). */
struct OpCount { long long n = 0; };
static OpCount g_ops;
struct CountD {
  double v;
  CountD(double x = 0.0) : v(x) {}
};
inline CountD cnt(double x) { ++g_ops.n; return CountD(x); }
inline CountD operator+(const CountD& a, const CountD& b) { return cnt(a.v + b.v); }
inline CountD operator-(const CountD& a, const CountD& b) { return cnt(a.v - b.v); }
inline CountD operator-(const CountD& a) { return CountD(-a.v); }
inline CountD operator*(const CountD& a, const CountD& b) { return cnt(a.v * b.v); }
inline CountD operator/(const CountD& a, const CountD& b) { return cnt(a.v / b.v); }
inline CountD operator+(const CountD& a, double b) { return cnt(a.v + b); }
inline CountD operator+(double a, const CountD& b) { return cnt(a + b.v); }
inline CountD operator-(const CountD& a, double b) { return cnt(a.v - b); }
inline CountD operator-(double a, const CountD& b) { return cnt(a - b.v); }
inline CountD operator*(const CountD& a, double b) { return cnt(a.v * b); }
inline CountD operator*(double a, const CountD& b) { return cnt(a * b.v); }
inline CountD operator/(const CountD& a, double b) { return cnt(a.v / b); }
inline CountD operator/(double a, const CountD& b) { return cnt(a / b.v); }
inline double val(const CountD& x) { return x.v; }
inline CountD sqrt_(const CountD& x) { return cnt(std::sqrt(x.v)); }
inline CountD pow_(const CountD& x, double y) { return cnt(std::pow(x.v, y)); }

inline double val(double x) { return x; }
inline double val(const Dual& x) { return x.v; }
inline double tan_(double) { return 0.0; }
inline double tan_(const Dual& x) { return x.d; }
inline double sqrt_(double x) { return std::sqrt(x); }
inline Dual sqrt_(const Dual& x) {
  double s = std::sqrt(x.v);
  return Dual(s, s > 0.0 ? x.d / (2.0 * s) : 0.0);
}
inline double pow_(double x, double y) { return std::pow(x, y); }
inline Dual pow_(const Dual& x, double y) {
  double p = std::pow(x.v, y);
  return Dual(p, x.d == 0.0 ? 0.0 : y * std::pow(x.v, y - 1.0) * x.d);
}
template <class T> inline T max_(const T& a, const T& b) { return val(a) >= val(b) ? a : b; }
template <class T> inline T min_(const T& a, const T& b) { return val(a) <= val(b) ? a : b; }
template <class T> inline T abs_(const T& a) { return val(a) < 0.0 ? -a : a; }

/* ---------------------------------- Riemann problems --------------------------------- */

/* Primitive state in the frame of a face: density, normal velocity, two tangential
 * velocities, pressure. */
template <class T> struct Prim { T rho, un, ut1, ut2, p; };

/* Pressure function of one side and its derivative (exact solver of Sect. 2.6): a shock
 * branch (Rankine-Hugoniot) when p > p_K, otherwise the isentropic rarefaction branch. */
template <class T>
T pressure_fn(const T& p, const T& rK, const T& pK, const T& cK, double g, T& dfdp) {
  if (val(p) > val(pK)) {
    T A = 2.0 / ((g + 1.0) * rK);
    T B = (g - 1.0) / (g + 1.0) * pK;
    T q = sqrt_(A / (p + B));
    dfdp = q * (1.0 - (p - pK) / (2.0 * (B + p)));
    return (p - pK) * q;
  }
  T pr = p / pK;
  dfdp = pow_(pr, -(g + 1.0) / (2.0 * g)) / (rK * cK);
  return 2.0 * cK / (g - 1.0) * (pow_(pr, (g - 1.0) / (2.0 * g)) - 1.0);
}

struct RiemannInfo { int iters; int vacuum; int noconv; };

/* Gas state on the left of a rarefaction fan, inside the fan, at x/t = 0. */
template <class T>
Prim<T> fan_left(const Prim<T>& L, const T& cL, double g) {
  T c = 2.0 / (g + 1.0) * (cL + 0.5 * (g - 1.0) * L.un);
  T ratio = c / cL;
  Prim<T> W;
  W.rho = L.rho * pow_(ratio, 2.0 / (g - 1.0));
  W.un = c;
  W.p = L.p * pow_(ratio, 2.0 * g / (g - 1.0));
  W.ut1 = L.ut1;
  W.ut2 = L.ut2;
  return W;
}
template <class T>
Prim<T> fan_right(const Prim<T>& R, const T& cR, double g) {
  T c = 2.0 / (g + 1.0) * (cR - 0.5 * (g - 1.0) * R.un);
  T ratio = c / cR;
  Prim<T> W;
  W.rho = R.rho * pow_(ratio, 2.0 / (g - 1.0));
  W.un = -c;
  W.p = R.p * pow_(ratio, 2.0 * g / (g - 1.0));
  W.ut1 = R.ut1;
  W.ut2 = R.ut2;
  return W;
}

/* Exact Riemann problem for the ideal gas (Sect. 2.6), solution sampled at x/t = 0.
 * Newton on p* from the primitive-variable guess; iterate until the relative change
 * 2|dp|/(p_new + p_old) <= 1e-12 (at least one step, at most 50).  The tangential
 * velocities are passive and taken from the side of the contact containing x/t = 0. */
template <class T>
Prim<T> riemann_gas(double g, const Prim<T>& L, const Prim<T>& R, T* pstar_out, T* ustar_out,
                    RiemannInfo& info, int max_iter = 50) {
  info.iters = 0;
  info.vacuum = 0;
  info.noconv = 0;
  T cL = sqrt_(g * L.p / L.rho);
  T cR = sqrt_(g * R.p / R.rho);
  T du = R.un - L.un;
  if (val(2.0 / (g - 1.0) * (cL + cR)) <= val(du)) {
    /* pressure positivity condition violated: vacuum between two rarefactions */
    info.vacuum = 1;
    T sHL = L.un - cL, sSL = L.un + 2.0 * cL / (g - 1.0);
    T sSR = R.un - 2.0 * cR / (g - 1.0), sHR = R.un + cR;
    if (pstar_out) *pstar_out = 0.0;
    if (ustar_out) *ustar_out = 0.0;
    if (0.0 <= val(sHL)) return L;
    if (0.0 < val(sSL)) return fan_left(L, cL, g);
    if (0.0 <= val(sSR)) {
      Prim<T> V;
      V.rho = 0.0; V.un = 0.0; V.ut1 = 0.0; V.ut2 = 0.0; V.p = 0.0;
      return V;
    }
    if (0.0 < val(sHR)) return fan_right(R, cR, g);
    return R;
  }
  T ppv = 0.5 * (L.p + R.p) - 0.125 * du * (L.rho + R.rho) * (cL + cR);
  T p = max_(ppv, T(1e-8 * min_(L.p, R.p)));
  bool conv = false;
  for (int it = 1; it <= max_iter; ++it) {
    T dL, dR;
    T fL = pressure_fn(p, L.rho, L.p, cL, g, dL);
    T fR = pressure_fn(p, R.rho, R.p, cR, g, dR);
    T pn = p - (fL + fR + du) / (dL + dR);
    if (val(pn) < 1e-8 * val(p)) pn = 1e-8 * p;
    double change = 2.0 * std::fabs(val(pn) - val(p)) / (val(pn) + val(p));
    p = pn;
    info.iters = it;
    if (change <= 1e-12) { conv = true; break; }
  }
  if (!conv) info.noconv = 1;
  T dL, dR;
  T fL = pressure_fn(p, L.rho, L.p, cL, g, dL);
  T fR = pressure_fn(p, R.rho, R.p, cR, g, dR);
  T us = 0.5 * (L.un + R.un) + 0.5 * (fR - fL);
  if (pstar_out) *pstar_out = p;
  if (ustar_out) *ustar_out = us;

  Prim<T> W;
  if (0.0 <= val(us)) {
    /* x/t = 0 lies left of the contact */
    if (val(p) > val(L.p)) {
      T sL = L.un - cL * sqrt_((g + 1.0) / (2.0 * g) * p / L.p + (g - 1.0) / (2.0 * g));
      if (0.0 <= val(sL)) return L;
      T q = p / L.p, k = (g - 1.0) / (g + 1.0);
      W.rho = L.rho * (q + k) / (k * q + 1.0);
      W.un = us; W.p = p;
    } else {
      T sHL = L.un - cL;
      if (0.0 <= val(sHL)) return L;
      T cml = cL * pow_(p / L.p, (g - 1.0) / (2.0 * g));
      T sTL = us - cml;
      if (0.0 > val(sTL)) {
        W.rho = L.rho * pow_(p / L.p, 1.0 / g);
        W.un = us; W.p = p;
      } else {
        return fan_left(L, cL, g);
      }
    }
    W.ut1 = L.ut1; W.ut2 = L.ut2;
    return W;
  }
  /* x/t = 0 lies right of the contact */
  if (val(p) > val(R.p)) {
    T sR = R.un + cR * sqrt_((g + 1.0) / (2.0 * g) * p / R.p + (g - 1.0) / (2.0 * g));
    if (0.0 >= val(sR)) return R;
    T q = p / R.p, k = (g - 1.0) / (g + 1.0);
    W.rho = R.rho * (q + k) / (k * q + 1.0);
    W.un = us; W.p = p;
  } else {
    T sHR = R.un + cR;
    if (0.0 >= val(sHR)) return R;
    T cmr = cR * pow_(p / R.p, (g - 1.0) / (2.0 * g));
    T sTR = us + cmr;
    if (0.0 <= val(sTR)) {
      W.rho = R.rho * pow_(p / R.p, 1.0 / g);
      W.un = us; W.p = p;
    } else {
      return fan_right(R, cR, g);
    }
  }
  W.ut1 = R.ut1; W.ut2 = R.ut2;
  return W;
}

/* Physical gas flux along the face normal from a primitive state: mass, normal momentum,
 * two tangential momenta, energy (Eq. (1) and App. B, with (E + P) u for the energy). */
template <class T>
void gas_flux(double g, const Prim<T>& W, T out[5]) {
  T en = W.p / (g - 1.0) + 0.5 * W.rho * (W.un * W.un + W.ut1 * W.ut1 + W.ut2 * W.ut2);
  out[0] = W.rho * W.un;
  out[1] = W.rho * W.un * W.un + W.p;
  out[2] = W.rho * W.un * W.ut1;
  out[3] = W.rho * W.un * W.ut2;
  out[4] = (en + W.p) * W.un;
}

/* Pressureless (dust) Riemann problem sampled at x/t = 0 (Sect. 2.9: the gas solver with
 * the pressure removed).  Diverging or equal velocities: each side moves away or stays,
 * with vacuum between; converging velocities: a delta shock of speed
 * s = (sqrt(rho_L) u_L + sqrt(rho_R) u_R) / (sqrt(rho_L) + sqrt(rho_R)).  The state at
 * x/t = 0 is the upwind one; at s = 0 the mean of both fluxes is taken.
 * Output: mass, normal momentum, tangential momenta. */
template <class T>
void riemann_dust(const Prim<T>& Lin, const Prim<T>& Rin, T out[4]) {
  Prim<T> L = Lin, R = Rin;
  if (val(L.rho) <= 0.0) { L.rho = 0.0; L.un = 0.0; L.ut1 = 0.0; L.ut2 = 0.0; }
  if (val(R.rho) <= 0.0) { R.rho = 0.0; R.un = 0.0; R.ut1 = 0.0; R.ut2 = 0.0; }
  for (int q = 0; q < 4; ++q) out[q] = 0.0;
  if (val(L.rho) + val(R.rho) == 0.0) return;
  auto flux_of = [](const Prim<T>& W, T f[4]) {
    f[0] = W.rho * W.un;
    f[1] = W.rho * W.un * W.un;
    f[2] = W.rho * W.un * W.ut1;
    f[3] = W.rho * W.un * W.ut2;
  };
  if (val(L.un) <= val(R.un)) {
    if (val(L.un) > 0.0) flux_of(L, out);
    else if (val(R.un) < 0.0) flux_of(R, out);
    return; /* vacuum at x/t = 0: zero flux */
  }
  T sl = sqrt_(L.rho), sr = sqrt_(R.rho);
  T a = sl * L.un;
  T b = sr * R.un;
  T num = a + b;
  if (val(num) > 0.0) flux_of(L, out);
  else if (val(num) < 0.0) flux_of(R, out);
  else {
    T fl[4], fr[4];
    flux_of(L, fl);
    flux_of(R, fr);
    for (int q = 0; q < 4; ++q) out[q] = 0.5 * (fl[q] + fr[q]);
  }
}

/* ---------------------------------- reconstruction ----------------------------------- */

/* sign-agreeing minimum of three numbers, zero when the signs differ */
template <class T> T minmod3(const T& x, const T& y, const T& z) {
  if (val(x) > 0.0 && val(y) > 0.0 && val(z) > 0.0) return min_(x, min_(y, z));
  if (val(x) < 0.0 && val(y) < 0.0 && val(z) < 0.0) return max_(x, max_(y, z));
  return T(0.0);
}

/* Increment of the three-point parabola on E' from the centre x0 of cell i to a face xf
 * of that cell (Sect. 2.7): with the one-sided gradients dE'(i) = (E'_i - E'_{i-1})/(x_i -
 * x_{i-1}) and dE'(i+1), a = [dE'(i+1) - dE'(i)] / (x_{i+1} - x_{i-1}) and
 * b = [dE'(i+1)(x_i - x_{i-1}) + dE'(i)(x_{i+1} - x_i)] / (x_{i+1} - x_{i-1}); the
 * increment a d^2 + b d (d = xf - x_i) is then limited by MinMod against 2 d dE'(i) and
 * 2 d dE'(i+1), which leaves smooth monotone data untouched and flattens extrema. */
template <class T>
T parabola_increment(const T& em, const T& e0, const T& ep, double xm, double x0, double xp,
                     double xf) {
  T Dm = (e0 - em) / (x0 - xm);
  T Dp = (ep - e0) / (xp - x0);
  T a = (Dp - Dm) / (xp - xm);
  T b = (Dp * (x0 - xm) + Dm * (xp - x0)) / (xp - xm);
  double d = xf - x0;
  T inc = a * d * d + b * d;
  return minmod3(inc, 2.0 * d * Dm, 2.0 * d * Dp);
}

inline int wrapi(int j, int n) { j %= n; return j < 0 ? j + n : j; }

/* ------------------------------------- simulation ------------------------------------ */

template <class T>
struct Sim {
  OrConfig c;
  int nr, nth, nz, nd, nf;
  bool twod;
  size_t N;
  double dth, dz;
  std::vector<double> rf;  /* r faces, i = -2..nr+2 at [i+2] */
  std::vector<double> rc;  /* r centres, i = -2..nr+1 at [i+2] */
  std::vector<double> zc;  /* z centres, k = 0..nz-1 */
  std::vector<double> zf;  /* z faces,  k = 0..nz   */
  std::vector<double> V, Ar, Ath, Az;
  std::vector<double> bg_c, bg_r, bg_z, R0;
  std::vector<T> E, Es, Gb, Ep, Fr, Fth, Fz;
  T stokes[4];
  double t = 0.0;
  long step = 0;
  int flags = 0;
  int first_bad_step = -1;
  long first_bad_cell = -1;
  long fallbacks = 0, vacuum_faces = 0;
  int max_newton = 0;
  long newton_hist[8] = {0, 0, 0, 0, 0, 0, 0, 0};  /* gas solves by Newton iterations */
  long negative_dust = 0;  /* dust densities negative at the end of a step */
  double outflow[5] = {0, 0, 0, 0, 0};
  double dt_last = 0.0;

  size_t idx(int k, int i, int j) const { return ((size_t)k * nr + i) * nth + j; }
  double rfa(int i) const { return rf[i + 2]; }
  double rce(int i) const { return rc[i + 2]; }

  bool setup(const OrConfig& cfg) {
    c = cfg;
    nr = c.nr; nth = c.nth; nz = c.nz; nd = c.n_dust;
    if (nr < 3 || nth < 1 || nz < 1 || nd < 0 || nd > 4) return false;
    if (c.gamma <= 1.0) return false;
    if (c.bc_r < 0 || c.bc_r > 1 || c.bc_z < 0 || c.bc_z > 2) return false;
    if ((c.bc_r == 1 || c.bc_z == 2) &&
        (!(c.GM > 0.0) || !(c.damp_tau > 0.0) || !(c.damp_r_in > 1.0) ||
         !(c.damp_r_out > 0.0 && c.damp_r_out < 1.0) || !(c.damp_z > 0.0 && c.damp_z < 1.0)))
      return false;
    nf = 5 + 4 * nd;
    twod = (nz == 1);
    N = (size_t)nr * nth * nz;
    dth = 2.0 * M_PI / nth;
    dz = twod ? 1.0 : 2.0 * c.z_half / nz;
    /* mesh, Sect. 2.3: logarithmic or uniform in r, uniform in theta and z */
    rf.resize(nr + 5);
    for (int i = -2; i <= nr + 2; ++i) {
      if (c.log_r) rf[i + 2] = c.r_in * std::pow(c.r_out / c.r_in, (double)i / nr);
      else rf[i + 2] = c.r_in + i * (c.r_out - c.r_in) / nr;
    }
    rc.resize(nr + 4);
    for (int i = -2; i <= nr + 1; ++i) rc[i + 2] = 0.5 * (rfa(i) + rfa(i + 1));
    zc.resize(nz);
    zf.resize(nz + 1);
    for (int k = 0; k < nz; ++k) zc[k] = twod ? 0.0 : (k + 0.5 - 0.5 * nz) * dz;
    for (int k = 0; k <= nz; ++k) zf[k] = twod ? 0.0 : (k - 0.5 * nz) * dz;
    /* exact annular volumes and face areas */
    V.resize(nr); Ath.resize(nr); Az.resize(nr); Ar.resize(nr + 1);
    for (int i = 0; i < nr; ++i) {
      double rm = rfa(i), rp = rfa(i + 1);
      V[i] = 0.5 * (rp * rp - rm * rm) * dth * dz;
      Ath[i] = (rp - rm) * dz;
      Az[i] = 0.5 * (rp * rp - rm * rm) * dth;
    }
    for (int i = 0; i <= nr; ++i) Ar[i] = rfa(i) * dth * dz;
    for (int s = 0; s < 4; ++s) stokes[s] = c.stokes[s];
    /* stationary solution at cell centres and face centres (App. A) */
    bg_c.assign((size_t)nz * nr * nf, 0.0);
    bg_r.assign((size_t)nz * (nr + 1) * nf, 0.0);
    bg_z.assign((size_t)(nz + 1) * nr * nf, 0.0);
    for (int k = 0; k < nz; ++k)
      for (int i = 0; i < nr; ++i) split_ref(rce(i), zc[k], &bg_c[((size_t)k * nr + i) * nf]);
    for (int k = 0; k < nz; ++k)
      for (int i = 0; i <= nr; ++i) split_ref(rfa(i), zc[k], &bg_r[((size_t)k * (nr + 1) + i) * nf]);
    for (int k = 0; k <= nz; ++k)
      for (int i = 0; i < nr; ++i) split_ref(rce(i), zf[k], &bg_z[((size_t)k * nr + i) * nf]);
    E.assign(nf * N, T(0.0));
    Es.assign(nf * N, T(0.0));
    Gb.assign(nf * N, T(0.0));
    Ep.assign(nf * N, T(0.0));
    Fr.assign((size_t)nf * nz * (nr + 1) * nth, T(0.0));
    Fth.assign((size_t)nf * nz * nr * nth, T(0.0));
    Fz.assign(twod ? 0 : (size_t)nf * (nz + 1) * nr * nth, T(0.0));
    R0.assign((size_t)nz * nr * 5, 0.0);
    return true;
  }

  void sod_state(const double* s, double* out) const {
    /* s = (rho, p, u_r): conservative (rho u, rho v, rho w, E, rho) */
    double rho = s[0], p = s[1], u = s[2];
    out[0] = rho * u; out[1] = 0.0; out[2] = 0.0;
    out[3] = p / (c.gamma - 1.0) + 0.5 * rho * u * u;
    out[4] = rho;
  }

  /* isothermal sound speed squared, T0 r^beta_T with H/r = h0 at r = 1 */
  double ciso2(double r) const { return c.h0 * c.h0 * c.GM * std::pow(r, c.beta_T); }

  /* Stationary solution of App. A at (r, z): density, pressure, azimuthal velocity.
   * rho0 = rho_mid(r) exp[(GM/c^2)(1/sqrt(r^2+z^2) - 1/r)], P0 = c^2 rho0,
   * v_theta0 = sqrt(-r f_star,r + (r/rho) dP/dr) with the radial pressure gradient
   * differentiated analytically. */
  void equilibrium(double r, double z, double& rho, double& P, double& vth) const {
    double GM = c.GM;
    double c2 = ciso2(r);
    double s = std::sqrt(r * r + z * z);
    double rho_mid = c.rho_mid0 * std::pow(r, c.beta_rho);
    double phi = GM / c2 * (1.0 / s - 1.0 / r);
    rho = rho_mid * std::exp(phi);
    P = c2 * rho;
    double dln_c2 = c.beta_T / r;
    double dln_mid = c.beta_rho / r;
    double dphi = -dln_c2 * phi + GM / c2 * (-r / (s * s * s) + 1.0 / (r * r));
    double dPdr = P * (dln_c2 + dln_mid + dphi);
    double f_r = -GM * r / (s * s * s);
    vth = std::sqrt(-r * f_r + r / rho * dPdr);
  }

  /* dust layer of species s at (r, z): rho_d = eps (H/H_d) rho_mid(r) exp(-z^2/(2 H_d^2))
   * with H = c_iso/Omega_K and H_d = (H_d/H) H (Sect. 4.4 profile, paper's H = sqrt(2)
   * times this H) */
  double dust_density(int s, double r, double z) const {
    double H = std::sqrt(ciso2(r)) / std::sqrt(c.GM / (r * r * r));
    double Hd = c.hd_over_h[s] * H;
    double rho_mid = c.rho_mid0 * std::pow(r, c.beta_rho);
    return c.eps_dust[s] * (H / Hd) * rho_mid * std::exp(-z * z / (2.0 * Hd * Hd));
  }

  /* conservative gas variables (rho u, rho v, rho w, E, rho) of a state with w = 0 */
  template <class S>
  void gas_conservative(double rho, const S& u, const S& v, double P, S* out) const {
    out[0] = rho * u;
    out[1] = rho * v;
    out[2] = S(0.0);
    out[3] = P / (c.gamma - 1.0) + 0.5 * rho * (u * u + v * v);
    out[4] = S(rho);
  }

  /* Background E0 at (r, z): the stationary gas flow; the dust background is the initial
   * axisymmetric dust layer moving with the gas.  Zero for the Sod annulus. */
  void background(double r, double z, double* out) const {
    for (int f = 0; f < nf; ++f) out[f] = 0.0;
    if (c.init_kind != INIT_DISC) return;
    double rho, P, vth;
    equilibrium(r, z, rho, P, vth);
    gas_conservative(rho, 0.0, vth, P, out);
    for (int s = 0; s < nd; ++s) {
      double rd = dust_density(s, r, z);
      out[5 + 4 * s + 0] = 0.0;
      out[5 + 4 * s + 1] = rd * vth;
      out[5 + 4 * s + 2] = 0.0;
      out[5 + 4 * s + 3] = rd;
    }
  }

  /* Reference of the E = E0 + E' split (Sect. 2.7): the stationary gas flow.  The dust
   * has no stationary solution (it settles), so its variables are reconstructed whole:
   * its reference is zero. */
  void split_ref(double r, double z, double* out) const {
    background(r, z, out);
    for (int f = 5; f < nf; ++f) out[f] = 0.0;
  }

  /* Initial state: Sod annulus, or the disc with the column Gaussian vortex (velocity
   * from the streamfunction psi = psi0 exp(-X^2/2sr^2 - Y^2/2sa^2), X = r - r_v,
   * Y = r_v wrap(theta - theta_v), centre vorticity 2 Ro Omega_K(r_v), Ro = -amplitude),
   * density noise rho0 (1 + a xi) on the gas at unchanged pressure and on each dust
   * layer (its own noise field: noise holds (1 + n_dust) fields of N values), dust moving
   * with the gas. */
  void initial_state(const double* noise, const T* amp) {
    for (int k = 0; k < nz; ++k)
      for (int i = 0; i < nr; ++i)
        for (int j = 0; j < nth; ++j) {
          size_t id = idx(k, i, j);
          double r = rce(i), z = zc[k], th = (j + 0.5) * dth;
          if (c.init_kind == INIT_SOD) {
            double s[5];
            sod_state(rce(i) < c.sod_r0 ? c.sod_left : c.sod_right, s);
            for (int f = 0; f < 5; ++f) E[f * N + id] = s[f];
            continue;
          }
          double rho0, P0, vth0;
          equilibrium(r, z, rho0, P0, vth0);
          T A = amp ? amp[id] : T(c.vortex_amp);
          double rv = c.vortex_r0, sr = c.vortex_sig_r, sa = c.vortex_sig_a;
          double X = r - rv;
          double d = th - c.vortex_th0;
          d -= 2.0 * M_PI * std::floor((d + M_PI) / (2.0 * M_PI));
          double Y = rv * d;
          double Om = std::sqrt(c.GM / (rv * rv * rv));
          double psi_hat = -2.0 * Om / (1.0 / (sr * sr) + 1.0 / (sa * sa)) *
                           std::exp(-X * X / (2.0 * sr * sr) - Y * Y / (2.0 * sa * sa));
          double dvr_hat = -psi_hat * rv * Y / (r * sa * sa);
          double dvt_hat = psi_hat * X / (sr * sr);
          /* Rossby-wave-instability seed (Sect. 4.3): a Gaussian overdensity bump
           * B = 1 + delta exp(-(r - r0)^2 / (2 dr^2)) on the density and, at unchanged
           * temperature, on the pressure; the azimuthal velocity rebalanced radially,
           * v^2 = v0^2 + (r/rho) dP/dr - (r/rho0) dP0/dr = v0^2 + r c_iso^2 B'/B; and the
           * radial velocity eps v0 sin(m theta) exp(-(r - r0)^2 / (2 dr^2)). */
          double bump = 1.0, vrw = 0.0, vth = vth0;
          if (c.rwi_delta != 0.0 || c.rwi_eps != 0.0) {
            double x = r - c.rwi_r0;
            double gx = std::exp(-x * x / (2.0 * c.rwi_dr * c.rwi_dr));
            bump = 1.0 + c.rwi_delta * gx;
            double dbump = -c.rwi_delta * x / (c.rwi_dr * c.rwi_dr) * gx;
            vth = std::sqrt(vth0 * vth0 + r * (P0 / rho0) * dbump / bump);
            vrw = c.rwi_eps * vth0 * std::sin(c.rwi_m * th) * gx;
          }
          T u = A * dvr_hat + vrw;
          T v = vth + A * dvt_hat;
          double xi = noise ? noise[id] : 0.0;
          double rho = rho0 * bump * (1.0 + c.noise_amp * xi);
          T q[5];
          gas_conservative(rho, u, v, P0 * bump, q);
          for (int f = 0; f < 5; ++f) E[f * N + id] = q[f];
          for (int s = 0; s < nd; ++s) {
            double xd = noise ? noise[(size_t)(1 + s) * N + id] : 0.0;
            double rd = dust_density(s, r, z) * (1.0 + c.noise_amp * xd);
            E[(5 + 4 * s + 0) * N + id] = rd * u;
            E[(5 + 4 * s + 1) * N + id] = rd * v;
            E[(5 + 4 * s + 2) * N + id] = T(0.0);
            E[(5 + 4 * s + 3) * N + id] = T(rd);
          }
        }
  }

  double ghost_z(int k) const { return twod ? 0.0 : (k + 0.5 - 0.5 * nz) * dz; }

  /* relaxation rate R / tau of the boundary damping zones at a cell centre (0 outside) */
  double damp_rate(double r, double z) const {
    const double two_pi = 6.283185307179586;
    double rate = 0.0;
    if (c.bc_r == 1) {
      double ri = c.damp_r_in * c.r_in, ro = c.damp_r_out * c.r_out;
      if (r < ri) {
        double x = (ri - r) / (ri - c.r_in);
        double tau = c.damp_tau * two_pi / std::sqrt(c.GM / (c.r_in * c.r_in * c.r_in));
        rate += x * x / tau;
      }
      if (r > ro) {
        double x = (r - ro) / (c.r_out - ro);
        double tau = c.damp_tau * two_pi / std::sqrt(c.GM / (c.r_out * c.r_out * c.r_out));
        rate += x * x / tau;
      }
    }
    if (c.bc_z == 2 && !twod) {
      double zd = c.damp_z * c.z_half, az = std::fabs(z);
      if (az > zd) {
        double x = (az - zd) / (c.z_half - zd);
        double tau = c.damp_tau * two_pi / std::sqrt(c.GM / (r * r * r));
        rate += x * x / tau;
      }
    }
    return rate;
  }

  /* Reconstructed variable of any cell, interior or ghost: E' for the gas, the whole
   * conservative variable for the dust.  Ghost cells (Sect. 2.4) hold the stationary
   * flow (gas E' = 0) and the initial dust layer; for the Sod annulus they keep the
   * initial gas state at their radius. */
  T dev(int f, int k, int i, int j) const {
    bool ghost = i < 0 || i >= nr || k < 0 || k >= nz;
    if (!ghost) return Ep[f * N + idx(k, i, wrapi(j, nth))];
    if (c.bc_z == 1 && (k < 0 || k >= nz) && i >= 0 && i < nr) {
      const int kb = k < 0 ? 0 : nz - 1;
      const T e = Ep[f * N + idx(kb, i, wrapi(j, nth))];
      if (f >= 5) return e;
      /* outflow: the boundary cell's gas deviation relative to the stationary density
       * carried into the ghost (zero gradient of E'/rho0) */
      double bg[24], bb[24];
      background(rce(i), ghost_z(k), bg);
      background(rce(i), zc[kb], bb);
      return e * (bg[4] / bb[4]);
    }
    if (f >= 5) {
      double b[24];
      background(rce(i), ghost_z(k), b);
      return T(b[f]);
    }
    if (c.init_kind == INIT_SOD) {
      double q[5];
      sod_state(rce(i) < c.sod_r0 ? c.sod_left : c.sod_right, q);
      return T(q[f]);
    }
    return T(0.0);
  }

  /* primitive gas variables of a conservative state, in the slots of the fields:
   * (u_r, v_theta, w_z, P, rho) from (rho u, rho v, rho w, E, rho) with
   * E = rho |V|^2 / 2 + P / (gamma - 1) (Sect. 2.1, App. B) */
  template <class S>
  void gas_primitives(const S* q, S* w) const {
    w[0] = q[0] / q[4];
    w[1] = q[1] / q[4];
    w[2] = q[2] / q[4];
    w[3] = (c.gamma - 1.0) * (q[3] - 0.5 * (q[0] * w[0] + q[1] * w[1] + q[2] * w[2]));
    w[4] = q[4];
  }
  /* primitive dust variables (u, v, w, rho_d) of (rho_d u, rho_d v, rho_d w, rho_d);
   * the velocity of an empty cell is zero */
  template <class S>
  void dust_primitives(const S* q, S* w) const {
    bool full = val(q[3]) > 0.0;
    for (int a = 0; a < 3; ++a) w[a] = full ? q[a] / q[3] : S(0.0);
    w[3] = q[3];
  }
  /* primitive variables of the stationary flow from its conservative form (zero where
   * the split has no reference: the Sod annulus) */
  void reference_primitives(const double* q0, double* w0) const {
    if (c.init_kind != INIT_DISC) {
      for (int f = 0; f < 5; ++f) w0[f] = 0.0;
      return;
    }
    gas_primitives(q0, w0);
  }
  /* reconstructed variables of a full conservative state at a point whose stationary
   * flow is q0: gas W(E) - W(E0), dust whole primitives */
  void recon_vars(const T* q, const double* q0, T* w, int nfl) const {
    double w0[5];
    reference_primitives(q0, w0);
    gas_primitives(q, w);
    for (int f = 0; f < 5; ++f) w[f] = w[f] - w0[f];
    for (int o = 5; o < nfl; o += 4) dust_primitives(q + o, w + o);
  }
  /* reconstructed variable f of any cell, interior or ghost */
  T recon(int f, int k, int i, int j) const {
    if (i >= 0 && i < nr && k >= 0 && k < nz) return Wr[f * N + idx(k, i, wrapi(j, nth))];
    T q[24], w[24];
    double b[24];
    centre_state(k, i, j, q);
    background(rce(i), ghost_z(k), b);
    recon_vars(q, b, w, nf);
    return w[f];
  }

  /* full state at the centre of any cell, interior or ghost (used by the face-state
   * positivity fallback) */
  void centre_state(int k, int i, int j, T* out) const {
    if (i >= 0 && i < nr && k >= 0 && k < nz) {
      size_t id = idx(k, i, wrapi(j, nth));
      for (int f = 0; f < nf; ++f) out[f] = cur[f * N + id];
      return;
    }
    double b[24];
    background(rce(i), ghost_z(k), b);
    for (int f = 0; f < 5; ++f) out[f] = b[f] + dev(f, k, i, j);
    for (int f = 5; f < nf; ++f) out[f] = dev(f, k, i, j);
  }

  const T* cur = nullptr; /* state whose operator is being evaluated */
  std::vector<T> Wr;      /* reconstructed variables of its interior cells */
  bool in_empty_run = false;
  double last_A = 0.0, last_B = 0.0; /* indirect-gravity sums of the last evaluation */

  /* primitive state in the frame of direction d (0 r, 1 theta, 2 z) from field-slot
   * primitives: gas (u, v, w, P, rho), dust (u, v, w, rho_d) */
  Prim<T> frame_gas(const T* w, int d) const {
    int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
    Prim<T> W;
    W.rho = w[4]; W.un = w[d]; W.ut1 = w[t1]; W.ut2 = w[t2]; W.p = w[3];
    return W;
  }
  Prim<T> frame_dust(const T* w, int d) const {
    int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
    Prim<T> W;
    W.rho = w[3]; W.un = w[d]; W.ut1 = w[t1]; W.ut2 = w[t2]; W.p = 0.0;
    return W;
  }

  /* Numerical flux at one face (Sect. 2.6, steps 1-3): parabolic face states of the two
   * adjacent cells, exact Riemann problem, F* = F(E*).  Cells a, b, cR, d are the four
   * cells along the direction (a, b left of the face; cR, d right), given by their
   * reconstructed variables (gas W', dust primitives); x their coordinates, xf the face
   * coordinate; bgf is E0 at the face; centre_b / centre_c give the full states of b and
   * cR (called only when a fallback needs them).  The face
   * state is W0(face) + W'(b) + increment (Sect. 2.7 on the primitive variables); a gas
   * face state with rho <= 0 or P <= 0 (a dust face state with rho_d < 0) is replaced by
   * the cell-centre state. */
  template <class CB, class CC>
  void face_flux(int dir, const T* va, const T* vb, const T* vc, const T* vd, const double x[4],
                 double xf, const double* bgf, CB&& centre_b, CC&& centre_c, bool with_dust,
                 T* F, long& nfall, long& nvac, int& maxit, int& noconv, long* hist) const {
    const double g = c.gamma;
    int nfl = with_dust ? nf : 5;
    double wf[5];
    reference_primitives(bgf, wf);
    T qL[24], qR[24];
    for (int f = 0; f < nfl; ++f) {
      T incL = parabola_increment(va[f], vb[f], vc[f], x[0], x[1], x[2], xf);
      T incR = parabola_increment(vb[f], vc[f], vd[f], x[1], x[2], x[3], xf);
      double ref = f < 5 ? wf[f] : 0.0;
      qL[f] = ref + (vb[f] + incL);
      qR[f] = ref + (vc[f] + incR);
    }
    /* positivity of the reconstructed states: fall back to the cell-centre state */
    T centL[24], centR[24], wc[24];
    bool haveL = false, haveR = false;
    Prim<T> WL = frame_gas(qL, dir), WR = frame_gas(qR, dir);
    if (!(val(WL.rho) > 0.0 && val(WL.p) > 0.0)) {
      centre_b(centL); haveL = true;
      gas_primitives(centL, wc);
      WL = frame_gas(wc, dir);
      ++nfall;
    }
    if (!(val(WR.rho) > 0.0 && val(WR.p) > 0.0)) {
      centre_c(centR); haveR = true;
      gas_primitives(centR, wc);
      WR = frame_gas(wc, dir);
      ++nfall;
    }
    RiemannInfo info;
    Prim<T> W = riemann_gas(g, WL, WR, (T*)nullptr, (T*)nullptr, info,
                            c.newton_max_iter > 0 ? c.newton_max_iter : 50);
    if (info.vacuum) ++nvac;
    if (info.noconv) noconv = 1;
    maxit = std::max(maxit, info.iters);
    hist[std::min(info.vacuum ? 0 : info.iters, 7)]++;
    T fl[5];
    gas_flux(g, W, fl);
    int t1 = dir == 0 ? 1 : 0, t2 = dir == 2 ? 1 : 2;
    F[4] = fl[0];
    F[dir] = fl[1];
    F[t1] = fl[2];
    F[t2] = fl[3];
    F[3] = fl[4];
    if (!with_dust) return;
    for (int s = 0; s < nd; ++s) {
      int o = 5 + 4 * s;
      if (val(qL[o + 3]) < 0.0) {
        if (!haveL) { centre_b(centL); haveL = true; }
        dust_primitives(&centL[o], &qL[o]);
        ++nfall;
      }
      if (val(qR[o + 3]) < 0.0) {
        if (!haveR) { centre_c(centR); haveR = true; }
        dust_primitives(&centR[o], &qR[o]);
        ++nfall;
      }
      Prim<T> DL = frame_dust(&qL[o], dir), DR = frame_dust(&qR[o], dir);
      T fd[4];
      riemann_dust(DL, DR, fd);
      F[o + 3] = fd[0];
      F[o + dir] = fd[1];
      F[o + t1] = fd[2];
      F[o + t2] = fd[3];
    }
  }

  /* G(U) = S V - sum_s A_s F*.n_s (Sect. 2.2) [- R0 when balanced], for every cell. */
  int evaluate(const std::vector<T>& U, bool with_dust, bool subtract_R0, std::vector<T>& G) {
    cur = U.data();
    int nfl = with_dust ? nf : 5;
    /* deviations from the stationary flow (Sect. 2.7) */
    for (int f = 0; f < nfl; ++f)
      for (int k = 0; k < nz; ++k)
        for (int i = 0; i < nr; ++i)
          for (int j = 0; j < nth; ++j) {
            size_t id = idx(k, i, j);
            Ep[f * N + id] = U[f * N + id] - bg_c[((size_t)k * nr + i) * nf + f];
          }
    /* the variables the parabola is taken on (gas W' about the stationary flow, dust
     * primitives), for the interior cells */
    Wr.assign((size_t)nf * N, T(0.0));
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < nz; ++k)
      for (int i = 0; i < nr; ++i)
        for (int j = 0; j < nth; ++j) {
          size_t id = idx(k, i, j);
          T q[24], w[24];
          for (int f = 0; f < nfl; ++f) q[f] = U[f * N + id];
          recon_vars(q, &bg_c[((size_t)k * nr + i) * nf], w, nfl);
          for (int f = 0; f < nfl; ++f) Wr[f * N + id] = w[f];
        }
    long nfall = 0, nvac = 0;
    int maxit = 0, noconv = 0;
    long nh[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    /* r faces: face fi at rf[fi], between cells fi-1 and fi */
#pragma omp parallel for collapse(2) schedule(static) reduction(+ : nfall, nvac, nh) reduction(max : maxit, noconv)
    for (int k = 0; k < nz; ++k)
      for (int fi = 0; fi <= nr; ++fi)
        for (int j = 0; j < nth; ++j) {
          T va[24], vb[24], vc[24], vd[24], F[24];
          for (int f = 0; f < nfl; ++f) {
            va[f] = recon(f, k, fi - 2, j); vb[f] = recon(f, k, fi - 1, j);
            vc[f] = recon(f, k, fi, j);     vd[f] = recon(f, k, fi + 1, j);
          }
          double x[4] = {rce(fi - 2), rce(fi - 1), rce(fi), rce(fi + 1)};
          face_flux(0, va, vb, vc, vd, x, rfa(fi), &bg_r[((size_t)k * (nr + 1) + fi) * nf],
                    [&](T* q) { centre_state(k, fi - 1, j, q); },
                    [&](T* q) { centre_state(k, fi, j, q); }, with_dust, F, nfall, nvac, maxit,
                    noconv, nh);
          for (int f = 0; f < nfl; ++f) Fr[(((size_t)f * nz + k) * (nr + 1) + fi) * nth + j] = F[f];
        }
    /* theta faces: face j+1/2 between cells j and j+1 (periodic), index coordinates */
#pragma omp parallel for collapse(2) schedule(static) reduction(+ : nfall, nvac, nh) reduction(max : maxit, noconv)
    for (int k = 0; k < nz; ++k)
      for (int i = 0; i < nr; ++i)
        for (int j = 0; j < nth; ++j) {
          T va[24], vb[24], vc[24], vd[24], F[24];
          for (int f = 0; f < nfl; ++f) {
            va[f] = recon(f, k, i, j - 1); vb[f] = recon(f, k, i, j);
            vc[f] = recon(f, k, i, j + 1); vd[f] = recon(f, k, i, j + 2);
          }
          double x[4] = {(double)(j - 1), (double)j, (double)(j + 1), (double)(j + 2)};
          face_flux(1, va, vb, vc, vd, x, j + 0.5, &bg_c[((size_t)k * nr + i) * nf],
                    [&](T* q) { centre_state(k, i, j, q); },
                    [&](T* q) { centre_state(k, i, j + 1, q); }, with_dust, F, nfall, nvac, maxit,
                    noconv, nh);
          for (int f = 0; f < nfl; ++f) Fth[(((size_t)f * nz + k) * nr + i) * nth + j] = F[f];
        }
    /* z faces: face fk at zf[fk], between cells fk-1 and fk, index coordinates */
    if (!twod) {
#pragma omp parallel for collapse(2) schedule(static) reduction(+ : nfall, nvac, nh) reduction(max : maxit, noconv)
      for (int fk = 0; fk <= nz; ++fk)
        for (int i = 0; i < nr; ++i)
          for (int j = 0; j < nth; ++j) {
            T va[24], vb[24], vc[24], vd[24], F[24];
            for (int f = 0; f < nfl; ++f) {
              va[f] = recon(f, fk - 2, i, j); vb[f] = recon(f, fk - 1, i, j);
              vc[f] = recon(f, fk, i, j);     vd[f] = recon(f, fk + 1, i, j);
            }
            double x[4] = {(double)(fk - 2), (double)(fk - 1), (double)fk, (double)(fk + 1)};
            face_flux(2, va, vb, vc, vd, x, fk - 0.5, &bg_z[((size_t)fk * nr + i) * nf],
                      [&](T* q) { centre_state(fk - 1, i, j, q); },
                      [&](T* q) { centre_state(fk, i, j, q); }, with_dust, F, nfall, nvac, maxit,
                      noconv, nh);
            for (int f = 0; f < nfl; ++f) Fz[(((size_t)f * (nz + 1) + fk) * nr + i) * nth + j] = F[f];
          }
    }
    fallbacks += nfall;
    vacuum_faces += nvac;
    for (int b = 0; b < 8; ++b) newton_hist[b] += nh[b];
    max_newton = std::max(max_newton, maxit);
    if (nvac) flags |= F_VAC;
    if (noconv) flags |= F_NOCONV;

    /* indirect gravity (Sect. 2.10): the star is accelerated by the disc,
     * a_star = G sum_cells m r_vec / |r_vec|^3 (gas and dust mass), and the frame centred on
     * the star adds -a_star to every fluid element; with A = sum m r cos(theta)/|r|^3 and
     * B = sum m r sin(theta)/|r|^3 its cylindrical components are
     * -G (A cos(theta) + B sin(theta), -A sin(theta) + B cos(theta), 0).  G = GM (unit star
     * mass).  Not part of the empty run: the stationary flow is axisymmetric. */
    T Aind = 0.0, Bind = 0.0;
    const bool ind = c.indirect != 0 && !in_empty_run;
    if (ind) {
      for (int k = 0; k < nz; ++k)
        for (int i = 0; i < nr; ++i) {
          double r = rce(i), z = zc[k];
          double wgt = V[i] * r / std::pow(r * r + z * z, 1.5);
          for (int j = 0; j < nth; ++j) {
            size_t id = idx(k, i, j);
            double th = (j + 0.5) * dth;
            T m = U[4 * N + id];
            for (int s = 0; s < nd && with_dust; ++s) m = m + U[(5 + 4 * s + 3) * N + id];
            Aind = Aind + m * (wgt * std::cos(th));
            Bind = Bind + m * (wgt * std::sin(th));
          }
        }
      last_A = val(Aind);
      last_B = val(Bind);
    }

    /* divergence and sources per cell */
    const double g = c.gamma;
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < nz; ++k)
      for (int i = 0; i < nr; ++i)
        for (int j = 0; j < nth; ++j) {
          size_t id = idx(k, i, j);
          int jm = wrapi(j - 1, nth);
          T Gc[24];
          for (int f = 0; f < nfl; ++f) {
            T fr_p = Fr[(((size_t)f * nz + k) * (nr + 1) + i + 1) * nth + j];
            T fr_m = Fr[(((size_t)f * nz + k) * (nr + 1) + i) * nth + j];
            T ft_p = Fth[(((size_t)f * nz + k) * nr + i) * nth + j];
            T ft_m = Fth[(((size_t)f * nz + k) * nr + i) * nth + jm];
            T div = (Ar[i + 1] * fr_p - Ar[i] * fr_m) + Ath[i] * (ft_p - ft_m);
            if (!twod) {
              T fz_p = Fz[(((size_t)f * (nz + 1) + k + 1) * nr + i) * nth + j];
              T fz_m = Fz[(((size_t)f * (nz + 1) + k) * nr + i) * nth + j];
              div = div + Az[i] * (fz_p - fz_m);
            }
            Gc[f] = -div;
          }
          /* sources (App. B): geometric terms, star gravity per unit mass, drag */
          double r = rce(i), z = zc[k];
          double s3 = std::pow(r * r + z * z, 1.5);
          double gr = -c.GM * r / s3, gz = -c.GM * z / s3;
          T rho = U[4 * N + id];
          T u = U[0 * N + id] / rho, v = U[1 * N + id] / rho, w = U[2 * N + id] / rho;
          T p = (g - 1.0) * (U[3 * N + id] - 0.5 * (U[0 * N + id] * u + U[1 * N + id] * v +
                                                     U[2 * N + id] * w));
          T S[24];
          S[0] = rho * v * v / r + rho * gr + p / r;
          S[1] = -rho * u * v / r;
          S[2] = rho * gz;
          S[3] = rho * u * gr + rho * w * gz;
          S[4] = T(0.0);
          if (with_dust) {
            double omk = std::sqrt(c.GM / (r * r * r));
            T dragx = 0.0, dragy = 0.0, dragz = 0.0;
            for (int s = 0; s < nd; ++s) {
              int o = 5 + 4 * s;
              T rd = U[(o + 3) * N + id];
              T ud = 0.0, vd = 0.0, wd = 0.0;
              if (val(rd) > 0.0) {
                ud = U[(o + 0) * N + id] / rd; vd = U[(o + 1) * N + id] / rd;
                wd = U[(o + 2) * N + id] / rd;
              }
              T fx = 0.0, fy = 0.0, fz = 0.0;
              if (!c.drag_exact) {
                T ts = stopping_time(s, omk, rho, p);
                fx = rd * (ud - u) / ts; fy = rd * (vd - v) / ts; fz = rd * (wd - w) / ts;
              }
              dragx = dragx + fx; dragy = dragy + fy; dragz = dragz + fz;
              S[o + 0] = rd * vd * vd / r + rd * gr - fx;
              S[o + 1] = -rd * ud * vd / r - fy;
              S[o + 2] = rd * gz - fz;
              S[o + 3] = T(0.0);
            }
            S[0] = S[0] + dragx;
            S[1] = S[1] + dragy;
            S[2] = S[2] + dragz;
            S[3] = S[3] + (u * dragx + v * dragy + w * dragz);
          }
          if (ind) {
            double th = (j + 0.5) * dth;
            double cs = std::cos(th), sn = std::sin(th);
            T ar = -c.GM * (Aind * cs + Bind * sn);
            T at = -c.GM * (Bind * cs - Aind * sn);
            S[0] = S[0] + rho * ar;
            S[1] = S[1] + rho * at;
            S[3] = S[3] + rho * (u * ar + v * at);
            for (int s = 0; s < nd && with_dust; ++s) {
              int o = 5 + 4 * s;
              T rd = U[(o + 3) * N + id];
              S[o + 0] = S[o + 0] + rd * ar;
              S[o + 1] = S[o + 1] + rd * at;
            }
          }
          /* boundary damping zones: the gas deviation relaxes to the stationary flow */
          if (c.bc_r == 1 || c.bc_z == 2) {
            double kd = damp_rate(r, z);
            for (int f = 0; f < 5; ++f) S[f] = S[f] - kd * Ep[f * N + id];
          }
          for (int f = 0; f < nfl; ++f) {
            T gv = Gc[f] + S[f] * V[i];
            if (subtract_R0 && f < 5) gv = gv - R0[((size_t)k * nr + i) * 5 + f];
            G[f * N + id] = gv;
          }
        }
    return 0;
  }

  /* empty run (Sect. 2.8): R0 = G(E0) for the gas, evaluated once by the same operator */
  void empty_run() {
    std::vector<T> U(nf * N, T(0.0));
    for (int f = 0; f < nf; ++f)
      for (int k = 0; k < nz; ++k)
        for (int i = 0; i < nr; ++i)
          for (int j = 0; j < nth; ++j)
            U[f * N + idx(k, i, j)] = bg_c[((size_t)k * nr + i) * nf + f];
    std::vector<T> G(nf * N, T(0.0));
    int sf = flags;
    in_empty_run = true;
    evaluate(U, false, false, G);
    in_empty_run = false;
    flags = sf;
    for (int k = 0; k < nz; ++k)
      for (int i = 0; i < nr; ++i)
        for (int f = 0; f < 5; ++f) R0[((size_t)k * nr + i) * 5 + f] = val(G[f * N + idx(k, i, 0)]);
  }

  /* CFL time step (Sect. 2.5): min over cells of N_CFL V / ((|v| + c_s) max |dA|), the
   * dust adding its own speed |v_d| with no sound speed. */
  double cfl_dt(const std::vector<T>& U) const {
    const double g = c.gamma;
    double dtmin = 1e300;
#pragma omp parallel for collapse(2) reduction(min : dtmin)
    for (int k = 0; k < nz; ++k)
      for (int i = 0; i < nr; ++i) {
        double amax = std::max(std::max(Ar[i], Ar[i + 1]), Ath[i]);
        if (!twod) amax = std::max(amax, Az[i]);
        for (int j = 0; j < nth; ++j) {
          size_t id = idx(k, i, j);
          double rho = val(U[4 * N + id]);
          double u = val(U[0 * N + id]) / rho, v = val(U[1 * N + id]) / rho, w = val(U[2 * N + id]) / rho;
          double p = (g - 1.0) * (val(U[3 * N + id]) - 0.5 * rho * (u * u + v * v + w * w));
          double cs = std::sqrt(g * p / rho);
          double speed = std::sqrt(u * u + v * v + w * w) + cs;
          for (int s = 0; s < nd; ++s) {
            int o = 5 + 4 * s;
            double rd = val(U[(o + 3) * N + id]);
            if (rd > 0.0) {
              double ud = val(U[o * N + id]) / rd, vd = val(U[(o + 1) * N + id]) / rd,
                     wd = val(U[(o + 2) * N + id]) / rd;
              speed = std::max(speed, std::sqrt(ud * ud + vd * vd + wd * wd));
            }
          }
          double dtc = c.cfl * V[i] / (speed * amax);
          dtmin = std::min(dtmin, dtc);
        }
      }
    return dtmin;
  }

  /* first cell (lowest global index) with rho <= 0 or p <= 0 (NaN included), or -1 */
  long first_negative(const std::vector<T>& U) const {
    const double g = c.gamma;
    long bad = -1;
    for (size_t id = 0; id < N && bad < 0; ++id) {
      double rho = val(U[4 * N + id]);
      double m2 = 0.0;
      for (int q = 0; q < 3; ++q) m2 += val(U[q * N + id]) * val(U[q * N + id]);
      double p = (g - 1.0) * (val(U[3 * N + id]) - 0.5 * m2 / rho);
      if (!(rho > 0.0) || !(p > 0.0)) bad = (long)id;
    }
    return bad;
  }

  /* exp(tau A) of an n x n matrix (row-major), n <= 4: the Taylor series of exp(X),
   * X = tau A / 2^s with s the smallest such that the largest absolute row sum of X is at
   * most 1/2, summed to the 20th power (remainder below 1e-25), then squared s times. */
  static void expm(const T* A, int n, double tau, T* M) {
    double nrm = 0.0;
    for (int a = 0; a < n; ++a) {
      double row = 0.0;
      for (int b = 0; b < n; ++b) row += std::fabs(val(A[a * n + b]));
      nrm = std::max(nrm, row * tau);
    }
    int sq = 0;
    while (nrm > 0.5 && sq < 1100) { nrm *= 0.5; ++sq; }
    const double scale = std::ldexp(tau, -sq);
    T X[16], term[16], sum[16], tmp[16];
    for (int q = 0; q < n * n; ++q) {
      X[q] = A[q] * scale;
      term[q] = T((q / n) == (q % n) ? 1.0 : 0.0);
      sum[q] = term[q];
    }
    for (int k = 1; k <= 20; ++k) {
      for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) {
          T acc = 0.0;
          for (int m = 0; m < n; ++m) acc = acc + term[a * n + m] * X[m * n + b];
          tmp[a * n + b] = acc / (double)k;
        }
      for (int q = 0; q < n * n; ++q) { term[q] = tmp[q]; sum[q] = sum[q] + term[q]; }
    }
    for (int r = 0; r < sq; ++r) {
      for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) {
          T acc = 0.0;
          for (int m = 0; m < n; ++m) acc = acc + sum[a * n + m] * sum[m * n + b];
          tmp[a * n + b] = acc;
        }
      for (int q = 0; q < n * n; ++q) sum[q] = tmp[q];
    }
    for (int q = 0; q < n * n; ++q) M[q] = sum[q];
  }

  /* The drag alone over a time tau, exactly (Sect. 2.9 forces; the integration over a
   * step that may exceed the stopping times).  With the densities and stopping times of
   * the cell held, each velocity component of the gas and of the dust species with
   * rho_s > 0 obeys du_s/dt = -(u_s - u_g)/t_s, du_g/dt = sum_s eps_s (u_s - u_g)/t_s,
   * eps_s = rho_s/rho_g.  The total momentum P = rho_g u_g + sum_s rho_s u_s is constant,
   * and the relative velocities d_s = u_s - u_g obey the linear system
   * dd_s/dt = -d_s/t_s - sum_k eps_k d_k/t_k, so d(tau) = exp(tau B) d(0); then
   * u_g = (P - sum_s rho_s d_s) / (rho_g + sum_s rho_s) and u_s = u_g + d_s.  The gas energy
   * changes by the change of the gas kinetic energy (the work u_g . f of the force on the
   * gas, as in the explicit source), so the pressure is unchanged.  Species with
   * rho_s <= 0 take no part.  q: the cell's conservative variables, updated in place. */
  void relax_cell(T* q, double omk, double tau) const {
    const double g = c.gamma;
    T rho = q[4];
    T p = (g - 1.0) * (q[3] - 0.5 * (q[0] * q[0] + q[1] * q[1] + q[2] * q[2]) / rho);
    int sp[4];
    T ia[4], eps[4];
    int n = 0;
    for (int s = 0; s < nd; ++s) {
      T rd = q[5 + 4 * s + 3];
      if (!(val(rd) > 0.0)) continue;
      sp[n] = s;
      ia[n] = 1.0 / stopping_time(s, omk, rho, p);
      eps[n] = rd / rho;
      ++n;
    }
    if (n == 0) return;
    T B[16], M[16];
    for (int a = 0; a < n; ++a)
      for (int b = 0; b < n; ++b) B[a * n + b] = -(eps[b] * ia[b]) - (a == b ? ia[a] : T(0.0));
    expm(B, n, tau, M);
    T mtot = rho;
    for (int a = 0; a < n; ++a) mtot = mtot + q[5 + 4 * sp[a] + 3];
    T dE = 0.0;
    for (int d = 0; d < 3; ++d) {
      T ug = q[d] / rho;
      T P = q[d];
      T d0[4], d1[4];
      for (int a = 0; a < n; ++a) {
        int o = 5 + 4 * sp[a];
        P = P + q[o + d];
        d0[a] = q[o + d] / q[o + 3] - ug;
      }
      T pd = 0.0;
      for (int a = 0; a < n; ++a) {
        d1[a] = 0.0;
        for (int b = 0; b < n; ++b) d1[a] = d1[a] + M[a * n + b] * d0[b];
        pd = pd + q[5 + 4 * sp[a] + 3] * d1[a];
      }
      T ug1 = (P - pd) / mtot;
      q[d] = rho * ug1;
      for (int a = 0; a < n; ++a) {
        int o = 5 + 4 * sp[a];
        q[o + d] = q[o + 3] * (ug1 + d1[a]);
      }
      dE = dE + 0.5 * rho * (ug1 * ug1 - ug * ug);
    }
    q[3] = q[3] + dE;
  }

  /* relax_cell over every cell of U */
  void drag_relax(std::vector<T>& U, double tau) const {
#pragma omp parallel for schedule(static)
    for (long id = 0; id < (long)N; ++id) {
      int i = (int)((id / nth) % nr);
      double r = rce(i);
      T q[24];
      for (int f = 0; f < nf; ++f) q[f] = U[(size_t)f * N + id];
      relax_cell(q, std::sqrt(c.GM / (r * r * r)), tau);
      for (int f = 0; f < nf; ++f) U[(size_t)f * N + id] = q[f];
    }
  }

  /* stopping time of species s in a cell (Sect. 2.9).  Law 0: t_s = St / Omega_K.
   * Law 1: Epstein t = rho_s r_p / (rho_g c_s) while r_p <= 9 lambda / 4, else Stokes
   * t = (4/9) (r_p / lambda) t^E, with lambda = mfp_coef / rho_g (the mean free path
   * mu m_u / (sigma_eff rho_g) with its constant folded) and c_s = sqrt(p / rho_g). */
  T stopping_time(int s, double omk, T rho, T p) const {
    if (c.drag_law == 0) return stokes[s] / omk;
    T cs = sqrt_(p / rho);
    T tE = (c.grain_density[s] * c.grain_size[s]) / (rho * cs);
    T lam = c.mfp_coef / rho;
    if (c.grain_size[s] <= 9.0 * val(lam) / 4.0) return tE;
    return (4.0 / 9.0) * (c.grain_size[s] / lam) * tE;
  }

  /* smallest stopping time over species and cells of the state U */
  double min_stopping_time(const std::vector<T>& U) const {
    const double g = c.gamma;
    double tmin = 1e300;
    if (c.drag_law == 0) {
      for (int s = 0; s < nd; ++s)
        for (int i = 0; i < nr; ++i) {
          double r = rce(i);
          tmin = std::min(tmin, val(stokes[s]) / std::sqrt(c.GM / (r * r * r)));
        }
      return tmin;
    }
    for (size_t id = 0; id < N; ++id) {
      double rho = val(U[4 * N + id]);
      double m2 = 0.0;
      for (int q = 0; q < 3; ++q) m2 += val(U[q * N + id]) * val(U[q * N + id]);
      double p = (g - 1.0) * (val(U[3 * N + id]) - 0.5 * m2 / rho);
      for (int s = 0; s < nd; ++s) tmin = std::min(tmin, val(stopping_time(s, 1.0, T(rho), T(p))));
    }
    return tmin;
  }

  /* pairwise (fixed-tree) sum */
  static double psum(const double* a, size_t n) {
    if (n <= 8) {
      double s = 0.0;
      for (size_t q = 0; q < n; ++q) s += a[q];
      return s;
    }
    size_t h = n / 2;
    return psum(a, h) + psum(a + h, n - h);
  }

  void masses(double* out) const {
    std::vector<double> tmp(N);
    for (int s = 0; s <= nd; ++s) {
      int f = s == 0 ? 4 : 5 + 4 * (s - 1) + 3;
      for (int k = 0; k < nz; ++k)
        for (int i = 0; i < nr; ++i)
          for (int j = 0; j < nth; ++j) {
            size_t id = idx(k, i, j);
            tmp[id] = val(E[f * N + id]) * V[i];
          }
      out[s] = psum(tmp.data(), N);
    }
  }

  /* boundary mass outflow rate of the fluxes currently stored (outer minus inner r
   * boundary, top minus bottom z boundary) */
  void boundary_outflow(double* out) const {
    std::vector<double> tmp;
    for (int s = 0; s <= nd; ++s) {
      int f = s == 0 ? 4 : 5 + 4 * (s - 1) + 3;
      tmp.clear();
      for (int k = 0; k < nz; ++k)
        for (int j = 0; j < nth; ++j) {
          tmp.push_back(Ar[nr] * val(Fr[(((size_t)f * nz + k) * (nr + 1) + nr) * nth + j]));
          tmp.push_back(-Ar[0] * val(Fr[(((size_t)f * nz + k) * (nr + 1) + 0) * nth + j]));
        }
      if (!twod)
        for (int i = 0; i < nr; ++i)
          for (int j = 0; j < nth; ++j) {
            tmp.push_back(Az[i] * val(Fz[(((size_t)f * (nz + 1) + nz) * nr + i) * nth + j]));
            tmp.push_back(-Az[i] * val(Fz[(((size_t)f * (nz + 1) + 0) * nr + i) * nth + j]));
          }
      out[s] = psum(tmp.data(), tmp.size());
    }
  }

  void record_bad(long cell) {
    if (first_bad_cell < 0) { first_bad_cell = cell; first_bad_step = (int)step; }
  }

  /* One RK2 step (Sect. 2.5 with a = 0, b = 1, alpha = beta = 1/2, read with Eq. (4)):
   * E* = E^n + (dt/2V) G(E^n),  E^{n+1} = E^n + (dt/V) G(E*). */
  int one_step(double dt) {
    bool with_dust = nd > 0;
    bool bal = c.balanced != 0;
    const bool split = c.drag_exact && nd > 0;
    if (split) drag_relax(E, 0.5 * dt);
    evaluate(E, with_dust, bal, Gb);
    for (int f = 0; f < nf; ++f)
      for (int k = 0; k < nz; ++k)
        for (int i = 0; i < nr; ++i) {
          double cfac = 0.5 * dt / V[i];
          for (int j = 0; j < nth; ++j) {
            size_t id = f * N + idx(k, i, j);
            Es[id] = E[id] + cfac * Gb[id];
          }
        }
    if (flags & F_NOCONV) return OR_ENOCONV;
    long bad = first_negative(Es);
    if (bad >= 0) { flags |= F_NEG; record_bad(bad); return OR_ENEGATIVE; }
    evaluate(Es, with_dust, bal, Gb);
    for (int f = 0; f < nf; ++f)
      for (int k = 0; k < nz; ++k)
        for (int i = 0; i < nr; ++i) {
          double cfac = dt / V[i];
          for (int j = 0; j < nth; ++j) {
            size_t id = f * N + idx(k, i, j);
            E[id] = E[id] + cfac * Gb[id];
          }
        }
    boundary_outflow(outflow);
    for (int q = 0; q < nd; ++q)
      for (size_t id = 0; id < N; ++id)
        if (val(E[(size_t)(5 + 4 * q + 3) * N + id]) < 0.0) ++negative_dust;
    if (flags & F_NOCONV) return OR_ENOCONV;
    bad = first_negative(E);
    if (bad >= 0) { flags |= F_NEG; record_bad(bad); return OR_ENEGATIVE; }
    if (split) drag_relax(E, 0.5 * dt);
    t += dt;
    ++step;
    return OR_OK;
  }

  /* dt_kind: 0 CFL, 1 fixed, 2 list */
  int run(int n, int dt_kind, double dt_fixed, const double* dt_list, double* dt_out) {
    if (flags & (F_NEG | F_NOCONV | F_STIFF)) return OR_EINVAL;
    long bad0 = first_negative(E);
    if (bad0 >= 0) { flags |= F_NEG; record_bad(bad0); return OR_ENEGATIVE; }
    for (int q = 0; q < n; ++q) {
      double dt;
      if (dt_kind == 0) dt = cfl_dt(E);
      else if (dt_kind == 1) dt = dt_fixed;
      else dt = dt_list[q];
      if (!(dt > 0.0)) return OR_EINVAL;
      if (nd > 0 && !c.drag_exact && dt >= min_stopping_time(E)) { flags |= F_STIFF; return OR_ESTIFF; }
      if (dt_out) dt_out[q] = dt;
      dt_last = dt;
      int st = one_step(dt);
      if (st != OR_OK) return st;
    }
    return (flags & F_VAC) ? OR_EVACUUM : OR_OK;
  }

  /* dust mass in the vortex core: r in [r_lo, r_hi], |theta - theta_v| < dth_core */
  T core_dust_mass(double r_lo, double r_hi, double dcore) const {
    T J = 0.0;
    for (int s = 0; s < nd; ++s) {
      int f = 5 + 4 * s + 3;
      for (int k = 0; k < nz; ++k)
        for (int i = 0; i < nr; ++i) {
          double r = rce(i);
          if (r < r_lo || r > r_hi) continue;
          for (int j = 0; j < nth; ++j) {
            double th = (j + 0.5) * dth;
            if (std::fabs(th - c.vortex_th0) >= dcore) continue;
            J = J + E[f * N + idx(k, i, j)] * V[i];
          }
        }
    }
    return J;
  }
};

}  // namespace

/* ---------------------------------------- C ABI -------------------------------------- */

extern "C" {

int or_version(void) { return 1; }

void* or_create(const OrConfig* cfg, const double* noise, const double* amp) {
  Sim<double>* s = new Sim<double>();
  if (!s->setup(*cfg)) { delete s; return nullptr; }
  if (s->c.balanced) s->empty_run();
  s->initial_state(noise, amp);
  return s;
}

void or_destroy(void* h) { delete (Sim<double>*)h; }

int or_step(void* h, int n, int dt_kind, double dt_fixed, const double* dt_list, double* dt_out) {
  return ((Sim<double>*)h)->run(n, dt_kind, dt_fixed, dt_list, dt_out);
}

void or_get_state(void* h, double* out) {
  Sim<double>* s = (Sim<double>*)h;
  std::memcpy(out, s->E.data(), sizeof(double) * s->nf * s->N);
}

void or_set_state(void* h, const double* in) {
  Sim<double>* s = (Sim<double>*)h;
  std::memcpy(s->E.data(), in, sizeof(double) * s->nf * s->N);
}

void or_get_residual(void* h, double* out) {
  Sim<double>* s = (Sim<double>*)h;
  std::memcpy(out, s->R0.data(), sizeof(double) * s->R0.size());
}

/* where: 0 cell centres [nz][nr][nf], 1 r faces [nz][nr+1][nf], 2 z faces [nz+1][nr][nf] */
void or_get_background(void* h, int where, double* out) {
  Sim<double>* s = (Sim<double>*)h;
  const std::vector<double>& b = where == 0 ? s->bg_c : (where == 1 ? s->bg_r : s->bg_z);
  std::memcpy(out, b.data(), sizeof(double) * b.size());
}

/* rf[nr+1], rc[nr], zc[nz], V[nr], Ar[nr+1], Ath[nr], Az[nr] */
void or_get_geometry(void* h, double* rf, double* rc, double* zc, double* V, double* Ar,
                     double* Ath, double* Az) {
  Sim<double>* s = (Sim<double>*)h;
  for (int i = 0; i <= s->nr; ++i) { rf[i] = s->rfa(i); Ar[i] = s->Ar[i]; }
  for (int i = 0; i < s->nr; ++i) {
    rc[i] = s->rce(i); V[i] = s->V[i]; Ath[i] = s->Ath[i]; Az[i] = s->Az[i];
  }
  for (int k = 0; k < s->nz; ++k) zc[k] = s->zc[k];
}

/* G of the current state (balanced as configured), [nf][nz][nr][nth] */
void or_eval_G(void* h, int with_dust, int subtract_R0, double* out) {
  Sim<double>* s = (Sim<double>*)h;
  std::vector<double> G(s->nf * s->N, 0.0);
  s->evaluate(s->E, with_dust != 0 && s->nd > 0, subtract_R0 != 0, G);
  std::memcpy(out, G.data(), sizeof(double) * G.size());
}

double or_cfl_dt(void* h) {
  Sim<double>* s = (Sim<double>*)h;
  return s->cfl_dt(s->E);
}

/* stopping time of every dust species in every cell of the current state, [s][cell] */
void or_stopping_times(void* h, double* out) {
  Sim<double>* s = (Sim<double>*)h;
  const size_t N = s->N;
  const double g = s->c.gamma;
  for (size_t id = 0; id < N; ++id) {
    const std::vector<double>& U = s->E;
    double rho = U[4 * N + id];
    double m2 = U[0 * N + id] * U[0 * N + id] + U[1 * N + id] * U[1 * N + id] +
                U[2 * N + id] * U[2 * N + id];
    double p = (g - 1.0) * (U[3 * N + id] - 0.5 * m2 / rho);
    int i = (int)((id / s->nth) % s->nr);
    double r = s->rce(i);
    double omk = std::sqrt(s->c.GM / (r * r * r));
    for (int q = 0; q < s->nd; ++q) out[(size_t)q * N + id] = s->stopping_time(q, omk, rho, p);
  }
}

double or_min_stopping_time(void* h) {
  Sim<double>* s = (Sim<double>*)h;
  return s->min_stopping_time(s->E);
}

void or_mass(void* h, double* out) { ((Sim<double>*)h)->masses(out); }

void or_diag(void* h, OrDiag* d) {
  Sim<double>* s = (Sim<double>*)h;
  std::memset(d, 0, sizeof(*d));
  d->t = s->t;
  d->step = s->step;
  d->flags = s->flags;
  d->first_bad_step = s->first_bad_step;
  d->first_bad_cell = s->first_bad_cell;
  d->fallbacks = s->fallbacks;
  d->vacuum_faces = s->vacuum_faces;
  d->max_newton = s->max_newton;
  s->masses(d->mass);
  for (int q = 0; q < 5; ++q) d->outflow[q] = s->outflow[q];
  d->dt_last = s->dt_last;
  for (int b = 0; b < 8; ++b) d->newton_hist[b] = s->newton_hist[b];
  d->negative_dust = s->negative_dust;
}

/* indirect-gravity sums A, B of the current state (evaluates the operator once) */
void or_indirect_sums(void* h, double* A, double* B) {
  Sim<double>* s = (Sim<double>*)h;
  std::vector<double> G((size_t)s->nf * s->N);
  int sf = s->flags;
  s->evaluate(s->E, s->nd > 0, s->c.balanced != 0, G);
  s->flags = sf;
  *A = s->last_A;
  *B = s->last_B;
}

double or_core_dust_mass(void* h, double r_lo, double r_hi, double dcore) {
  return ((Sim<double>*)h)->core_dust_mass(r_lo, r_hi, dcore);
}

int or_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* sets the number of OpenMP threads of the oracle's loops (the CPU baseline times one
 * thread and all threads); returns the number now in use */
int or_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

/* Exact gas Riemann problem for unit tests.  WL/WR = (rho, u_n, u_t1, u_t2, p);
 * W = sampled state at x/t = 0; flux = (mass, normal mom., t1 mom., t2 mom., energy);
 * star = (p*, u*); returns the Newton iteration count (negative when vacuum). */
int or_riemann_gas(double g, const double* WL, const double* WR, double* W, double* flux,
                   double* star) {
  Prim<double> L{WL[0], WL[1], WL[2], WL[3], WL[4]}, R{WR[0], WR[1], WR[2], WR[3], WR[4]};
  RiemannInfo info;
  double ps = 0.0, us = 0.0;
  Prim<double> S = riemann_gas(g, L, R, &ps, &us, info);
  W[0] = S.rho; W[1] = S.un; W[2] = S.ut1; W[3] = S.ut2; W[4] = S.p;
  gas_flux(g, S, flux);
  star[0] = ps;
  star[1] = us;
  if (info.noconv) return 0;
  return info.vacuum ? -1 : info.iters;
}

/* Pressure function of one side and its derivative, for unit tests. */
double or_pressure_fn(double g, double p, double rhoK, double pK, double* dfdp) {
  double cK = std::sqrt(g * pK / rhoK);
  return pressure_fn(p, rhoK, pK, cK, g, *dfdp);
}

/* Pressureless Riemann flux for unit tests: W = (rho, u_n, u_t1, u_t2);
 * flux = (mass, normal mom., t1 mom., t2 mom.). */
void or_riemann_dust(const double* WL, const double* WR, double* flux) {
  Prim<double> L{WL[0], WL[1], WL[2], WL[3], 0.0}, R{WR[0], WR[1], WR[2], WR[3], 0.0};
  riemann_dust(L, R, flux);
}

/* One gas face for unit tests (Sect. 2.6-2.7): the four cells A, B | C, D along direction
 * dir (0 r, 1 theta, 2 z) given by their full conservative gas states q4[4][5] and their
 * stationary flow q0[4][5], coordinates x4, face coordinate xf, stationary flow at the face
 * qf[5]; flux[5] in field order; returns the number of face states that fell back to the
 * cell-centre state.  The configuration supplies gamma and the kind of split. */
int or_gas_face_flux(const OrConfig* cfg, int dir, const double* q4, const double* q0,
                     const double* x4, double xf, const double* qf, double* flux) {
  OrConfig c1 = *cfg;
  c1.n_dust = 0;
  Sim<double> s;
  if (!s.setup(c1)) return -1;
  double w[4][24];
  for (int a = 0; a < 4; ++a) s.recon_vars(q4 + 5 * a, q0 + 5 * a, w[a], 5);
  long nfall = 0, nvac = 0;
  int maxit = 0, noconv = 0;
  long nh[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  double F[24];
  s.face_flux(dir, w[0], w[1], w[2], w[3], x4, xf, qf,
              [&](double* q) { for (int f = 0; f < 5; ++f) q[f] = q4[5 + f]; },
              [&](double* q) { for (int f = 0; f < 5; ++f) q[f] = q4[10 + f]; }, false, F, nfall,
              nvac, maxit, noconv, nh);
  for (int f = 0; f < 5; ++f) flux[f] = F[f];
  return (int)nfall;
}

/* The exact drag relaxation of one cell over tau (Sect. 2.9): q holds the nf conservative
 * variables of a cell at radius r, updated in place.  Returns -1 on a bad config. */
int or_drag_relax(const OrConfig* cfg, double r, double* q, double tau) {
  Sim<double> s;
  if (!s.setup(*cfg)) return -1;
  s.relax_cell(q, std::sqrt(cfg->GM / (r * r * r)), tau);
  return 0;
}

/* Limited parabola increment for unit tests. */
double or_parabola_increment(double em, double e0, double ep, double xm, double x0, double xp,
                             double xf) {
  return parabola_increment(em, e0, ep, xm, x0, xp, xf);
}

/* Equilibrium point values for unit tests: out = (rho, P, v_theta). */
void or_equilibrium(const OrConfig* cfg, double r, double z, double* out) {
  Sim<double> s;
  s.c = *cfg;
  s.equilibrium(r, z, out[0], out[1], out[2]);
}

/* Algorithmic FP64 operations of one evaluation of the spatial operator G and one
 * stage update on the initial state, per cell (single thread; + - * / sqrt pow count
 * one each). */
double or_count_ops(const OrConfig* cfg, const double* noise) {
#ifdef _OPENMP
  int nt = omp_get_max_threads();
  omp_set_num_threads(1);
#endif
  Sim<CountD> s;
  if (!s.setup(*cfg)) return -1.0;
  if (s.c.balanced) s.empty_run();
  s.initial_state(noise, nullptr);
  g_ops.n = 0;
  s.evaluate(s.E, s.nd > 0, s.c.balanced != 0, s.Gb);
  for (int f = 0; f < s.nf; ++f)
    for (int k = 0; k < s.nz; ++k)
      for (int i = 0; i < s.nr; ++i) {
        double cfac = 0.5 * 1e-3 / s.V[i];
        for (int j = 0; j < s.nth; ++j) {
          size_t id = f * s.N + s.idx(k, i, j);
          s.Es[id] = s.E[id] + cfac * s.Gb[id];
        }
      }
  long long n = g_ops.n;
#ifdef _OPENMP
  omp_set_num_threads(nt);
#endif
  return (double)n / (double)s.N;
}

/* Tangent-linear run: the whole run with dual numbers.  The amplitude field carries the
 * tangent amp_dot and the Stokes numbers the tangents st_dot; returns J = dust mass in
 * the vortex core after n steps with the given dt list, and its directional derivative. */
int or_tangent(const OrConfig* cfg, const double* noise, const double* amp, const double* amp_dot,
               const double* st_dot, int n, const double* dt_list, double r_lo, double r_hi,
               double dcore, double* J, double* dJ) {
  Sim<Dual> s;
  if (!s.setup(*cfg)) return OR_EINVAL;
  for (int q = 0; q < s.nd; ++q) s.stokes[q] = Dual(cfg->stokes[q], st_dot ? st_dot[q] : 0.0);
  if (s.c.balanced) s.empty_run();
  std::vector<Dual> a(s.N);
  for (size_t q = 0; q < s.N; ++q)
    a[q] = Dual(amp ? amp[q] : cfg->vortex_amp, amp_dot ? amp_dot[q] : 0.0);
  s.initial_state(noise, a.data());
  int st = s.run(n, 2, 0.0, dt_list, nullptr);
  Dual Jv = s.core_dust_mass(r_lo, r_hi, dcore);
  *J = Jv.v;
  *dJ = Jv.d;
  return st;
}

/* Tangent-linear run from a given state: the state carries the tangent dstate0 and the
 * Stokes numbers the tangents st_dot; n steps with the given dt list.  Outputs the final
 * state and its tangent (both nfields x ncells, full values). */
int or_tangent_state(const OrConfig* cfg, const double* state0, const double* dstate0,
                     const double* st_dot, int n, const double* dt_list, double* state_out,
                     double* dstate_out) {
  Sim<Dual> s;
  if (!s.setup(*cfg)) return OR_EINVAL;
  for (int q = 0; q < s.nd; ++q) s.stokes[q] = Dual(cfg->stokes[q], st_dot ? st_dot[q] : 0.0);
  if (s.c.balanced) s.empty_run();
  const size_t M = (size_t)s.nf * s.N;
  for (size_t q = 0; q < M; ++q) s.E[q] = Dual(state0[q], dstate0 ? dstate0[q] : 0.0);
  int st = s.run(n, 2, 0.0, dt_list, nullptr);
  for (size_t q = 0; q < M; ++q) {
    state_out[q] = s.E[q].v;
    dstate_out[q] = s.E[q].d;
  }
  return st;
}

}  // extern "C"
