// Device-side building blocks shared by the forward stage kernels and the adjoint
// kernels: reconstruction, exact gas and pressureless dust Riemann solvers, face
// fluxes, state access with ghost cells, wave reductions, tile order.
#pragma once

#include <math.h>

#include <type_traits>

#include "rb_internal.h"

namespace rb {

// ------------------------------------------------------------------------------------
// small helpers

// minmod of three: when all three share a sign, the one of smallest magnitude, else zero.
// Three branch-free forms giving the same value (only the sign of a zero result can
// differ):
//  * FP32: minmod(a, b) is the median of a, b and 0, and minmod of three is
//    minmod(x, minmod(y, z)): two hardware medians, each returning one of its arguments;
//  * FP64: all positive, the smallest (first term); all negative, the largest (second
//    term); otherwise both terms are zero, and one term always is, so the sum is exact;
//  * FP64 with SEL: the sign test on the sign bits and the magnitude from two minima
//    (fewer live registers: the adjoint's face kernels take it).
__device__ __forceinline__ double minmod3_sel(double x, double y, double z) {
  const unsigned bx = (unsigned)(__double_as_longlong(x) >> 32);
  const unsigned by = (unsigned)(__double_as_longlong(y) >> 32);
  const unsigned bz = (unsigned)(__double_as_longlong(z) >> 32);
  const double m = fmin(fabs(x), fmin(fabs(y), fabs(z)));
  return (int)((bx ^ by) | (bx ^ bz)) >= 0 ? copysign(m, x) : 0.0;
}
template <class T, bool SEL = false>
__device__ __forceinline__ T minmod3(T x, T y, T z) {
  if constexpr (std::is_same<T, float>::value)
    return __builtin_amdgcn_fmed3f(x, __builtin_amdgcn_fmed3f(y, z, 0.0f), 0.0f);
  else if constexpr (SEL)
    return minmod3_sel(x, y, z);
  else
    return fmax(fmin(x, fmin(y, z)), T(0)) + fmin(fmax(x, fmax(y, z)), T(0));
}

// Uniform direction (index coordinates): the three-point parabola gives the upper-face
// increment (dm + 3 dp)/8 and the lower-face increment -(3 dm + dp)/8, limited by the
// one-sided differences (Sect. 2.7).  Written so that mirrored data give exactly
// opposite increments.
template <class T, bool SEL = false>
__device__ __forceinline__ T inc_up_u(T em, T e0, T ep) {
  T dm = e0 - em, dp = ep - e0;
  return minmod3<T, SEL>(fma(T(3), dp, dm) * T(0.125), dm, dp);
}
template <class T, bool SEL = false>
__device__ __forceinline__ T inc_lo_u(T em, T e0, T ep) {
  T dm = e0 - em, dp = ep - e0;
  return minmod3<T, SEL>(-(fma(T(3), dm, dp) * T(0.125)), -dm, -dp);
}
// Non-uniform r: precomputed parabola weights and limiter bounds of the cell.
template <class T, bool SEL = false>
__device__ __forceinline__ T inc_up_c(T em, T e0, T ep, const double* co) {
  T dm = e0 - em, dp = ep - e0;
  return minmod3<T, SEL>(fma(T(co[RC_WPP]), dp, T(co[RC_WPM]) * dm), T(co[RC_LPM]) * dm,
                         T(co[RC_LPP]) * dp);
}
template <class T, bool SEL = false>
__device__ __forceinline__ T inc_lo_c(T em, T e0, T ep, const double* co) {
  T dm = e0 - em, dp = ep - e0;
  return minmod3<T, SEL>(fma(T(co[RC_WMP]), dp, T(co[RC_WMM]) * dm), T(co[RC_LMM]) * dm,
                         T(co[RC_LMP]) * dp);
}

// x^(-1/7) for x > 0: FP32 hardware log2/exp2 seed (relative error ~1e-7 for x in the
// clamped range), then Newton on z^-7 = x written as z <- z + (z/7)(1 - x z^7), whose error
// goes e -> 4 e^2: two steps reach FP64 rounding (4 (4e-14)^2 ~ 1e-26); x = 1 is a fixed
// point.
__device__ __forceinline__ double inv_root7(double x) {
  if (x == 1.0) return 1.0;
  float xf = fminf(fmaxf((float)x, 1e-30f), 1e30f);
  double z = (double)__builtin_amdgcn_exp2f(-0.142857142857142857f * __builtin_amdgcn_logf(xf));
  const double k7 = 1.0 / 7.0;
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    double z2 = z * z;
    double z3 = z2 * z;
    double z7 = z3 * z3 * z;
    z = fma(z * k7, fma(-x, z7, 1.0), z);
  }
  return z;
}

// 1/x for normal positive or negative x: hardware estimate and two Newton steps
// (within an ulp of the correctly rounded quotient).
__device__ __forceinline__ double frcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// 1/sqrt(x) for normal positive x: hardware estimate and two Newton steps
// r <- r (3/2 - x r^2 / 2) (error e -> 3/2 e^2; within an ulp or two of the rounded value).
__device__ __forceinline__ double frsq(double x) {
  double r = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  r = r * fma(-h * r, r, 1.5);
  r = r * fma(-h * r, r, 1.5);
  return r;
}

struct GasC {
  double g, gm1, inv_gm1, g2m1, gm1_2g, gp1_2g, kshock, a2, half_gm1, inv_g, inv_gp1_2g, inv_a2;
  int max_iter;  // Newton iteration cap
};

__device__ __forceinline__ GasC gas_consts(double g, int max_iter = 50) {
  GasC c;
  c.max_iter = max_iter;
  c.g = g;
  c.gm1 = g - 1.0;
  c.inv_gm1 = 1.0 / (g - 1.0);
  c.g2m1 = 2.0 / (g - 1.0);
  c.gm1_2g = (g - 1.0) / (2.0 * g);
  c.gp1_2g = (g + 1.0) / (2.0 * g);
  c.kshock = (g - 1.0) / (g + 1.0);
  c.a2 = 2.0 / (g + 1.0);
  c.half_gm1 = 0.5 * (g - 1.0);
  c.inv_g = 1.0 / g;
  c.inv_gp1_2g = (2.0 * g) / (g + 1.0);
  c.inv_a2 = 0.5 * (g + 1.0);
  return c;
}

// Powers of x = p/p_K needed by the exact solver: x^((g-1)/2g), x^(-(g+1)/2g), x^(1/g).
// With g = 7/5 they are x^(1/7), x^(-6/7), x^(5/7), all from one x^(-1/7).
template <bool G75> struct Pow3 {
  double p17, pm67, p57;
  __device__ __forceinline__ Pow3(double x, const GasC& c) {
    if (G75) {
      double z = inv_root7(x);
      double z2 = z * z;
      double z6 = z2 * z2 * z2;
      p17 = x * z6;
      pm67 = z6;
      p57 = x * z2;
    } else {
      p17 = pow(x, c.gm1_2g);
      pm67 = pow(x, -c.gp1_2g);
      p57 = pow(x, 1.0 / c.g);
    }
  }
};

template <bool G75>
__device__ __forceinline__ double ipow_fan_rho(double ratio, const GasC& c) {
  if (G75) { double r2 = ratio * ratio; return r2 * r2 * ratio; }
  return pow(ratio, c.g2m1);
}
template <bool G75>
__device__ __forceinline__ double ipow_fan_p(double ratio, const GasC& c) {
  if (G75) { double r2 = ratio * ratio; double r3 = r2 * ratio; return r3 * r3 * ratio; }
  return pow(ratio, 2.0 * c.g / (c.g - 1.0));
}

// One side of the pressure function of the exact solver (Sect. 2.6) and its derivative.
// Per-side constants of the pressure function: A = 2/((g+1) rho), B = (g-1)/(g+1) p,
// 1/p and 1/(rho c).
struct Side {
  double r, u, p, c, A, B, ip, irc, iA;
};

// c and 1/c of the side come in as c2 * rs and rs, rs = 1/sqrt(c2)
__device__ __forceinline__ Side make_side(double r, double ir, double u, double p, double c,
                                          double rs, const GasC& g) {
  Side s;
  s.r = r; s.u = u; s.p = p; s.c = c;
  s.A = g.a2 * ir;
  s.B = g.kshock * p;
  s.ip = frcp(p);
  s.irc = ir * rs;
  s.iA = r * g.inv_a2;
  return s;
}

template <bool G75>
__device__ __forceinline__ void pfun(double p, const Side& K, const GasC& c, double& f,
                                     double& df) {
  if (p > K.p) {
    // q = sqrt(A / (p + B)) = 1/sqrt((p + B)/A) and 1/(p + B) = q^2 / A
    const double q = frsq((p + K.B) * K.iA);
    const double ipb = q * q * K.iA;
    f = (p - K.p) * q;
    df = q * (1.0 - 0.5 * (p - K.p) * ipb);
  } else {
    Pow3<G75> w(p * K.ip, c);
    f = c.g2m1 * K.c * (w.p17 - 1.0);
    df = w.pm67 * K.irc;
  }
}

struct TStat {
  int fall, vac, maxit, noconv, resolve;
  int last;  // Newton iterations of the latest gas solve (0: none was needed)
  int negd;  // dust densities that came out negative
};

// Wave pattern taken by the exact gas solver at x/t = 0 (kept by the adjoint, which
// differentiates the branch the primal solve took).
enum : int {
  GR_LEFT = 0,      // the left state
  GR_RIGHT,         // the right state
  GR_FAN_L,         // inside the left rarefaction fan
  GR_FAN_R,         // inside the right rarefaction fan
  GR_VACUUM,        // inside a vacuum region
  GR_STAR_L_SHOCK,  // left star state behind a shock
  GR_STAR_L_RARE,   // left star state behind a rarefaction
  GR_STAR_R_SHOCK,
  GR_STAR_R_RARE
};
struct GasRec {
  int branch;
  double ps, us;                 // star pressure and velocity (star branches)
  double rho, un, t1, t2, p;     // the sampled state
};

// Exact Riemann problem of the ideal gas sampled at x/t = 0 (Sect. 2.6): Newton on p*
// from the primitive-variable guess (relative change <= 1e-12, at most c.max_iter),
// star velocity, then the wave pattern at x/t = 0; tangential velocities come from the
// side of the contact.  Output: mass, normal momentum, two tangential momenta, energy.
template <bool G75, bool REC = false>
__device__ void gas_riemann(const GasC& c, double rL, double irL, double uL, double aL, double bL,
                            double pL, double rR, double irR, double uR, double aR, double bR,
                            double pR, double fl[5], TStat& st, GasRec* rec = nullptr) {
  const double du = uR - uL;
  const double c2L = c.g * pL * irL, c2R = c.g * pR * irR;
  // Supersonic faces.  With u_L >= c_L, let p_hi be the star pressure at which a left
  // shock would stand still, p_hi = (rho_L u_L^2 / g - (g-1)/(2g) p_L) (2g)/(g+1).  If
  // p_hi >= p_R then f_R(p_hi) >= 0, and f_L(p_hi) + du >= 0 gives f(p_hi) >= 0, so
  // p* <= p_hi (f increases): the left wave (rarefaction with head u_L - c_L >= 0, or shock
  // with speed >= 0) lies at x/t >= 0, and u* = u_L - f_L(p*) >= u_L - f_L(p_hi) >= 0: the
  // solution at x/t = 0 is the left state, which is what the full solve returns.  Both
  // tests are taken on squares (f_L(p_hi)^2 = (p_hi - p_L)^2 A_L / (p_hi + B_L)), so no
  // square root or division is needed; faces that may open a vacuum are left to the full
  // solve.  Mirror for u_R <= -c_R.
  {
    const double g2 = c.g2m1 * c.g2m1;
    const bool novac_L = du <= 0.0 || du * du < g2 * c2L;
    const bool novac_R = du <= 0.0 || du * du < g2 * c2R;
    if (uL > 0.0 && uL * uL >= c2L && novac_L) {
      const double u2 = uL * uL;
      const double phi = (rL * u2 * c.inv_g - c.gm1_2g * pL) * c.inv_gp1_2g;
      if (phi >= pR) {
        const double D = phi - pL;
        const double D2A = D * D * (c.a2 * irL);
        const double pb = phi + c.kshock * pL;
        if ((du >= 0.0 || D2A >= du * du * pb) && u2 * pb >= D2A) {
          if constexpr (REC) {
            rec->branch = GR_LEFT;
            rec->rho = rL; rec->un = uL; rec->t1 = aL; rec->t2 = bL; rec->p = pL;
          }
          st.last = 0;
          const double m0 = rL * uL;
          const double en = pL * c.inv_gm1 + 0.5 * rL * (uL * uL + aL * aL + bL * bL);
          fl[0] = m0; fl[1] = m0 * uL + pL; fl[2] = m0 * aL; fl[3] = m0 * bL; fl[4] = (en + pL) * uL;
          return;
        }
      }
    } else if (uR < 0.0 && uR * uR >= c2R && novac_R) {
      const double u2 = uR * uR;
      const double phi = (rR * u2 * c.inv_g - c.gm1_2g * pR) * c.inv_gp1_2g;
      if (phi >= pL) {
        const double D = phi - pR;
        const double D2A = D * D * (c.a2 * irR);
        const double pb = phi + c.kshock * pR;
        if ((du >= 0.0 || D2A >= du * du * pb) && u2 * pb >= D2A) {
          if constexpr (REC) {
            rec->branch = GR_RIGHT;
            rec->rho = rR; rec->un = uR; rec->t1 = aR; rec->t2 = bR; rec->p = pR;
          }
          st.last = 0;
          const double m0 = rR * uR;
          const double en = pR * c.inv_gm1 + 0.5 * rR * (uR * uR + aR * aR + bR * bR);
          fl[0] = m0; fl[1] = m0 * uR + pR; fl[2] = m0 * aR; fl[3] = m0 * bR; fl[4] = (en + pR) * uR;
          return;
        }
      }
    }
  }
  const double rsL = frsq(c2L), rsR = frsq(c2R);
  const double cL = c2L * rsL;
  const double cR = c2R * rsR;
  double rho, un, t1, t2, p;
  if (c.g2m1 * (cL + cR) <= du) {
    // vacuum between two rarefactions
    st.vac++;
    st.last = 0;
    double sHL = uL - cL, sSL = uL + c.g2m1 * cL, sSR = uR - c.g2m1 * cR, sHR = uR + cR;
    int br;
    if (0.0 <= sHL) { rho = rL; un = uL; t1 = aL; t2 = bL; p = pL; br = GR_LEFT; }
    else if (0.0 < sSL) {
      double cc = c.a2 * (cL + c.half_gm1 * uL);
      double ratio = cc / cL;
      rho = rL * ipow_fan_rho<G75>(ratio, c); un = cc; p = pL * ipow_fan_p<G75>(ratio, c);
      t1 = aL; t2 = bL; br = GR_FAN_L;
    } else if (0.0 <= sSR) { rho = 0.0; un = 0.0; t1 = 0.0; t2 = 0.0; p = 0.0; br = GR_VACUUM; }
    else if (0.0 < sHR) {
      double cc = c.a2 * (cR - c.half_gm1 * uR);
      double ratio = cc / cR;
      rho = rR * ipow_fan_rho<G75>(ratio, c); un = -cc; p = pR * ipow_fan_p<G75>(ratio, c);
      t1 = aR; t2 = bR; br = GR_FAN_R;
    } else { rho = rR; un = uR; t1 = aR; t2 = bR; p = pR; br = GR_RIGHT; }
    if constexpr (REC) rec->branch = br;
  } else {
    const Side L = make_side(rL, irL, uL, pL, cL, rsL, c);
    const Side R = make_side(rR, irR, uR, pR, cR, rsR, c);
    double ppv = 0.5 * (pL + pR) - 0.125 * du * (rL + rR) * (cL + cR);
    double ps = fmax(ppv, 1e-8 * fmin(pL, pR));
    int it = 0;
    bool conv = false;
    double fL = 0.0, dL = 1.0, fR = 0.0, dR = 1.0, dp = 0.0;
    while (it < c.max_iter) {
      ++it;
      pfun<G75>(ps, L, c, fL, dL);
      pfun<G75>(ps, R, c, fR, dR);
      double pn = ps - (fL + fR + du) / (dL + dR);
      if (pn < 1e-8 * ps) pn = 1e-8 * ps;
      dp = pn - ps;
      // relative change 2|dp|/(p_new + p_old) <= 1e-12, written without a division
      bool done = 2.0 * fabs(dp) <= 1e-12 * (pn + ps);
      ps = pn;
      if (done) { conv = true; break; }
    }
    st.maxit = max(st.maxit, it);
    st.last = it;
    if (!conv) st.noconv = 1;
    // star velocity at the converged p*: the last iterate's f and f' extrapolated over
    // the final (<= 1e-12 relative) Newton update; the neglected term is O(dp^2)
    double us = 0.5 * (uL + uR) + 0.5 * ((fR + dR * dp) - (fL + dL * dp));
    p = ps;
    int br;
    if (0.0 <= us) {
      t1 = aL; t2 = bL;
      if (ps > pL) {
        double q = ps * L.ip;
        double sL = uL - cL * sqrt(c.gp1_2g * q + c.gm1_2g);
        if (0.0 <= sL) { rho = rL; un = uL; p = pL; br = GR_LEFT; }
        else { rho = rL * (q + c.kshock) * frcp(c.kshock * q + 1.0); un = us; br = GR_STAR_L_SHOCK; }
      } else {
        double sHL = uL - cL;
        if (0.0 <= sHL) { rho = rL; un = uL; p = pL; br = GR_LEFT; }
        else {
          Pow3<G75> w(ps * L.ip, c);
          double sTL = us - cL * w.p17;
          if (0.0 > sTL) { rho = rL * w.p57; un = us; br = GR_STAR_L_RARE; }
          else {
            double cc = c.a2 * (cL + c.half_gm1 * uL);
            double ratio = cc / cL;
            rho = rL * ipow_fan_rho<G75>(ratio, c); un = cc; p = pL * ipow_fan_p<G75>(ratio, c);
            br = GR_FAN_L;
          }
        }
      }
    } else {
      t1 = aR; t2 = bR;
      if (ps > pR) {
        double q = ps * R.ip;
        double sR = uR + cR * sqrt(c.gp1_2g * q + c.gm1_2g);
        if (0.0 >= sR) { rho = rR; un = uR; p = pR; br = GR_RIGHT; }
        else { rho = rR * (q + c.kshock) * frcp(c.kshock * q + 1.0); un = us; br = GR_STAR_R_SHOCK; }
      } else {
        double sHR = uR + cR;
        if (0.0 >= sHR) { rho = rR; un = uR; p = pR; br = GR_RIGHT; }
        else {
          Pow3<G75> w(ps * R.ip, c);
          double sTR = us + cR * w.p17;
          if (0.0 <= sTR) { rho = rR * w.p57; un = us; br = GR_STAR_R_RARE; }
          else {
            double cc = c.a2 * (cR - c.half_gm1 * uR);
            double ratio = cc / cR;
            rho = rR * ipow_fan_rho<G75>(ratio, c); un = -cc; p = pR * ipow_fan_p<G75>(ratio, c);
            br = GR_FAN_R;
          }
        }
      }
    }
    if constexpr (REC) { rec->branch = br; rec->ps = ps; rec->us = us; }
  }
  if constexpr (REC) { rec->rho = rho; rec->un = un; rec->t1 = t1; rec->t2 = t2; rec->p = p; }
  double en = p * c.inv_gm1 + 0.5 * rho * (un * un + t1 * t1 + t2 * t2);
  double m = rho * un;
  fl[0] = m;
  fl[1] = m * un + p;
  fl[2] = m * t1;
  fl[3] = m * t2;
  fl[4] = (en + p) * un;
}

// Exact pressureless Riemann problem at x/t = 0 (Sect. 2.9): diverging or equal streams
// leave vacuum between them (upwind state or zero flux); converging streams form a
// delta shock of speed (sqrt(rho_L) u_L + sqrt(rho_R) u_R)/(sqrt(rho_L) + sqrt(rho_R)),
// the flux being the upwind one and the mean of both at a standing shock.  The sign
// of the shock speed is formed without contraction so that mirrored states give zero.
// With REC the side taken is stored in *rec: -1 left, +1 right, 0 mean, 2 no flux.
template <bool REC = false>
__device__ void dust_riemann(double rL, double uL, double aL, double bL, double rR, double uR,
                             double aR, double bR, double fl[4], int* rec = nullptr) {
#pragma clang fp contract(off)
  fl[0] = 0.0; fl[1] = 0.0; fl[2] = 0.0; fl[3] = 0.0;
  if constexpr (REC) *rec = 2;
  if (!(rL > 0.0)) { rL = 0.0; uL = 0.0; aL = 0.0; bL = 0.0; }
  if (!(rR > 0.0)) { rR = 0.0; uR = 0.0; aR = 0.0; bR = 0.0; }
  if (rL + rR == 0.0) return;
  int side;  // -1 left, +1 right, 0 mean
  if (uL <= uR) {
    if (uL > 0.0) side = -1;
    else if (uR < 0.0) side = 1;
    else return;
  } else {
    // delta shock: its speed has the sign of sqrt(rL) uL + sqrt(rR) uR.  With uL > uR,
    // both terms share a sign unless uL > 0 > uR, where the sign is that of
    // rL uL^2 - rR uR^2 (both sides squared, no square root); mirror-symmetric states
    // give exactly zero either way
    if (uR >= 0.0 && uL > 0.0) side = -1;
    else if (uL <= 0.0 && uR < 0.0) side = 1;
    else {
      const double d = rL * uL * uL - rR * uR * uR;
      side = d > 0.0 ? -1 : (d < 0.0 ? 1 : 0);
    }
  }
  if constexpr (REC) *rec = side;
  double mL = rL * uL, mR = rR * uR;
  if (side < 0) { fl[0] = mL; fl[1] = mL * uL; fl[2] = mL * aL; fl[3] = mL * bL; }
  else if (side > 0) { fl[0] = mR; fl[1] = mR * uR; fl[2] = mR * aR; fl[3] = mR * bR; }
  else {
    fl[0] = 0.5 * (mL + mR);
    fl[1] = 0.5 * (mL * uL + mR * uR);
    fl[2] = 0.5 * (mL * aL + mR * aR);
    fl[3] = 0.5 * (mL * bL + mR * bR);
  }
}

// normal / tangential velocity slots of direction DIR (0 r, 1 theta, 2 z)
template <int DIR> struct Dirs {
  static constexpr int n = DIR;
  static constexpr int t1 = DIR == 0 ? 1 : 0;
  static constexpr int t2 = DIR == 2 ? 1 : 2;
};

// ------------------------------------------------------------------------------------
// Face states and fluxes.  The parabola and MinMod limiter of Sect. 2.7 act on the
// primitive form of the variables: the gas velocity, pressure and density as deviations
// W' = W(E) - W(E0) from the stationary flow, each dust fluid's velocity and density
// whole.  A gas face state is W0(face) + W'(cell) + limited increment; only the flux of
// the Riemann solution, F* = F(E*), is formed from the face states (Sect. 2.6).

// Reconstructed gas face states, positivity fallback to the cell-centre state
// W0(cell) + W'(cell), exact Riemann problem, F* in field order.  Cells A, B | C, D along
// DIR (the face lies between B and C), given by their W' in field slots (u, v, w, P, rho);
// bf: the stationary flow at the face, bB / bC: at the centres of B and C (WB_N entries).
template <int DIR, bool G75>
__device__ __forceinline__ void gas_face(const GasC& c, const double* wA, const double* wB,
                                         const double* wC, const double* wD, const double* coB,
                                         const double* coC, const double* bf, const double* bB,
                                         const double* bC, double F[5], TStat& st) {
  double qL[5], qR[5];
#pragma unroll
  for (int f = 0; f < 5; ++f) {
    double iB, iC;
    if (DIR == 0) {
      iB = inc_up_c(wA[f], wB[f], wC[f], coB);
      iC = inc_lo_c(wB[f], wC[f], wD[f], coC);
    } else {
      iB = inc_up_u(wA[f], wB[f], wC[f]);
      iC = inc_lo_u(wB[f], wC[f], wD[f]);
    }
    qL[f] = bf[f] + (wB[f] + iB);
    qR[f] = bf[f] + (wC[f] + iC);
  }
  if (!(qL[4] > 0.0 && qL[3] > 0.0)) {
#pragma unroll
    for (int f = 0; f < 5; ++f) qL[f] = bB[f] + wB[f];
    st.fall++;
  }
  if (!(qR[4] > 0.0 && qR[3] > 0.0)) {
#pragma unroll
    for (int f = 0; f < 5; ++f) qR[f] = bC[f] + wC[f];
    st.fall++;
  }
  constexpr int N = Dirs<DIR>::n, T1 = Dirs<DIR>::t1, T2 = Dirs<DIR>::t2;
  double fl[5];
  gas_riemann<G75>(c, qL[4], frcp(qL[4]), qL[N], qL[T1], qL[T2], qL[3], qR[4], frcp(qR[4]), qR[N],
                   qR[T1], qR[T2], qR[3], fl, st);
  F[4] = fl[0];
  F[N] = fl[1];
  F[T1] = fl[2];
  F[T2] = fl[3];
  F[3] = fl[4];
}

// Dust face: velocity and density reconstructed whole (no stationary reference); a face
// density below zero falls back to the cell-centre state.
template <int DIR>
__device__ __forceinline__ void dust_face(const double* wA, const double* wB, const double* wC,
                                          const double* wD, const double* coB, const double* coC,
                                          double F[4], TStat& st) {
  double qL[4], qR[4];
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    double iB, iC;
    if (DIR == 0) {
      iB = inc_up_c(wA[f], wB[f], wC[f], coB);
      iC = inc_lo_c(wB[f], wC[f], wD[f], coC);
    } else {
      iB = inc_up_u(wA[f], wB[f], wC[f]);
      iC = inc_lo_u(wB[f], wC[f], wD[f]);
    }
    qL[f] = wB[f] + iB;
    qR[f] = wC[f] + iC;
  }
  if (qL[3] < 0.0) {
#pragma unroll
    for (int f = 0; f < 4; ++f) qL[f] = wB[f];
    st.fall++;
  }
  if (qR[3] < 0.0) {
#pragma unroll
    for (int f = 0; f < 4; ++f) qR[f] = wC[f];
    st.fall++;
  }
  constexpr int N = Dirs<DIR>::n, T1 = Dirs<DIR>::t1, T2 = Dirs<DIR>::t2;
  double fl[4];
  dust_riemann(qL[3], qL[N], qL[T1], qL[T2], qR[3], qR[N], qR[T1], qR[T2], fl);
  F[3] = fl[0];
  F[N] = fl[1];
  F[T1] = fl[2];
  F[T2] = fl[3];
}

}  // namespace rb

#include "rb_pert32.h"

namespace rb {

// FP32-perturbation gas face: reconstructed W' about the face's stationary flow, the
// perturbation Riemann problem and the flux change dF = F* - F(W0); faces the FP32 form
// cannot take (strong perturbation, transonic fan, no convergence, non-positive face
// state) are re-solved in FP64 on the full states.
template <int DIR>
__device__ __forceinline__ void gas_face_p32(const GasC& c, const float* wA, const float* wB,
                                             const float* wC, const float* wD, const double* coB,
                                             const double* coC, const double* bf,
                                             const double* bB, const double* bC, float F[5],
                                             TStat& st) {
  float qL[5], qR[5];
#pragma unroll
  for (int f = 0; f < 5; ++f) {
    float iB, iC;
    if (DIR == 0) {
      iB = inc_up_c<float>(wA[f], wB[f], wC[f], coB);
      iC = inc_lo_c<float>(wB[f], wC[f], wD[f], coC);
    } else {
      iB = inc_up_u<float>(wA[f], wB[f], wC[f]);
      iC = inc_lo_u<float>(wB[f], wC[f], wD[f]);
    }
    qL[f] = wB[f] + iB;
    qR[f] = wC[f] + iC;
  }
  constexpr int N = Dirs<DIR>::n, T1 = Dirs<DIR>::t1, T2 = Dirs<DIR>::t2;
  const BgW b = bg_face<DIR>(bf);
  const PW L = {qL[4], qL[N], qL[T1], qL[T2], qL[3]};
  const PW R = {qR[4], qR[N], qR[T1], qR[T2], qR[3]};
  const bool okL = (b.rho + (double)L.rho > 0.0) && (b.p + (double)L.p > 0.0);
  const bool okR = (b.rho + (double)R.rho > 0.0) && (b.p + (double)R.p > 0.0);
  PW W;
  float fl[5];
  if (okL && okR && riemann_pert(b, L, R, c, W, st)) {
    flux_pert(b, W, (float)c.inv_gm1, fl);
  } else {
    st.resolve++;
    double xL[5], xR[5];
#pragma unroll
    for (int f = 0; f < 5; ++f) {
      xL[f] = okL ? bf[f] + (double)qL[f] : bB[f] + (double)wB[f];
      xR[f] = okR ? bf[f] + (double)qR[f] : bC[f] + (double)wC[f];
    }
    if (!okL) st.fall++;
    if (!okR) st.fall++;
    double f64[5];
    gas_riemann<true>(c, xL[4], frcp(xL[4]), xL[N], xL[T1], xL[T2], xL[3], xR[4], frcp(xR[4]),
                      xR[N], xR[T1], xR[T2], xR[3], f64, st);
    const double m0 = b.rho * b.un;
    fl[0] = (float)(f64[0] - m0);
    fl[1] = (float)(f64[1] - (m0 * b.un + b.p));
    fl[2] = (float)(f64[2] - m0 * b.t1);
    fl[3] = (float)(f64[3] - m0 * b.t2);
    fl[4] = (float)(f64[4] - b.h * b.un);
  }
  F[4] = fl[0];
  F[N] = fl[1];
  F[T1] = fl[2];
  F[T2] = fl[3];
  F[3] = fl[4];
}

// ------------------------------------------------------------------------------------
// state access with ghost cells (Sect. 2.4): r and z ghosts come from tables, theta wraps

// FP32-perturbation storage layout: the gas deviation E' (5 fields) and each dust
// species' velocity as a deviation from the stationary flow's velocity at the cell centre
// (3 per species; that velocity is azimuthal, App. A, so only the theta component
// differs) in FP32, then the dust densities in FP64 (mass is accumulated in FP64).
// f64_base: first double of that part.  A dust momentum is read as density x (stationary
// velocity + stored deviation); it is stored as momentum / density - stationary velocity
// after the cell's new density, which must therefore be written first (zero deviation
// where the density is below 1e-300; the velocity of a cell without dust reads as zero).
__device__ __forceinline__ size_t p32_f64_base(const Geo& g) {
  return (((size_t)(5 + 3 * g.nd) * g.N + 63) / 64 * 64) / 2;
}

// interior conservative value of field f (FP64 storage: the gas deviation E' and the dust
// variables; or the FP32-perturbation layout above)
template <bool P32>
__device__ __forceinline__ double ld_cell(const StageArgs& a, const void* st, int f, int k, int i,
                                          size_t cell) {
  const Geo& g = a.g;
  if (P32) {
    if (f < 5) return (double)((const float*)st)[(size_t)f * g.N + cell];
    const int sp = (f - 5) >> 2, c = (f - 5) & 3;
    const double rd = ((const double*)st)[p32_f64_base(g) + (size_t)sp * g.N + cell];
    if (c == 3) return rd;
    const double u0 = c == 1 ? a.t.wc[((size_t)k * g.nr + i) * WB_N + WB_V] : 0.0;
    return rd * (u0 + (double)((const float*)st)[(size_t)(5 + 3 * sp + c) * g.N + cell]);
  }
  return ((const double*)st)[(size_t)f * g.N + cell];
}

template <bool P32>
__device__ __forceinline__ void st_cell(const StageArgs& a, void* st, int f, int k, int i,
                                        size_t cell, double v) {
  const Geo& g = a.g;
  if (P32) {
    if (f < 5) { ((float*)st)[(size_t)f * g.N + cell] = (float)v; return; }
    const int sp = (f - 5) >> 2, c = (f - 5) & 3;
    double* dens = (double*)st + p32_f64_base(g) + (size_t)sp * g.N + cell;
    if (c == 3) { *dens = v; return; }
    const double rd = *dens;  // the new density, written before the momenta
    const double u0 = c == 1 ? a.t.wc[((size_t)k * g.nr + i) * WB_N + WB_V] : 0.0;
    ((float*)st)[(size_t)(5 + 3 * sp + c) * g.N + cell] = rd > 1e-300 ? (float)(v * frcp(rd) - u0) : 0.0f;
  } else {
    ((double*)st)[(size_t)f * g.N + cell] = v;
  }
}

// A whole dust cell (momenta r, theta, z, density) into the FP32 layout from registers:
// the density, then the velocity deviations formed with it (the same values st_cell
// stores field by field, without reading the density back); v0 is the stationary
// azimuthal velocity of the cell
__device__ __forceinline__ void st_dust32(const StageArgs& a, void* st, int sp, size_t cell,
                                          const double v[4], double v0) {
  const Geo& g = a.g;
  ((double*)st)[p32_f64_base(g) + (size_t)sp * g.N + cell] = v[3];
  const double ir = v[3] > 1e-300 ? frcp(v[3]) : 0.0;
  float* vel = (float*)st + (size_t)(5 + 3 * sp) * g.N + cell;
  const bool full = v[3] > 1e-300;
  vel[0] = full ? (float)(v[0] * ir) : 0.0f;
  vel[g.N] = full ? (float)(v[1] * ir - v0) : 0.0f;
  vel[2 * g.N] = full ? (float)(v[2] * ir) : 0.0f;
}

// All NG conservative fields of a group at an interior cell: the gas deviation E', the
// dust momenta and density.
template <bool P32, int NG>
__device__ __forceinline__ void load_cons(const StageArgs& a, const void* st, int F0, int k, int i,
                                          int j, double* out) {
  const Geo& g = a.g;
  const size_t cell = ((size_t)k * g.nr + i) * g.nth + j;
  if constexpr (P32 && NG == 4) {
    const int sp = (F0 - 5) >> 2;
    const double rd = ((const double*)st)[p32_f64_base(g) + (size_t)sp * g.N + cell];
    const float* vel = (const float*)st + (size_t)(5 + 3 * sp) * g.N + cell;
    const double v0 = a.t.wc[((size_t)k * g.nr + i) * WB_N + WB_V];
    out[0] = rd * (double)vel[0];
    out[1] = rd * (v0 + (double)vel[g.N]);
    out[2] = rd * (double)vel[2 * g.N];
    out[3] = rd;
    return;
  }
#pragma unroll
  for (int f = 0; f < NG; ++f) out[f] = ld_cell<P32>(a, st, F0 + f, k, i, cell);
}

// Gas deviation W' = W(E0 + E') - W(E0) of a cell from its conservative deviation e and
// its stationary flow b (WB_N entry), free of cancellation: rho' = e_rho,
// u' = (m' - u0 rho') / rho, P' = (g - 1)(E' - dKE) with the kinetic-energy change
// dKE = rho' |u0|^2 / 2 + rho u0.u' + rho |u'|^2 / 2.  Exactly zero for e = 0; for the Sod
// annulus (b = 0) it is the state's own primitives.
__device__ __forceinline__ void cell_w(const double* e, const double* b, double gm1, double* w) {
  const double rp = e[4];
  const double rho = b[WB_RHO] + rp;
  const double ir = frcp(rho);
  const double u0 = b[WB_U], v0 = b[WB_V], w0 = b[WB_W];
  const double up = (e[0] - u0 * rp) * ir, vp = (e[1] - v0 * rp) * ir, wp = (e[2] - w0 * rp) * ir;
  const double dke = 0.5 * rp * (u0 * u0 + v0 * v0 + w0 * w0) + rho * (u0 * up + v0 * vp + w0 * wp) +
                     0.5 * rho * (up * up + vp * vp + wp * wp);
  w[0] = up; w[1] = vp; w[2] = wp;
  w[3] = gm1 * (e[3] - dke);
  w[4] = rp;
}
__device__ __forceinline__ void cell_w(const float* e, const double* b, float gm1, float* w) {
  const float rp = e[4];
  const float rho = (float)(b[WB_RHO] + (double)rp);
  const float ir = rcp32(rho);
  const float u0 = (float)b[WB_U], v0 = (float)b[WB_V], w0 = (float)b[WB_W];
  const float u0sq = (float)(b[WB_U] * b[WB_U] + b[WB_V] * b[WB_V] + b[WB_W] * b[WB_W]);
  const float up = (e[0] - u0 * rp) * ir, vp = (e[1] - v0 * rp) * ir, wp = (e[2] - w0 * rp) * ir;
  const float dke = 0.5f * rp * u0sq + rho * (u0 * up + v0 * vp + w0 * wp) +
                    0.5f * rho * (up * up + vp * vp + wp * wp);
  w[0] = up; w[1] = vp; w[2] = wp;
  w[3] = gm1 * (e[3] - dke);
  w[4] = rp;
}

// Reconstructed variables of a group at any cell, interior or ghost: the gas W', or the
// dust velocity (zero where the density is not positive) and density.  EXT: the optional
// boundary options may be active (outflow z ghosts carry the boundary cell's gas
// deviation E' scaled by the ratio of the stationary densities, and its dust variables);
// the base instantiation compiles them out.
template <bool P32, bool EXT, int NG, class T>
__device__ __forceinline__ void load_recon(const StageArgs& a, const void* st, int F0, int k,
                                           int i, int j, T* out) {
  const Geo& g = a.g;
  constexpr bool GAS = NG == 5;
  int kc = k;             // interior cell whose data are read
  double scale = 1.0;     // outflow: gas deviation scale
  const double* bw = nullptr;
  if (k < 0 || k >= g.nz) {
    const int ii = min(max(i, 0), g.nr - 1);
    const int side = k < 0 ? 0 : 1;
    const int layer = min(k < 0 ? -1 - k : k - g.nz, 1);
    if (!(EXT && g.bc_z == 1)) {
      const double* gt = a.t.ghz + ((size_t)(side * 2 + layer) * g.nr + ii) * g.nf + F0;
#pragma unroll
      for (int f = 0; f < NG; ++f) out[f] = (T)gt[f];
      return;
    }
    kc = k < 0 ? 0 : g.nz - 1;
    i = ii;
    scale = a.t.ozr[(size_t)(side * 2 + layer) * g.nr + ii];
    bw = a.t.ghzw + ((size_t)(side * 2 + layer) * g.nr + ii) * WB_N;
  } else if (i < 0 || i >= g.nr) {
    const int side = i < 0 ? 0 : 1;
    const int layer = min(i < 0 ? -1 - i : i - g.nr, 1);
    const double* gt = a.t.ghr + ((size_t)(side * 2 + layer) * g.nz + k) * g.nf + F0;
#pragma unroll
    for (int f = 0; f < NG; ++f) out[f] = (T)gt[f];
    return;
  }
  const size_t cell = ((size_t)kc * g.nr + i) * g.nth + j;
  if constexpr (GAS) {
    if (!bw) bw = a.t.wc + ((size_t)kc * g.nr + i) * WB_N;
    if constexpr (std::is_same<T, float>::value && P32) {
      float e[5];
#pragma unroll
      for (int f = 0; f < 5; ++f) e[f] = ((const float*)st)[(size_t)f * g.N + cell];
      if (EXT && scale != 1.0) {
#pragma unroll
        for (int f = 0; f < 5; ++f) e[f] = (float)((double)e[f] * scale);
      }
      cell_w(e, bw, (float)(g.gamma - 1.0), out);
    } else {
      double e[5], w[5];
#pragma unroll
      for (int f = 0; f < 5; ++f) e[f] = ld_cell<P32>(a, st, f, kc, i, cell) * scale;
      cell_w(e, bw, g.gamma - 1.0, w);
#pragma unroll
      for (int f = 0; f < 5; ++f) out[f] = (T)w[f];
    }
  } else {
    const int sp = (F0 - 5) >> 2;
    if constexpr (P32) {
      // the FP32 layout stores the dust velocity deviations from the stationary flow
      // (all requested before the density decides: a load made conditional on it would wait)
      const float* vel = (const float*)st + (size_t)(5 + 3 * sp) * g.N + cell;
      const double v0 = a.t.wc[((size_t)kc * g.nr + i) * WB_N + WB_V];
      const double rd = ((const double*)st)[p32_f64_base(g) + (size_t)sp * g.N + cell];
      const float v[3] = {vel[0], vel[g.N], vel[2 * g.N]};
      const bool full = rd > 0.0;
      out[0] = full ? (T)v[0] : T(0);
      out[1] = full ? (T)(v0 + (double)v[1]) : T(0);
      out[2] = full ? (T)v[2] : T(0);
      out[3] = (T)rd;
    } else {
      const double* d = (const double*)st + (size_t)F0 * g.N + cell;
      const double rd = d[3 * g.N];
      const double id = rd > 0.0 ? 1.0 / rd : 0.0;
      out[0] = (T)(d[0] * id);
      out[1] = (T)(d[g.N] * id);
      out[2] = (T)(d[2 * g.N] * id);
      out[3] = (T)rd;
    }
  }
}

// A dust cell's reconstructed variables in two steps: dust_fetch issues the loads and does
// no arithmetic on what they return, dust_finish forms the variables (the same values as
// load_recon).  A wavefront waits for a load where its result is first used, so a fetch
// made a phase or a plane ahead of its finish keeps that wait off the critical path.
// Ghost cells carry their table values in d; interior cells carry the stored fields (FP64
// layout: momenta and density in d) or (FP32 layout) the density in d[3], the stationary
// azimuthal velocity in d[1] and the stored velocity deviations in v.
template <bool P32>
struct DustRaw {
  double d[4];
  float v[P32 ? 3 : 1];
  bool ghost;
};
template <bool P32, bool EXT>
__device__ __forceinline__ void dust_fetch(const StageArgs& a, const void* st, int F0, int k, int i,
                                           int j, DustRaw<P32>& R) {
  // the same loads on every path, from addresses chosen by selects (loads on separate
  // branches land in separate registers, and the copy that merges them waits for them)
  const Geo& g = a.g;
  const double* gt = nullptr;  // the ghost table row, if the cell is a ghost
  int kc = k;
  if (k < 0 || k >= g.nz) {
    const int ii = min(max(i, 0), g.nr - 1);
    if (!(EXT && g.bc_z == 1)) {
      const int side = k < 0 ? 0 : 1;
      const int layer = min(k < 0 ? -1 - k : k - g.nz, 1);
      gt = a.t.ghz + ((size_t)(side * 2 + layer) * g.nr + ii) * g.nf + F0;
    }
    kc = k < 0 ? 0 : g.nz - 1;  // outflow: the boundary cell's dust variables
  } else if (i < 0 || i >= g.nr) {
    const int side = i < 0 ? 0 : 1;
    const int layer = min(i < 0 ? -1 - i : i - g.nr, 1);
    gt = a.t.ghr + ((size_t)(side * 2 + layer) * g.nz + k) * g.nf + F0;
  }
  const int ic = min(max(i, 0), g.nr - 1);  // a valid cell for the loads a ghost ignores
  const bool gh = gt != nullptr;
  R.ghost = gh;
  const size_t cell = ((size_t)kc * g.nr + ic) * g.nth + j;
  if constexpr (P32) {
    const int sp = (F0 - 5) >> 2;
    const float* vel = (const float*)st + (size_t)(5 + 3 * sp) * g.N + cell;
    const double* v0 = a.t.wc + ((size_t)kc * g.nr + ic) * WB_N + WB_V;
    const double* rd = (const double*)st + p32_f64_base(g) + (size_t)sp * g.N + cell;
    const double* p0 = gh ? gt : v0;
    const double* p1 = gh ? gt + 1 : v0;
    const double* p2 = gh ? gt + 2 : v0;
    const double* p3 = gh ? gt + 3 : rd;
    R.d[0] = *p0;
    R.d[1] = *p1;
    R.d[2] = *p2;
    R.d[3] = *p3;
    R.v[0] = vel[0];
    R.v[1] = vel[g.N];
    R.v[2] = vel[2 * (size_t)g.N];
  } else {
    const double* d = (const double*)st + (size_t)F0 * g.N + cell;
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      const double* p = gh ? gt + f : d + (size_t)f * g.N;
      R.d[f] = *p;
    }
  }
}
// The same two steps for a gas cell in the FP32-perturbation layout (base boundary
// options): the stored deviations e and the cell's stationary density and azimuthal
// velocity (the form runs on the disc background, whose stationary flow has no radial or
// vertical velocity).  Ghost cells (tiles at the radial boundaries, the last planes) are
// formed at once.
struct GasRaw32 {
  double rho0, v0;
  float e[5];
  bool ghost;
};
__device__ __forceinline__ void gas_fetch32(const StageArgs& a, const void* st, int k, int i, int j,
                                            GasRaw32& R) {
  const Geo& g = a.g;
  const double* gt = nullptr;
  if (k < 0 || k >= g.nz) {
    const int ii = min(max(i, 0), g.nr - 1);
    const int side = k < 0 ? 0 : 1;
    const int layer = min(k < 0 ? -1 - k : k - g.nz, 1);
    gt = a.t.ghz + ((size_t)(side * 2 + layer) * g.nr + ii) * g.nf;
  } else if (i < 0 || i >= g.nr) {
    const int side = i < 0 ? 0 : 1;
    const int layer = min(i < 0 ? -1 - i : i - g.nr, 1);
    gt = a.t.ghr + ((size_t)(side * 2 + layer) * g.nz + k) * g.nf;
  }
  R.ghost = gt != nullptr;
  if (gt) {
#pragma unroll
    for (int f = 0; f < 5; ++f) R.e[f] = (float)gt[f];
  } else {
    const size_t cell = ((size_t)k * g.nr + i) * g.nth + j;
    const double* bw = a.t.wc + ((size_t)k * g.nr + i) * WB_N;
#pragma unroll
    for (int f = 0; f < 5; ++f) R.e[f] = ((const float*)st)[(size_t)f * g.N + cell];
    R.rho0 = bw[WB_RHO];
    R.v0 = bw[WB_V];
  }
}
__device__ __forceinline__ void gas_finish32(const GasRaw32& R, float gm1, float* out) {
  double bw[WB_N];
  bw[WB_RHO] = R.rho0;
  bw[WB_U] = 0.0;
  bw[WB_V] = R.v0;
  bw[WB_W] = 0.0;
  float w[5];
  cell_w(R.e, bw, gm1, w);
#pragma unroll
  for (int f = 0; f < 5; ++f) out[f] = R.ghost ? R.e[f] : w[f];
}
template <bool P32>
__device__ __forceinline__ void dust_finish(const DustRaw<P32>& R, double* out) {
  const double rd = R.d[3];
  const bool full = rd > 0.0;
  if constexpr (P32) {
    out[0] = R.ghost ? R.d[0] : (full ? (double)R.v[0] : 0.0);
    out[1] = R.ghost ? R.d[1] : (full ? R.d[1] + (double)R.v[1] : 0.0);
    out[2] = R.ghost ? R.d[2] : (full ? (double)R.v[2] : 0.0);
  } else {
    const double id = full ? 1.0 / rd : 0.0;
#pragma unroll
    for (int f = 0; f < 3; ++f) out[f] = R.ghost ? R.d[f] : R.d[f] * id;
  }
  out[3] = rd;
}

// stationary-flow primitives (WB_N entry) of an interior cell or of the ghost next to the
// boundary (the face-state fallback's cell-centre state is this plus the cell's W')
__device__ __forceinline__ const double* bg_ptr(const StageArgs& a, int k, int i) {
  const Geo& g = a.g;
  if (k < 0 || k >= g.nz) {
    const int ii = min(max(i, 0), g.nr - 1);
    return a.t.ghzw + ((size_t)(k < 0 ? 0 : 2) * g.nr + ii) * WB_N;
  }
  if (i < 0 || i >= g.nr) return a.t.ghrw + ((size_t)(i < 0 ? 0 : 2) * g.nz + k) * WB_N;
  return a.t.wc + ((size_t)k * g.nr + i) * WB_N;
}

__device__ __forceinline__ const double* rco_ptr(const StageArgs& a, int i) {
  int c = min(max(i, -1), a.g.nr);
  return a.t.rco + (size_t)(c + 1) * RC_N;
}

__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ int wave_isum(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ int wave_imax(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

// Inverse dust stopping time of species s in a cell whose gas has density rho and
// pressure p (Sect. 2.9).  Law 0: Omega_K / St.  Law 1: Epstein 1/t = rho c_s / (rho_s r_p)
// with the isothermal c_s = sqrt(p / rho), i.e. sqrt(p rho) / (rho_s r_p); in the Stokes
// regime (r_p > 9 lambda / 4, lambda = mfp / rho) the Epstein rate times 9 lambda / (4 r_p).
template <bool EXT = true>
__device__ __forceinline__ double inv_tstop(const Geo& g, int s, double omk, double rho, double p) {
  if (!EXT || g.drag_law == 0) return omk * g.inv_st[s];
  const double ie = sqrt(p * rho) * g.inv_mp[s];
  const double x = g.rp94[s] * rho;
  return x <= g.mfp ? ie : ie * g.mfp / x;
}

// XCD-aware tile order: workgroup b is dispatched to XCD b % 8; give every XCD a
// contiguous range of tiles so that halo re-reads hit its own L2.
__device__ __forceinline__ int xcd_tile(int b, int nblk) {
  int q = nblk >> 3, rem = nblk & 7, x = b & 7;
  return x * q + min(x, rem) + (b >> 3);
}

}  // namespace rb
