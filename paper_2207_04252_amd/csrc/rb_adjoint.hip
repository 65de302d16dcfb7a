// Discrete adjoint of the RK2 stage operator on gfx950 (FP64).
//
// A stage is E_out = base + c dt V^-1 (G(E) - R0).  Given a cotangent lambda of E_out,
// the kernels here form J_G(E)^T w with w = c dt V^-1 lambda: the reverse of every
// face flux -- the exact Riemann solution differentiated on the wave pattern the
// primal solve took (star pressure by implicit differentiation of the pressure-function
// equation, Sect. 2.6), the limited parabolic reconstruction on the limiter branch taken
// (Sect. 2.7), the positivity fallback on the side it was taken -- scattered back to the
// four cells of each face stencil, plus the cell-local reverse of the geometric and
// gravity sources and of the gas-dust drag (Sect. 2.9, App. B).  The primal face
// solves are recomputed with the forward solver itself (recording variant), so every
// branch decision is the forward run's.
//
// k_adj_plane follows the forward stage kernel's tiles: a workgroup owns a 64 (theta) x
// 8 (r) tile and a chunk of z planes.  Each plane is staged in LDS with a three-cell halo
// (a cell receives contributions from the faces 3/2 cells away); the contributions of
// the theta and r faces to the tile's cells are accumulated in LDS in a fixed order, one
// phase per stencil position, so results are deterministic.  k_adj_z then marches every
// column upwards in registers and adds the z faces' contributions, each cell's in the
// order of its faces.
#include <algorithm>

#include "rb_device.h"

namespace rb {

// ------------------------------------------------------------------------------------
// reverse of the building blocks

// which argument minmod3 returned: 0 the first, 1 the second, 2 the third, 3 none (zero)
__device__ __forceinline__ int minmod3_arg(double x, double y, double z) {
  if (x > 0.0 && y > 0.0 && z > 0.0) return x <= fmin(y, z) ? 0 : (y <= z ? 1 : 2);
  if (x < 0.0 && y < 0.0 && z < 0.0) return x >= fmax(y, z) ? 0 : (y >= z ? 1 : 2);
  return 3;
}

// Derivative (cm, cp) of a limited face increment with respect to the backward and
// forward differences dm = e0 - em, dp = ep - e0, on the branch the limiter took (the
// arguments are the forward increments' own expressions).
__device__ __forceinline__ void dinc_up_u(double em, double e0, double ep, double& cm, double& cp) {
  const double dm = e0 - em, dp = ep - e0;
  switch (minmod3_arg(fma(3.0, dp, dm) * 0.125, dm, dp)) {
    case 0: cm = 0.125; cp = 0.375; break;
    case 1: cm = 1.0; cp = 0.0; break;
    case 2: cm = 0.0; cp = 1.0; break;
    default: cm = 0.0; cp = 0.0;
  }
}
__device__ __forceinline__ void dinc_lo_u(double em, double e0, double ep, double& cm, double& cp) {
  const double dm = e0 - em, dp = ep - e0;
  switch (minmod3_arg(-(fma(3.0, dm, dp) * 0.125), -dm, -dp)) {
    case 0: cm = -0.375; cp = -0.125; break;
    case 1: cm = -1.0; cp = 0.0; break;
    case 2: cm = 0.0; cp = -1.0; break;
    default: cm = 0.0; cp = 0.0;
  }
}
__device__ __forceinline__ void dinc_up_c(double em, double e0, double ep, const double* co,
                                          double& cm, double& cp) {
  const double dm = e0 - em, dp = ep - e0;
  switch (minmod3_arg(fma(co[RC_WPP], dp, co[RC_WPM] * dm), co[RC_LPM] * dm, co[RC_LPP] * dp)) {
    case 0: cm = co[RC_WPM]; cp = co[RC_WPP]; break;
    case 1: cm = co[RC_LPM]; cp = 0.0; break;
    case 2: cm = 0.0; cp = co[RC_LPP]; break;
    default: cm = 0.0; cp = 0.0;
  }
}
__device__ __forceinline__ void dinc_lo_c(double em, double e0, double ep, const double* co,
                                          double& cm, double& cp) {
  const double dm = e0 - em, dp = ep - e0;
  switch (minmod3_arg(fma(co[RC_WMP], dp, co[RC_WMM] * dm), co[RC_LMM] * dm, co[RC_LMP] * dp)) {
    case 0: cm = co[RC_WMM]; cp = co[RC_WMP]; break;
    case 1: cm = co[RC_LMM]; cp = 0.0; break;
    case 2: cm = 0.0; cp = co[RC_LMP]; break;
    default: cm = 0.0; cp = 0.0;
  }
}

// One side's pressure function at p and its partial derivatives: df/dp, and df/drho_K,
// df/dp_K at fixed p (shock: f = (p - p_K) sqrt(A/(p + B)); rarefaction:
// f = 2 c_K/(g-1) ((p/p_K)^((g-1)/2g) - 1)).
struct PD {
  double f, df, fr, fp;
};
template <bool G75>
__device__ __forceinline__ PD pfun_pd(double p, double rK, double pK, double cK, const GasC& c) {
  PD o;
  if (p > pK) {
    const double ipb = 1.0 / (p + c.kshock * pK);
    const double q = sqrt(c.a2 / rK * ipb);
    o.f = (p - pK) * q;
    o.df = q * (1.0 - 0.5 * (p - pK) * ipb);
    o.fr = -0.5 * o.f / rK;
    o.fp = -q - 0.5 * o.f * c.kshock * ipb;
  } else {
    Pow3<G75> w(p / pK, c);
    o.f = c.g2m1 * cK * (w.p17 - 1.0);
    o.df = w.pm67 / (rK * cK);
    o.fr = -0.5 * o.f / rK;
    o.fp = 0.5 * o.f / pK - cK * w.p17 / (c.g * pK);
  }
  return o;
}

// Reverse of F(W) for the sampled primitive state W = (rho, un, t1, t2, p); flb in the
// order mass, normal momentum, two tangential momenta, energy.  Output: W cotangent.
__device__ __forceinline__ void flux_rev(const GasC& c, const GasRec& w, const double flb[5],
                                         double Wb[5]) {
  const double m = w.rho * w.un;
  const double ke = 0.5 * (w.un * w.un + w.t1 * w.t1 + w.t2 * w.t2);
  const double en = w.p * c.inv_gm1 + w.rho * ke;
  const double mb = flb[0] + flb[1] * w.un + flb[2] * w.t1 + flb[3] * w.t2;
  const double enb = flb[4] * w.un;
  Wb[0] = enb * ke + mb * w.un;
  Wb[1] = flb[1] * m + flb[4] * (en + w.p) + enb * w.rho * w.un + mb * w.rho;
  Wb[2] = flb[2] * m + enb * w.rho * w.t1;
  Wb[3] = flb[3] * m + enb * w.rho * w.t2;
  Wb[4] = flb[1] + flb[4] * w.un + enb * c.inv_gm1;
}

// Reverse of the Riemann solution at x/t = 0 on the recorded wave pattern: W cotangent
// -> cotangents of the primitive face states WL, WR (rho, un, t1, t2, p).  The star
// state depends on the face states directly and through p*, u*:
//   f_L(p*) + f_R(p*) + u_R - u_L = 0,  u* = (u_L + u_R)/2 + (f_R(p*) - f_L(p*))/2.
template <bool G75>
__device__ void riemann_rev(const GasC& c, const double* WL, const double* WR, const GasRec& rec,
                            const double* Wb, double* WLb, double* WRb) {
#pragma unroll
  for (int q = 0; q < 5; ++q) { WLb[q] = 0.0; WRb[q] = 0.0; }
  const int br = rec.branch;
  if (br == GR_LEFT) {
#pragma unroll
    for (int q = 0; q < 5; ++q) WLb[q] = Wb[q];
    return;
  }
  if (br == GR_RIGHT) {
#pragma unroll
    for (int q = 0; q < 5; ++q) WRb[q] = Wb[q];
    return;
  }
  if (br == GR_VACUUM) return;
  if (br == GR_FAN_L || br == GR_FAN_R) {
    // inside a fan: c_c = 2/(g+1) (c_K +- (g-1)/2 u_K), rho = rho_K (c_c/c_K)^(2/(g-1)),
    // p = p_K (c_c/c_K)^(2g/(g-1)), un = +-c_c
    const bool left = br == GR_FAN_L;
    const double* W = left ? WL : WR;
    double* Wk = left ? WLb : WRb;
    const double sg = left ? 1.0 : -1.0;
    const double rK = W[0], uK = W[1], pK = W[4];
    const double cK = sqrt(c.g * pK / rK);
    const double cc = c.a2 * (cK + sg * c.half_gm1 * uK);
    const double ratio = cc / cK;
    const double e1 = c.g2m1, e2 = 2.0 * c.g / (c.g - 1.0);
    const double r1 = pow(ratio, e1 - 1.0), r2 = pow(ratio, e2 - 1.0);
    const double ratb = Wb[0] * rK * e1 * r1 + Wb[4] * pK * e2 * r2;
    Wk[0] += Wb[0] * r1 * ratio;
    Wk[4] += Wb[4] * r2 * ratio;
    const double ccb = sg * Wb[1] + ratb / cK;
    const double cKb = -ratb * cc / (cK * cK) + c.a2 * ccb;
    Wk[1] += sg * c.a2 * c.half_gm1 * ccb;
    Wk[4] += cKb * cK / (2.0 * pK);
    Wk[0] -= cKb * cK / (2.0 * rK);
    Wk[2] += Wb[2];
    Wk[3] += Wb[3];
    return;
  }
  // star states
  const bool left = br == GR_STAR_L_SHOCK || br == GR_STAR_L_RARE;
  const double* W = left ? WL : WR;
  double* Wk = left ? WLb : WRb;
  const double ps = rec.ps;
  double psb = Wb[4];
  const double usb = Wb[1];
  Wk[2] += Wb[2];
  Wk[3] += Wb[3];
  const double rK = W[0], pK = W[4];
  if (br == GR_STAR_L_SHOCK || br == GR_STAR_R_SHOCK) {
    // rho* = rho_K (q + k)/(k q + 1), q = p*/p_K, k = (g-1)/(g+1)
    const double q = ps / pK, k = c.kshock, den = k * q + 1.0;
    Wk[0] += Wb[0] * (q + k) / den;
    const double qb = Wb[0] * rK * (1.0 - k * k) / (den * den);
    psb += qb / pK;
    Wk[4] -= qb * q / pK;
  } else {
    // rho* = rho_K (p*/p_K)^(1/g)
    const double rho = rec.rho;
    Wk[0] += Wb[0] * rho / rK;
    psb += Wb[0] * rho / (c.g * ps);
    Wk[4] -= Wb[0] * rho / (c.g * pK);
  }
  const double cL = sqrt(c.g * WL[4] / WL[0]), cR = sqrt(c.g * WR[4] / WR[0]);
  const PD L = pfun_pd<G75>(ps, WL[0], WL[4], cL, c);
  const PD R = pfun_pd<G75>(ps, WR[0], WR[4], cR, c);
  // u*
  WLb[1] += 0.5 * usb;
  WRb[1] += 0.5 * usb;
  psb += 0.5 * usb * (R.df - L.df);
  WRb[0] += 0.5 * usb * R.fr;
  WRb[4] += 0.5 * usb * R.fp;
  WLb[0] -= 0.5 * usb * L.fr;
  WLb[4] -= 0.5 * usb * L.fp;
  // p*: dp* = -(dPhi) / (f_L' + f_R')
  const double s = psb / (L.df + R.df);
  WLb[1] += s;
  WRb[1] -= s;
  WLb[0] -= s * L.fr;
  WLb[4] -= s * L.fp;
  WRb[0] -= s * R.fr;
  WRb[4] -= s * R.fp;
}

// Cotangent of a cell's reconstructed variables -> cotangent of its conservative
// variables.  Gas: W = (u, v, w, P, rho) of E = (rho u, rho v, rho w, E, rho) at the full
// state (the stationary flow b plus the cell's W'), u = m / rho,
// P = (g - 1)(E - |m|^2 / (2 rho)).
__device__ __forceinline__ void gas_cot_to_cons(const double* w, const double* b, double gm1,
                                                const double* wb, double* eb) {
  const double rho = b[WB_RHO] + w[4];
  const double ir = 1.0 / rho;
  const double u[3] = {b[WB_U] + w[0], b[WB_V] + w[1], b[WB_W] + w[2]};
  const double pb = gm1 * wb[3];
  double dot = 0.0, u2 = 0.0;
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    eb[m] = wb[m] * ir - pb * u[m];
    dot += wb[m] * u[m];
    u2 += u[m] * u[m];
  }
  eb[3] = pb;
  eb[4] = wb[4] - dot * ir + 0.5 * pb * u2;
}
// Dust: W = (u, v, w, rho_d) of (rho_d u, rho_d v, rho_d w, rho_d); the velocity of an
// empty cell is held at zero.
__device__ __forceinline__ void dust_cot_to_cons(const double* w, const double* wb, double* eb) {
  const double rd = w[3];
  if (rd > 0.0) {
    const double ir = 1.0 / rd;
    eb[0] = wb[0] * ir;
    eb[1] = wb[1] * ir;
    eb[2] = wb[2] * ir;
    eb[3] = wb[3] - (wb[0] * w[0] + wb[1] * w[1] + wb[2] * w[2]) * ir;
  } else {
    eb[0] = 0.0; eb[1] = 0.0; eb[2] = 0.0;
    eb[3] = wb[3];
  }
}

// limited face states of the gas (stationary flow at the face + W' + increment), rebuilt
// for the reverse sweep rather than kept across the solve (registers)
template <int DIR>
__device__ __forceinline__ void gas_face_states(const double* wA, const double* wB,
                                                const double* wC, const double* wD,
                                                const double* coB, const double* coC,
                                                const double* bf, double qL[5], double qR[5]) {
#pragma unroll
  for (int f = 0; f < 5; ++f) {
    double iB, iC;
    if (DIR == 0) {
      iB = inc_up_c<double, true>(wA[f], wB[f], wC[f], coB);
      iC = inc_lo_c<double, true>(wB[f], wC[f], wD[f], coC);
    } else {
      iB = inc_up_u<double, true>(wA[f], wB[f], wC[f]);
      iC = inc_lo_u<double, true>(wB[f], wC[f], wD[f]);
    }
    qL[f] = bf[f] + (wB[f] + iB);
    qR[f] = bf[f] + (wC[f] + iC);
  }
}

// Reverse of one gas face: Fb (field order) is the cotangent of the face flux; the
// contributions to the reconstructed variables W' of the stencil cells A, B | C, D are
// added to cA..cD.
template <int DIR, bool G75>
__device__ void gas_face_vjp(const GasC& c, const double* wA, const double* wB, const double* wC,
                             const double* wD, const double* coB, const double* coC,
                             const double* bf, const double* bB, const double* bC,
                             const double* Fb, double* cA, double* cB, double* cC, double* cD) {
  constexpr int N = Dirs<DIR>::n, T1 = Dirs<DIR>::t1, T2 = Dirs<DIR>::t2;
  double qL[5], qR[5];
  gas_face_states<DIR>(wA, wB, wC, wD, coB, coC, bf, qL, qR);
  const bool fbL = !(qL[4] > 0.0 && qL[3] > 0.0);
  const bool fbR = !(qR[4] > 0.0 && qR[3] > 0.0);
  if (fbL) {
#pragma unroll
    for (int f = 0; f < 5; ++f) qL[f] = bB[f] + wB[f];
  }
  if (fbR) {
#pragma unroll
    for (int f = 0; f < 5; ++f) qR[f] = bC[f] + wC[f];
  }
  double WLb[5], WRb[5];
  {
    double fl[5];
    TStat st = {0, 0, 0, 0, 0, 0, 0};
    GasRec rec;
    gas_riemann<G75, true>(c, qL[4], frcp(qL[4]), qL[N], qL[T1], qL[T2], qL[3], qR[4], frcp(qR[4]),
                           qR[N], qR[T1], qR[T2], qR[3], fl, st, &rec);
    const double flb[5] = {Fb[4], Fb[N], Fb[T1], Fb[T2], Fb[3]};
    double Wb[5];
    flux_rev(c, rec, flb, Wb);
    const double WL[5] = {qL[4], qL[N], qL[T1], qL[T2], qL[3]};
    const double WR[5] = {qR[4], qR[N], qR[T1], qR[T2], qR[3]};
    riemann_rev<G75>(c, WL, WR, rec, Wb, WLb, WRb);
  }
  // face-frame cotangents (rho, un, t1, t2, p) -> field slots (u, v, w, P, rho)
  double qLb[5], qRb[5];
  qLb[4] = WLb[0]; qLb[N] = WLb[1]; qLb[T1] = WLb[2]; qLb[T2] = WLb[3]; qLb[3] = WLb[4];
  qRb[4] = WRb[0]; qRb[N] = WRb[1]; qRb[T1] = WRb[2]; qRb[T2] = WRb[3]; qRb[3] = WRb[4];
  // left face state -> cells A, B, C (or B alone after a fallback); right -> B, C, D
#pragma unroll
  for (int f = 0; f < 5; ++f) {
    if (fbL) {
      cB[f] += qLb[f];
    } else {
      double cm, cp;
      if (DIR == 0) dinc_up_c(wA[f], wB[f], wC[f], coB, cm, cp);
      else dinc_up_u(wA[f], wB[f], wC[f], cm, cp);
      cA[f] -= cm * qLb[f];
      cB[f] += (1.0 + cm - cp) * qLb[f];
      cC[f] += cp * qLb[f];
    }
    if (fbR) {
      cC[f] += qRb[f];
    } else {
      double cm, cp;
      if (DIR == 0) dinc_lo_c(wB[f], wC[f], wD[f], coC, cm, cp);
      else dinc_lo_u(wB[f], wC[f], wD[f], cm, cp);
      cB[f] -= cm * qRb[f];
      cC[f] += (1.0 + cm - cp) * qRb[f];
      cD[f] += cp * qRb[f];
    }
  }
}

// Reverse of one dust face (velocity and density reconstructed whole; a negative face
// density falls back to the cell value).  Contributions to the cells' reconstructed
// variables.
template <int DIR>
__device__ void dust_face_vjp(const double* wA, const double* wB, const double* wC,
                              const double* wD, const double* coB, const double* coC,
                              const double* Fb, double* cA, double* cB, double* cC, double* cD) {
  constexpr int N = Dirs<DIR>::n, T1 = Dirs<DIR>::t1, T2 = Dirs<DIR>::t2;
  double qL[4], qR[4], cmB[4], cpB[4], cmC[4], cpC[4];
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    double iB, iC;
    if (DIR == 0) {
      iB = inc_up_c<double, true>(wA[f], wB[f], wC[f], coB);
      iC = inc_lo_c<double, true>(wB[f], wC[f], wD[f], coC);
      dinc_up_c(wA[f], wB[f], wC[f], coB, cmB[f], cpB[f]);
      dinc_lo_c(wB[f], wC[f], wD[f], coC, cmC[f], cpC[f]);
    } else {
      iB = inc_up_u<double, true>(wA[f], wB[f], wC[f]);
      iC = inc_lo_u<double, true>(wB[f], wC[f], wD[f]);
      dinc_up_u(wA[f], wB[f], wC[f], cmB[f], cpB[f]);
      dinc_lo_u(wB[f], wC[f], wD[f], cmC[f], cpC[f]);
    }
    qL[f] = wB[f] + iB;
    qR[f] = wC[f] + iC;
  }
  const bool fbL = qL[3] < 0.0, fbR = qR[3] < 0.0;
  if (fbL) {
#pragma unroll
    for (int f = 0; f < 4; ++f) qL[f] = wB[f];
  }
  if (fbR) {
#pragma unroll
    for (int f = 0; f < 4; ++f) qR[f] = wC[f];
  }
  double fl[4];
  int side;
  dust_riemann<true>(qL[3], qL[N], qL[T1], qL[T2], qR[3], qR[N], qR[T1], qR[T2], fl, &side);
  const double flb[4] = {Fb[3], Fb[N], Fb[T1], Fb[T2]};
  double qLb[4] = {0.0, 0.0, 0.0, 0.0}, qRb[4] = {0.0, 0.0, 0.0, 0.0};
  // one side's flux (r u, r u^2, r u a, r u b) in its face state (r, u, a, b); zero for an
  // empty side (its velocity is held at zero)
  auto side_rev = [&](const double* q, double wgt, double* qb) {
    const double r = q[3];
    if (!(r > 0.0)) return;
    const double u = q[N], ta = q[T1], tb = q[T2];
    qb[3] += wgt * (flb[0] * u + flb[1] * u * u + flb[2] * u * ta + flb[3] * u * tb);
    qb[N] += wgt * (flb[0] * r + 2.0 * flb[1] * r * u + flb[2] * r * ta + flb[3] * r * tb);
    qb[T1] += wgt * flb[2] * r * u;
    qb[T2] += wgt * flb[3] * r * u;
  };
  if (side == -1) side_rev(qL, 1.0, qLb);
  else if (side == 1) side_rev(qR, 1.0, qRb);
  else if (side == 0) {
    side_rev(qL, 0.5, qLb);
    side_rev(qR, 0.5, qRb);
  }
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    if (fbL) {
      cB[f] += qLb[f];
    } else {
      cA[f] -= cmB[f] * qLb[f];
      cB[f] += (1.0 + cmB[f] - cpB[f]) * qLb[f];
      cC[f] += cpB[f] * qLb[f];
    }
    if (fbR) {
      cC[f] += qRb[f];
    } else {
      cB[f] -= cmC[f] * qRb[f];
      cC[f] += (1.0 + cmC[f] - cpC[f]) * qRb[f];
      cD[f] += cpC[f] * qRb[f];
    }
  }
}

// ------------------------------------------------------------------------------------
// the adjoint stage kernels: the theta and r faces and the cell-local sources of a tile
// of planes (k_adj_plane, LDS-staged), then the z faces of every column (k_adj_z,
// registers only, adding into the output of the first).  Two kernels keep each one's
// register footprint within the file (one kernel holding both spilled to scratch).

// group-independent set-up shared by both kernels
template <bool GAS>
struct AdjCtx {
  static constexpr int NG = GAS ? 5 : 4;
  const AdjArgs& A;
  const StageArgs& a;
  const Geo& g;
  GasC gc;
  int F0;
  __device__ AdjCtx(const AdjArgs& A_, int species)
      : A(A_), a(A_.s), g(A_.s.g), gc(gas_consts(A_.s.g.gamma, A_.s.g.newton_max)), F0(GAS ? 0 : 5 + 4 * species) {}
  __device__ int jwrap(int j) const {
    j %= g.nth;
    return j < 0 ? j + g.nth : j;
  }
  // w = cw V^-1 lambda of an interior cell (zero outside the grid)
  __device__ double wc(int f, int k, int i, int j) const {
    if (k < 0 || k >= g.nz || i < 0 || i >= g.nr) return 0.0;
    return A.cw * a.t.rt[(size_t)i * RT_N + RT_INVV] *
           A.cot[(size_t)(F0 + f) * g.N + ((size_t)k * g.nr + i) * g.nth + j];
  }
  // w of every field of a cell (zero outside the grid), all loads requested together
  __device__ void wc_all(int k, int i, int j, double* out) const {
    const bool in = !(k < 0 || k >= g.nz || i < 0 || i >= g.nr);
    const size_t c = in ? ((size_t)k * g.nr + i) * g.nth + j : 0;
    const double v = in ? a.t.rt[(size_t)i * RT_N + RT_INVV] : 0.0;
    double x[NG];
#pragma unroll
    for (int f = 0; f < NG; ++f) x[f] = A.cot[(size_t)(F0 + f) * g.N + c];
#pragma unroll
    for (int f = 0; f < NG; ++f) out[f] = in ? A.cw * v * x[f] : 0.0;
  }
  // the difference w(k1, i1, j1) - w(k0, i0, j0) of every field, times s, with all loads
  // requested before any arithmetic (loads under per-field conditions each waited)
  __device__ void wc_diff(int k1, int i1, int j1, int k0, int i0, int j0, double s,
                          double* out) const {
    const bool in1 = !(k1 < 0 || k1 >= g.nz || i1 < 0 || i1 >= g.nr);
    const bool in0 = !(k0 < 0 || k0 >= g.nz || i0 < 0 || i0 >= g.nr);
    const size_t c1 = in1 ? ((size_t)k1 * g.nr + i1) * g.nth + j1 : 0;
    const size_t c0 = in0 ? ((size_t)k0 * g.nr + i0) * g.nth + j0 : 0;
    const double v1 = in1 ? a.t.rt[(size_t)i1 * RT_N + RT_INVV] : 0.0;
    const double v0 = in0 ? a.t.rt[(size_t)i0 * RT_N + RT_INVV] : 0.0;
    double x1[NG], x0[NG];
#pragma unroll
    for (int f = 0; f < NG; ++f) {
      x1[f] = A.cot[(size_t)(F0 + f) * g.N + c1];
      x0[f] = A.cot[(size_t)(F0 + f) * g.N + c0];
    }
#pragma unroll
    for (int f = 0; f < NG; ++f)
      out[f] = s * ((in1 ? A.cw * v1 * x1[f] : 0.0) - (in0 ? A.cw * v0 * x0[f] : 0.0));
  }
};

template <int D, bool GAS, bool G75>
__device__ __forceinline__ void face_vjp(const GasC& gc, const double* wA, const double* wB,
                                         const double* wC, const double* wD, const double* coB,
                                         const double* coC, const double* bf, const double* bB,
                                         const double* bC, const double* Fb, double* oA,
                                         double* oB, double* oC, double* oD) {
  if constexpr (GAS)
    gas_face_vjp<D, G75>(gc, wA, wB, wC, wD, coB, coC, bf, bB, bC, Fb, oA, oB, oC, oD);
  else
    dust_face_vjp<D>(wA, wB, wC, wD, coB, coC, Fb, oA, oB, oC, oD);
}

// cotangent of a cell's reconstructed variables w (stationary flow b) -> conservative
template <bool GAS>
__device__ __forceinline__ void cot_to_cons(const double* w, const double* b, double gm1,
                                            const double* wb, double* eb) {
  if constexpr (GAS) gas_cot_to_cons(w, b, gm1, wb, eb);
  else dust_cot_to_cons(w, wb, eb);
}

template <bool GAS, int ND, bool G75>
__global__ void __launch_bounds__(NT) k_adj_plane(AdjArgs A, int species) {
  using C = AdjCtx<GAS>;
  constexpr int NG = C::NG;
  constexpr int H = 3;
  __shared__ double s_e[NG][TI + 2 * H][TJ + 2 * H];
  // w = cw V^-1 lambda of the staged cells (zero outside the grid), staged with the plane
  // so that the faces read no global memory
  __shared__ double s_w[NG][TI + 2 * H][TJ + 2 * H];
  __shared__ double s_at[NG][TI][TJ];
  __shared__ double s_ar[NG][TI][TJ];
  __shared__ double s_red[NT / 64];

  const C X(A, species);
  const StageArgs& a = X.a;
  const Geo& g = X.g;
  const int F0 = X.F0;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int tjb = tile % a.ntj;
  const int tib = (tile / a.ntj) % a.nti;
  const int kcb = tile / (a.ntj * a.nti);
  // the row index is wavefront-uniform (one 64-lane wavefront per row of a 1D workgroup):
  // per-row tables go to scalar registers
  const int tid = threadIdx.x, tj = tid & (TJ - 1);
  const int ti = __builtin_amdgcn_readfirstlane(tid / TJ);
  const int j0 = tjb * TJ, i0 = tib * TI;
  const int k0 = kcb * A.tk, k1 = min(g.nz, k0 + A.tk);
  const int jg = j0 + tj;
  const int ig = i0 + ti;
  const bool act = jg < g.nth && ig < g.nr;
  const bool colok = jg < g.nth;
  const int igc = min(ig, g.nr - 1);
  const double* E = (const double*)a.in;
  const double* cot = A.cot;
  const size_t N = g.N;
  const double cw = A.cw;
  const double* rt = a.t.rt + (size_t)igc * RT_N;
  const double invrc = rt[RT_INVRC], omk = rt[RT_OMK];
  using DR = std::integral_constant<int, 0>;
  using DT = std::integral_constant<int, 1>;

  // theta face between tile columns cb and cb + 1 (s_e column cb + H) of tile row r:
  // contributions to columns cb - 1 .. cb + 2
  auto theta_face = [&](int k, int r, int cb, double* oA, double* oB, double* oC, double* oD) {
    double eA[NG], eB[NG], eC[NG], eD[NG], Fb[NG];
    const int i = i0 + r;
    const double ath = a.t.rt[(size_t)i * RT_N + RT_ATH];
#pragma unroll
    for (int f = 0; f < NG; ++f) Fb[f] = ath * (s_w[f][r + H][cb + 1 + H] - s_w[f][r + H][cb + H]);
#pragma unroll
    for (int f = 0; f < NG; ++f) {
      eA[f] = s_e[f][r + H][cb + H - 1]; eB[f] = s_e[f][r + H][cb + H];
      eC[f] = s_e[f][r + H][cb + H + 1]; eD[f] = s_e[f][r + H][cb + H + 2];
      oA[f] = 0.0; oB[f] = 0.0; oC[f] = 0.0; oD[f] = 0.0;
    }
    const double* bf = a.t.wc + ((size_t)k * g.nr + i) * WB_N;
    face_vjp<DT::value, GAS, G75>(X.gc, eA, eB, eC, eD, nullptr, nullptr, bf, bf, bf, Fb, oA, oB,
                                  oC, oD);
  };
  // r face between tile rows rb and rb + 1 (s_e row rb + H) of tile column cl
  auto r_face = [&](int k, int rb, int cl, double* oA, double* oB, double* oC, double* oD) {
    double eA[NG], eB[NG], eC[NG], eD[NG], Fb[NG];
    const int ib = i0 + rb;
    const double ar = a.t.ar[ib + 1];
#pragma unroll
    for (int f = 0; f < NG; ++f) Fb[f] = ar * (s_w[f][rb + 1 + H][cl + H] - s_w[f][rb + H][cl + H]);
#pragma unroll
    for (int f = 0; f < NG; ++f) {
      eA[f] = s_e[f][rb + H - 1][cl + H]; eB[f] = s_e[f][rb + H][cl + H];
      eC[f] = s_e[f][rb + H + 1][cl + H]; eD[f] = s_e[f][rb + H + 2][cl + H];
      oA[f] = 0.0; oB[f] = 0.0; oC[f] = 0.0; oD[f] = 0.0;
    }
    const double* bf = a.t.wr + ((size_t)k * (g.nr + 1) + (ib + 1)) * WB_N;
    face_vjp<DR::value, GAS, G75>(X.gc, eA, eB, eC, eD, rco_ptr(a, ib), rco_ptr(a, ib + 1), bf,
                                  bg_ptr(a, k, ib), bg_ptr(a, k, ib + 1), Fb, oA, oB, oC, oD);
  };

  double stb = 0.0;  // Stokes-number partial (dust)
  for (int k = k0; k < k1; ++k) {
    // ---- stage the plane with a three-cell halo; clear the tile accumulators
    {
      // at most two cells per thread; both cells' loads issued before the stores
      constexpr int W = TJ + 2 * H, NC = (TI + 2 * H) * W;
      static_assert(NC <= 2 * NT, "two staged cells per thread");
      const int h0 = tid, h1 = tid + NT;
      const int ia = i0 + h0 / W - H, ja = X.jwrap(j0 + h0 % W - H);
      const int ib = i0 + h1 / W - H, jb = X.jwrap(j0 + h1 % W - H);
      double v0[NG], v1[NG], c0[NG], c1[NG];
      X.wc_all(k, ia, ja, c0);
      if (h1 < NC) X.wc_all(k, ib, jb, c1);
      load_recon<false, false, NG>(a, E, F0, k, ia, ja, v0);
      if (h1 < NC) load_recon<false, false, NG>(a, E, F0, k, ib, jb, v1);
#pragma unroll
      for (int f = 0; f < NG; ++f) {
        s_e[f][h0 / W][h0 % W] = v0[f];
        s_w[f][h0 / W][h0 % W] = c0[f];
      }
      if (h1 < NC) {
#pragma unroll
        for (int f = 0; f < NG; ++f) {
          s_e[f][h1 / W][h1 % W] = v1[f];
          s_w[f][h1 / W][h1 % W] = c1[f];
        }
      }
    }
#pragma unroll
    for (int f = 0; f < NG; ++f) { s_at[f][ti][tj] = 0.0; s_ar[f][ti][tj] = 0.0; }
    __syncthreads();

    double oA[NG], oB[NG], oC[NG], oD[NG];
    // ---- theta faces j+1/2 of the thread's own cell; four ordered scatter phases
    const bool tok = ig < g.nr;
    if (tok) theta_face(k, ti, tj, oA, oB, oC, oD);
#pragma unroll
    for (int ph = 0; ph < 4; ++ph) {
      const int col = tj - 1 + ph;
      if (tok && col >= 0 && col < TJ) {
        const double* o = ph == 0 ? oA : ph == 1 ? oB : ph == 2 ? oC : oD;
#pragma unroll
        for (int f = 0; f < NG; ++f) s_at[f][ti][col] += o[f];
      }
      __syncthreads();
    }
    // ---- r faces i+1/2 of the thread's own cell
    const bool rok = ig < g.nr && colok;
    if (rok) r_face(k, ti, tj, oA, oB, oC, oD);
#pragma unroll
    for (int ph = 0; ph < 4; ++ph) {
      const int row = ti - 1 + ph;
      if (rok && row >= 0 && row < TI) {
        const double* o = ph == 0 ? oA : ph == 1 ? oB : ph == 2 ? oC : oD;
#pragma unroll
        for (int f = 0; f < NG; ++f) s_ar[f][row][tj] += o[f];
      }
      __syncthreads();
    }
    // ---- the remaining faces within 3/2 cells of the tile: theta faces at tile columns
    //      -3/2, -1/2, 64+1/2 of each row (threads 0..23), r faces at tile rows -3/2,
    //      -1/2, 8+1/2 of each column (threads 24..215)
    int ekind = 0, eline = 0, epos = 0;  // 1 theta, 2 r; tile row/column; face lower cell
    if (tid < 3 * TI) {
      const int q = tid % 3;
      ekind = 1; eline = tid / 3; epos = q == 0 ? -2 : (q == 1 ? -1 : TJ);
      if (i0 + eline >= g.nr) ekind = 0;
    } else if (tid < 3 * TI + 3 * TJ) {
      const int e = tid - 3 * TI;
      const int q = e / TJ;
      ekind = 2; eline = e % TJ; epos = q == 0 ? -2 : (q == 1 ? -1 : TI);
      const int ib = i0 + epos;
      if (ib + 1 < 0 || ib >= g.nr || j0 + eline >= g.nth) ekind = 0;
    }
    if (ekind == 1) theta_face(k, eline, epos, oA, oB, oC, oD);
    else if (ekind == 2) r_face(k, epos, eline, oA, oB, oC, oD);
#pragma unroll
    for (int ph = 0; ph < 4; ++ph) {
      const int t = epos - 1 + ph;  // target cell along the face normal
      if (ekind == 1 && t >= 0 && t < TJ) {
        const double* o = ph == 0 ? oA : ph == 1 ? oB : ph == 2 ? oC : oD;
#pragma unroll
        for (int f = 0; f < NG; ++f) s_at[f][eline][t] += o[f];
      } else if (ekind == 2 && t >= 0 && t < TI) {
        const double* o = ph == 0 ? oA : ph == 1 ? oB : ph == 2 ? oC : oD;
#pragma unroll
        for (int f = 0; f < NG; ++f) s_ar[f][t][eline] += o[f];
      }
      __syncthreads();
    }
    // ---- in-plane total of the thread's cell, the reverse of its sources, the bases
    if (!act) continue;
    double cur[NG];
    {
      // in-plane faces' cotangent of the cell's reconstructed variables -> conservative
      double wb[NG], w[NG];
#pragma unroll
      for (int f = 0; f < NG; ++f) {
        wb[f] = s_at[f][ti][tj] + s_ar[f][ti][tj];
        w[f] = s_e[f][ti + H][tj + H];
      }
      cot_to_cons<GAS>(w, a.t.wc + ((size_t)k * g.nr + ig) * WB_N, X.gc.gm1, wb, cur);
    }
    const size_t cell = ((size_t)k * g.nr + ig) * g.nth + jg;
    const double gr = a.t.grav[((size_t)k * g.nr + ig) * 2 + 0];
    const double gz = a.t.grav[((size_t)k * g.nr + ig) * 2 + 1];
    const double* bgc = a.t.bgc + ((size_t)k * g.nr + ig) * 5;
    double q[5], sg[5];
#pragma unroll
    for (int f = 0; f < 5; ++f) {
      q[f] = bgc[f] + E[(size_t)f * N + cell];
      sg[f] = cw * cot[(size_t)f * N + cell];
    }
    const double ir = 1.0 / q[4];
    const double U[3] = {q[0] * ir, q[1] * ir, q[2] * ir};
    if constexpr (GAS) {
      const double gm1 = X.gc.gm1;
      const double u = U[0], v = U[1], w = U[2];
      // S_r = (m_th v + p)/r + rho g_r, S_th = -m_r v / r, S_z = rho g_z,
      // S_E = m_r g_r + m_z g_z
      cur[0] += sg[0] * (-gm1 * u * invrc) + sg[1] * (-v * invrc) + sg[3] * gr;
      cur[1] += sg[0] * ((2.0 - gm1) * v * invrc) + sg[1] * (-u * invrc);
      cur[2] += sg[0] * (-gm1 * w * invrc) + sg[3] * gz;
      cur[3] += sg[0] * gm1 * invrc;
      cur[4] += sg[0] * ((-v * v + 0.5 * gm1 * (u * u + v * v + w * w)) * invrc + gr) +
                sg[1] * (u * v * invrc) + sg[2] * gz;
      // drag D_s = rho_d (v_d - v) Omega_K / St on the gas (+) and the dust (-), and
      // v . D in the gas energy
      double Ub[3] = {0.0, 0.0, 0.0}, Dt[3] = {0.0, 0.0, 0.0};
      // every species' variables and cotangents requested together (loads made
      // conditional on the density would each wait for it)
      double ev[ND > 0 ? ND : 1][4], cv[ND > 0 ? ND : 1][3];
#pragma unroll
      for (int s = 0; s < ND; ++s)
#pragma unroll
        for (int c2 = 0; c2 < 4; ++c2) {
          ev[s][c2] = E[(size_t)(5 + 4 * s + c2) * N + cell];
          if (c2 < 3) cv[s][c2] = cot[(size_t)(5 + 4 * s + c2) * N + cell];
        }
#pragma unroll
      for (int s = 0; s < ND; ++s) {
        const double rdn = ev[s][3];
        double vd[3] = {0.0, 0.0, 0.0};
        if (rdn > 0.0) {
          const double id = 1.0 / rdn;
#pragma unroll
          for (int c2 = 0; c2 < 3; ++c2) vd[c2] = ev[s][c2] * id;
        }
        const double its = omk * g.inv_st[s];
#pragma unroll
        for (int c2 = 0; c2 < 3; ++c2) {
          Dt[c2] += rdn * (vd[c2] - U[c2]) * its;
          const double Db = sg[c2] + sg[3] * U[c2] - cw * cv[s][c2];
          Ub[c2] -= its * rdn * Db;
        }
      }
      double dot = 0.0;
#pragma unroll
      for (int c2 = 0; c2 < 3; ++c2) {
        Ub[c2] += sg[3] * Dt[c2];
        cur[c2] += Ub[c2] * ir;
        dot += Ub[c2] * U[c2];
      }
      cur[4] -= dot * ir;
    } else {
      const double m[3] = {E[(size_t)F0 * N + cell], E[(size_t)(F0 + 1) * N + cell],
                           E[(size_t)(F0 + 2) * N + cell]};
      const double rdn = E[(size_t)(F0 + 3) * N + cell];
      double sd[4];
#pragma unroll
      for (int f = 0; f < 4; ++f) sd[f] = cw * cot[(size_t)(F0 + f) * N + cell];
      double vd[3] = {0.0, 0.0, 0.0};
      if (rdn > 0.0) {
        const double id = 1.0 / rdn;
        vd[0] = m[0] * id; vd[1] = m[1] * id; vd[2] = m[2] * id;
        // S_r = m_th v_d / r + rho_d g_r, S_th = -m_r v_d / r
        cur[1] += sd[0] * 2.0 * vd[1] * invrc - sd[1] * vd[0] * invrc;
        cur[0] += -sd[1] * vd[1] * invrc;
        cur[3] += sd[0] * (-vd[1] * vd[1] * invrc) + sd[1] * (vd[0] * vd[1] * invrc);
      }
      cur[3] += sd[0] * gr + sd[2] * gz;
      const double its = omk * g.inv_st[species];
      const double st = 1.0 / g.inv_st[species];
      double dotU = 0.0, dotD = 0.0;
#pragma unroll
      for (int c2 = 0; c2 < 3; ++c2) {
        const double Ds = rdn * (vd[c2] - U[c2]) * its;
        const double Db = sg[c2] + sg[3] * U[c2] - sd[c2];
        if (rdn > 0.0) cur[c2] += its * Db;
        dotU += Db * U[c2];
        dotD += Db * Ds;
      }
      cur[3] -= its * dotU;
      stb -= dotD / st;
    }
    // all loads before any store (out may be one of the bases), each base's fields
    // requested together
    double v[NG], b1[NG], b2[NG];
    if (A.base1) {
#pragma unroll
      for (int f = 0; f < NG; ++f) b1[f] = A.base1[(size_t)(F0 + f) * N + cell];
    }
    if (A.base2) {
#pragma unroll
      for (int f = 0; f < NG; ++f) b2[f] = A.base2[(size_t)(F0 + f) * N + cell];
    }
#pragma unroll
    for (int f = 0; f < NG; ++f) {
      v[f] = cur[f];
      if (A.base1) v[f] += b1[f];
      if (A.base2) v[f] += b2[f];
    }
#pragma unroll
    for (int f = 0; f < NG; ++f) A.out[(size_t)(F0 + f) * N + cell] = v[f];
  }
  // ---- Stokes-number partial of the block (dust)
  if constexpr (!GAS) {
    const double ws = wave_sum(stb);
    if ((tid & 63) == 0) s_red[tid / 64] = ws;
    __syncthreads();
    if (tid == 0) {
      double acc = 0.0;
      for (int w = 0; w < NT / 64; ++w) acc += s_red[w];
      A.stpart[blockIdx.x] = acc;
    }
  }
}

// z faces: one thread per column and chunk of planes, marching up; adds the four stencil
// contributions of every z face to the output written by k_adj_plane (each cell
// completed in order: its faces k-3/2 .. k+3/2, lower first).
template <bool GAS, int ND, bool G75>
__global__ void __launch_bounds__(256, 2) k_adj_z(AdjArgs A, int species, int tkz) {
  using C = AdjCtx<GAS>;
  constexpr int NG = C::NG;
  const C X(A, species);
  const StageArgs& a = X.a;
  const Geo& g = X.g;
  const int F0 = X.F0;
  const size_t ncol = (size_t)g.nr * g.nth;
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t col = t % ncol;
  const int kc = (int)(t / ncol);
  const int k0 = kc * tkz;
  if (k0 >= g.nz) return;
  const int k1 = min(g.nz, k0 + tkz);
  const int ig = (int)(col / g.nth), jg = (int)(col % g.nth);
  const double* E = (const double*)a.in;
  const double Az = a.t.rt[(size_t)ig * RT_N + RT_AZ];

  double ra[NG], rb[NG], rc[NG], rd[NG];  // cells kf-1 .. kf+2 of the face kf+1/2
  auto load = [&](double* dst, int k) { load_recon<false, false, NG>(a, E, F0, k, ig, jg, dst); };
  // adds the face's contributions into oA..oD
  auto zface = [&](int kf, double* oA, double* oB, double* oC, double* oD) {
    double Fb[NG];
    X.wc_diff(kf + 1, ig, jg, kf, ig, jg, Az, Fb);
    const double* bf = a.t.wz + ((size_t)(kf + 1) * g.nr + ig) * WB_N;
    face_vjp<2, GAS, G75>(X.gc, ra, rb, rc, rd, nullptr, nullptr, bf, bg_ptr(a, kf, ig),
                          bg_ptr(a, kf + 1, ig), Fb, oA, oB, oC, oD);
  };
  auto real = [&](int kf) { return kf >= -1 && kf <= g.nz - 1; };
  // adds the z faces' cotangent v of cell k's reconstructed variables (w: the cell's W')
  // to the cell's conservative cotangent
  auto add_out = [&](int k, const double* w, const double* v) {
    const size_t cell = ((size_t)k * g.nr + ig) * g.nth + jg;
    double ec[NG];
    cot_to_cons<GAS>(w, a.t.wc + ((size_t)k * g.nr + ig) * WB_N, X.gc.gm1, v, ec);
    double o[NG];
#pragma unroll
    for (int f = 0; f < NG; ++f) o[f] = A.out[(size_t)(F0 + f) * g.N + cell] + ec[f];
#pragma unroll
    for (int f = 0; f < NG; ++f) A.out[(size_t)(F0 + f) * g.N + cell] = o[f];
  };

  // contributions of the faces below cell k to cells k (zb) and k+1 (zc); za = cell k-1
  // za, zb, zc, zd: cells k-1, k, k+1, k+2 of the face k+1/2 being processed; the
  // contributions to cells below k0 (faces k0-3/2, k0-1/2) land in scratch accumulators
  double za[NG], zb[NG], zc[NG], zd[NG];
#pragma unroll
  for (int f = 0; f < NG; ++f) { za[f] = 0.0; zb[f] = 0.0; zc[f] = 0.0; zd[f] = 0.0; }
  load(ra, k0 - 3); load(rb, k0 - 2); load(rc, k0 - 1); load(rd, k0);
  // face k0-3/2: cells k0-3 .. k0 -> (za, za, za, zb); only its last one is kept
  if (real(k0 - 2)) {
    zface(k0 - 2, zd, zd, zc, zb);
#pragma unroll
    for (int f = 0; f < NG; ++f) { zc[f] = 0.0; zd[f] = 0.0; }
  }
#pragma unroll
  for (int f = 0; f < NG; ++f) { ra[f] = rb[f]; rb[f] = rc[f]; rc[f] = rd[f]; }
  load(rd, k0 + 1);
  // face k0-1/2: cells k0-2 .. k0+1 -> (-, -, zb, zc)
  if (real(k0 - 1)) {
    zface(k0 - 1, zd, za, zb, zc);
#pragma unroll
    for (int f = 0; f < NG; ++f) { za[f] = 0.0; zd[f] = 0.0; }
  }
  if constexpr (GAS) {
    for (int k = k0; k <= k1; ++k) {
#pragma unroll
      for (int f = 0; f < NG; ++f) { ra[f] = rb[f]; rb[f] = rc[f]; rc[f] = rd[f]; }
      load(rd, k + 2);
      // face k+1/2 (cells k-1, k, k+1, k+2)
      if (real(k)) zface(k, za, zb, zc, zd);
      if (k - 1 >= k0) add_out(k - 1, ra, za);
#pragma unroll
      for (int f = 0; f < NG; ++f) { za[f] = zb[f]; zb[f] = zc[f]; zc[f] = zd[f]; zd[f] = 0.0; }
    }
  } else {
    // dust (registers to spare): the next plane's loads are requested one plane ahead and
    // used raw a plane later — the column's next cell, the cotangent of the next face's
    // upper cell and the output cell of the next step — so that no plane waits for memory
    const double vinv = a.t.rt[(size_t)ig * RT_N + RT_INVV];
    // w of a cell of the column from its cotangent (zero outside the grid)
    auto wcell = [&](int k, const double* x, double* w) {
      const bool in = k >= 0 && k < g.nz;
#pragma unroll
      for (int f = 0; f < NG; ++f) w[f] = in ? A.cw * vinv * x[f] : 0.0;
    };
    // a field group of cell k of the column (k clamped into the grid: a cell outside it is
    // never used)
    auto col_fetch = [&](const double* src, int k, double* x) {
      const size_t c = ((size_t)min(max(k, 0), g.nz - 1) * g.nr + ig) * g.nth + jg;
#pragma unroll
      for (int f = 0; f < NG; ++f) x[f] = src[(size_t)(F0 + f) * g.N + c];
    };
    double wlo[NG], xr[NG], orw[NG];
    {
      double x[NG];
      col_fetch(A.cot, k0, x);
      wcell(k0, x, wlo);
    }
    col_fetch(A.cot, k0 + 1, xr);
    DustRaw<false> nraw;
    dust_fetch<false, false>(a, E, F0, k0 + 2, ig, jg, nraw);
#pragma unroll
    for (int f = 0; f < NG; ++f) orw[f] = 0.0;
    for (int k = k0; k <= k1; ++k) {
#pragma unroll
      for (int f = 0; f < NG; ++f) { ra[f] = rb[f]; rb[f] = rc[f]; rc[f] = rd[f]; }
      dust_finish<false>(nraw, rd);  // cell k+2
      double whi[NG], ocur[NG];
      wcell(k + 1, xr, whi);
#pragma unroll
      for (int f = 0; f < NG; ++f) ocur[f] = orw[f];  // the output of cell k-1
      if (k + 1 <= k1) {
        dust_fetch<false, false>(a, E, F0, k + 3, ig, jg, nraw);
        col_fetch(A.cot, k + 2, xr);
        col_fetch(A.out, k, orw);
      }
      // face k+1/2 (cells k-1, k, k+1, k+2)
      if (real(k)) {
        double Fb[NG];
#pragma unroll
        for (int f = 0; f < NG; ++f) Fb[f] = Az * (whi[f] - wlo[f]);
        face_vjp<2, GAS, G75>(X.gc, ra, rb, rc, rd, nullptr, nullptr, nullptr, nullptr, nullptr,
                              Fb, za, zb, zc, zd);
      }
      if (k - 1 >= k0) {
        const size_t cell = ((size_t)(k - 1) * g.nr + ig) * g.nth + jg;
        double ec[NG];
        cot_to_cons<GAS>(ra, nullptr, X.gc.gm1, za, ec);
#pragma unroll
        for (int f = 0; f < NG; ++f) A.out[(size_t)(F0 + f) * g.N + cell] = ocur[f] + ec[f];
      }
#pragma unroll
      for (int f = 0; f < NG; ++f) {
        wlo[f] = whi[f];
        za[f] = zb[f]; zb[f] = zc[f]; zc[f] = zd[f]; zd[f] = 0.0;
      }
    }
  }
}

// acc[0] += sum of parts[0 .. n) in a fixed order
__global__ void __launch_bounds__(256) k_st_accum(const double* parts, int n, double* acc) {
  __shared__ double s_s[4];
  double v = 0.0;
  for (int b = threadIdx.x; b < n; b += blockDim.x) v += parts[b];
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) s_s[threadIdx.x / 64] = v;
  __syncthreads();
  if (threadIdx.x == 0) acc[0] += (s_s[0] + s_s[1]) + (s_s[2] + s_s[3]);
}

// ------------------------------------------------------------------------------------
// launchers

template <int ND>
static void adj_nd(const AdjArgs& a, int blocks, int zblocks, int tkz, int group, hipStream_t s) {
  if (group == 0) {
    if (a.s.g.gamma == 1.4) {
      hipLaunchKernelGGL((k_adj_plane<true, ND, true>), dim3(blocks), dim3(NT), 0, s, a, 0);
      if (!a.s.g.twod)
        hipLaunchKernelGGL((k_adj_z<true, ND, true>), dim3(zblocks), dim3(256), 0, s, a, 0, tkz);
    } else {
      hipLaunchKernelGGL((k_adj_plane<true, ND, false>), dim3(blocks), dim3(NT), 0, s, a, 0);
      if (!a.s.g.twod)
        hipLaunchKernelGGL((k_adj_z<true, ND, false>), dim3(zblocks), dim3(256), 0, s, a, 0, tkz);
    }
  } else {
    if constexpr (ND > 0) {
      hipLaunchKernelGGL((k_adj_plane<false, ND, true>), dim3(blocks), dim3(NT), 0, s, a, group - 1);
      if (!a.s.g.twod)
        hipLaunchKernelGGL((k_adj_z<false, ND, true>), dim3(zblocks), dim3(256), 0, s, a, group - 1,
                           tkz);
    }
  }
}

hipError_t launch_adj_group(const AdjArgs& a, int blocks, int group, hipStream_t s) {
  // z kernel: whole columns when they alone give 2048 wavefronts (8 per SIMD), else
  // chunks of 8 planes (each chunk re-solves the 3 faces below its first plane)
  const size_t ncol = (size_t)a.s.g.nr * a.s.g.nth;
  const int tkz = ncol / 64 >= 2048 ? a.s.g.nz : std::min(8, a.s.g.nz);
  const size_t nthreads = ncol * (size_t)((a.s.g.nz + tkz - 1) / tkz);
  const int zblocks = (int)((nthreads + 255) / 256);
  switch (a.s.g.nd) {
    case 0: adj_nd<0>(a, blocks, zblocks, tkz, group, s); break;
    case 1: adj_nd<1>(a, blocks, zblocks, tkz, group, s); break;
    case 2: adj_nd<2>(a, blocks, zblocks, tkz, group, s); break;
    case 3: adj_nd<3>(a, blocks, zblocks, tkz, group, s); break;
    default: adj_nd<4>(a, blocks, zblocks, tkz, group, s); break;
  }
  return hipGetLastError();
}

hipError_t launch_st_accum(const double* parts, int nblocks, double* acc, hipStream_t s) {
  hipLaunchKernelGGL(k_st_accum, dim3(1), dim3(256), 0, s, parts, nblocks, acc);
  return hipGetLastError();
}

}  // namespace rb
