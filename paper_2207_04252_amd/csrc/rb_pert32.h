// FP32 perturbation form of the gas face flux (included by rb_kernels.hip).
//
// The face background W0 (the stationary flow at the face, FP64) is the same on both
// sides, so the Riemann problem between W0 + W'_L and W0 + W'_R (the reconstructed
// primitive deviations) is solved for the perturbations: q = p* - p0 by Newton in FP32,
// every pressure-function term written without cancellation ((1+x)^(1/7) - 1 =
// x / sum_{k<7} y^k), the sampled state as a perturbation, and the flux returned as
// dF = F(W0 + W') - F(W0).  The empty-run
// residual is then never formed: G(E) - G(E0) = S' V - sum A dF.  Strong perturbations,
// a transonic fan or a Newton failure fall back to the FP64 solver.
#pragma once

namespace rb {

// FP32 reciprocal and square root from the hardware instructions (within an ulp or two;
// the perturbation form's accuracy target is 1e-5 relative)
__device__ __forceinline__ float rcp32(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float sqrt32(float x) { return __builtin_amdgcn_sqrtf(x); }

// stationary-flow primitives at a face in the face frame (FP64), from its WB_N entry
struct BgW {
  double rho, un, t1, t2, p, c, h;  // h = E + p per volume
};

template <int DIR>
__device__ __forceinline__ BgW bg_face(const double* w) {
  BgW b;
  b.rho = w[WB_RHO];
  b.un = w[Dirs<DIR>::n];
  b.t1 = w[Dirs<DIR>::t1];
  b.t2 = w[Dirs<DIR>::t2];
  b.p = w[WB_P];
  b.c = w[WB_C];
  b.h = w[WB_H];
  return b;
}

// perturbation of a primitive face state
struct PW {
  float rho, un, t1, t2, p;
};

// flux perturbation of a primitive perturbation about the face background
__device__ __forceinline__ void flux_pert(const BgW& b, const PW& w, float inv_gm1, float out[5]) {
  const float un0 = (float)b.un, t10 = (float)b.t1, t20 = (float)b.t2;
  const float rho = (float)(b.rho + (double)w.rho);
  const float dmass = w.rho * un0 + rho * w.un;
  const float mflux = (float)(b.rho * b.un) + dmass;
  const float u0sq = (float)(b.un * b.un + b.t1 * b.t1 + b.t2 * b.t2);
  const float dot = un0 * w.un + t10 * w.t1 + t20 * w.t2;
  const float usq = w.un * w.un + w.t1 * w.t1 + w.t2 * w.t2;
  const float dke = 0.5f * w.rho * u0sq + rho * dot + 0.5f * rho * usq;
  const float dh = w.p * inv_gm1 + dke + w.p;
  const float h = (float)b.h + dh;
  out[0] = dmass;
  out[1] = dmass * un0 + mflux * w.un + w.p;
  out[2] = dmass * t10 + mflux * w.t1;
  out[3] = dmass * t20 + mflux * w.t2;
  out[4] = dh * un0 + h * w.un;
}

// one side of the perturbation Riemann problem
struct SideP {
  float pp;       // p'_K
  float p;        // p_K = p0 + p'_K
  float rho, c, A, B, irc, ip;
  float u;        // full normal velocity u0 + u'_K
  float up;       // u'_K
};

__device__ __forceinline__ SideP make_side_p(const BgW& b, const PW& w, const GasC& g) {
  SideP s;
  s.pp = w.p;
  s.p = (float)(b.p + (double)w.p);
  s.rho = (float)(b.rho + (double)w.rho);
  s.c = sqrt32((float)g.g * s.p * rcp32(s.rho));
  s.A = (float)g.a2 * rcp32(s.rho);
  s.B = (float)g.kshock * s.p;
  s.irc = rcp32(s.rho * s.c);
  s.ip = rcp32(s.p);
  s.up = w.un;
  s.u = (float)b.un + w.un;
  return s;
}

// y = (1 + x)^(1/7) (FP32 hardware log2/exp2, one Newton step) and (1 + x)^(1/7) - 1
// written as x / sum_{k<7} y^k (no cancellation for small x)
__device__ __forceinline__ void root7p(float x, float& y, float& ym1) {
  const float a = 1.0f + x;
  y = __builtin_amdgcn_exp2f(0.142857142857f * __builtin_amdgcn_logf(a));
  float y2 = y * y, y3 = y2 * y, y6 = y3 * y3;
  y = y - (y6 * y - a) * rcp32(7.0f * y6);
  y2 = y * y;
  y3 = y2 * y;
  const float s = 1.0f + y + y2 + y3 + y3 * y + y3 * y2 + y3 * y3;
  ym1 = x * rcp32(s);
}

// pressure function of one side at p* = p0 + q (gamma = 7/5): value and derivative
__device__ __forceinline__ void pfun_p(float q, const SideP& K, float& f, float& df) {
  const float d = q - K.pp;  // p* - p_K
  if (d > 0.0f) {
    const float ps = K.p + d;
    const float ipb = rcp32(ps + K.B);
    const float qs = sqrt32(K.A * ipb);
    f = d * qs;
    df = qs * (1.0f - 0.5f * d * ipb);
  } else {
    float y, ym1;
    root7p(d * K.ip, y, ym1);
    f = 5.0f * K.c * ym1;
    const float y2 = y * y, y3 = y2 * y, y6 = y3 * y3;
    df = rcp32(y6) * K.irc;
  }
}

// Perturbation exact Riemann problem (gamma = 7/5) at x/t = 0.  Returns false when the
// FP64 solver must be used instead.
__device__ __forceinline__ bool riemann_pert(const BgW& b, const PW& WL, const PW& WR, const GasC& g,
                                             PW& W, TStat& st) {
  st.last = 0;
  // strong perturbations are left to the FP64 solver
  const float p0 = (float)b.p, r0 = (float)b.rho, c0 = (float)b.c;
  if (!(fabsf(WL.p) < 0.1f * p0 && fabsf(WR.p) < 0.1f * p0 && fabsf(WL.rho) < 0.1f * r0 &&
        fabsf(WR.rho) < 0.1f * r0 && fabsf(WL.un) < 0.1f * c0 && fabsf(WR.un) < 0.1f * c0))
    return false;
  const SideP L = make_side_p(b, WL, g);
  const SideP R = make_side_p(b, WR, g);
  const float du = WR.un - WL.un;
  // supersonic faces: the left (right) state is the solution when f(p_hi) >= 0 and the
  // contact moves the same way (same argument as the FP64 solver, with margins)
  if (L.u >= L.c) {
    const float m = L.u * rcp32(L.c);
    const float phi = L.p * (m * m - (float)g.gm1_2g) * (float)g.inv_gp1_2g;
    float fL, dL, fR, dR;
    pfun_p(phi - p0, L, fL, dL);
    pfun_p(phi - p0, R, fR, dR);
    if (fL + fR + du >= 1e-3f * fL && L.u - fL >= 1e-3f * L.u) {
      W = WL;
      return true;
    }
  } else if (R.u <= -R.c) {
    const float m = -R.u * rcp32(R.c);
    const float phi = R.p * (m * m - (float)g.gm1_2g) * (float)g.inv_gp1_2g;
    float fL, dL, fR, dR;
    pfun_p(phi - p0, L, fL, dL);
    pfun_p(phi - p0, R, fR, dR);
    if (fL + fR + du >= 1e-3f * fR && R.u + fR <= 1e-3f * R.u) {
      W = WR;
      return true;
    }
  }
  // Newton on q = p* - p0 from the primitive-variable guess
  float q = 0.5f * (WL.p + WR.p) - 0.125f * du * (L.rho + R.rho) * (L.c + R.c);
  const float qfloor = 1e-8f * fminf(L.p, R.p) - p0;
  q = fmaxf(q, qfloor);
  float fL = 0.f, dL = 1.f, fR = 0.f, dR = 1.f, dq = 0.f;
  bool conv = false;
  int it = 0;
  while (it < 20) {
    ++it;
    pfun_p(q, L, fL, dL);
    pfun_p(q, R, fR, dR);
    float qn = q - (fL + fR + du) * rcp32(dL + dR);
    qn = fmaxf(qn, 1e-8f * (p0 + q) - p0);
    dq = qn - q;
    q = qn;
    if (fabsf(dq) <= 1e-6f * fabsf(q) + 1e-9f * p0) { conv = true; break; }
  }
  st.maxit = max(st.maxit, it);
  st.last = it;
  if (!conv) return false;
  const float us = 0.5f * (WL.un + WR.un) + 0.5f * ((fR + dR * dq) - (fL + dL * dq));
  const float usfull = (float)b.un + us;
  const float kk = (float)g.kshock;
  if (0.0f <= usfull) {
    if (q > WL.p) {
      const float x = (q - WL.p) * L.ip;
      const float sL = L.u - L.c * sqrt32((float)g.gp1_2g * (1.0f + x) + (float)g.gm1_2g);
      if (0.0f <= sL) { W = WL; return true; }
      const float rm1 = x * (1.0f - kk) * rcp32(kk * (1.0f + x) + 1.0f);
      W.rho = WL.rho + L.rho * rm1;
    } else {
      if (0.0f <= L.u - L.c) { W = WL; return true; }
      float y, ym1;
      root7p((q - WL.p) * L.ip, y, ym1);
      if (!(0.0f > usfull - L.c * y)) return false;  // transonic fan: FP64
      const float y5m1 = ym1 * (1.0f + y + y * y + y * y * y + y * y * y * y);
      W.rho = WL.rho + L.rho * y5m1;
    }
    W.un = us; W.p = q; W.t1 = WL.t1; W.t2 = WL.t2;
    return true;
  }
  if (q > WR.p) {
    const float x = (q - WR.p) * R.ip;
    const float sR = R.u + R.c * sqrt32((float)g.gp1_2g * (1.0f + x) + (float)g.gm1_2g);
    if (0.0f >= sR) { W = WR; return true; }
    const float rm1 = x * (1.0f - kk) * rcp32(kk * (1.0f + x) + 1.0f);
    W.rho = WR.rho + R.rho * rm1;
  } else {
    if (0.0f >= R.u + R.c) { W = WR; return true; }
    float y, ym1;
    root7p((q - WR.p) * R.ip, y, ym1);
    if (!(0.0f <= usfull + R.c * y)) return false;
    const float y5m1 = ym1 * (1.0f + y + y * y + y * y * y + y * y * y * y);
    W.rho = WR.rho + R.rho * y5m1;
  }
  W.un = us; W.p = q; W.t1 = WR.t1; W.t2 = WR.t2;
  return true;
}

}  // namespace rb
