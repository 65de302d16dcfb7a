// Device kernels of the bi-fluid finite-volume library for gfx950 (MI355X).
//
// One RK2 stage is one launch of k_stage: a workgroup owns a 64 (theta) x 8 (r) tile of
// cells and marches through a chunk of z planes.  Each z plane of the tile, with a
// two-cell halo, is staged in LDS; every thread solves the Riemann problems at the upper
// theta and r faces of its own cell (the tile's lower-edge faces are solved by the first
// 72 threads), exchanges the fluxes through LDS, and keeps the z direction in registers
// (a three-plane ring of the cell's column and the flux of the face below).  Fluxes,
// divergence, sources, drag and the update are fused: the state is read once per
// stage (plus the L2-resident halo) and written once.
#include "rb_device.h"

namespace rb {

// ------------------------------------------------------------------------------------
// the stage kernels: one launch per group of fields (the gas; each dust species).  The
// groups interact only through the cell-local drag, which each kernel evaluates from
// the other group's centre state of the same stage input.

template <bool GAS, int ND, bool G75, bool P32, bool EXT>
__global__ void __launch_bounds__(NTM, WPE) k_march(StageArgs a, int species) {
  constexpr int NG = GAS ? 5 : 4;
  constexpr bool PG = GAS && P32;  // gas in the FP32 perturbation form
  using T = typename std::conditional<PG, float, double>::type;
  // a hard error stops the evolution; the flag is read once and broadcast so that the
  // whole workgroup takes the same branch (other workgroups may set it meanwhile)
  __shared__ int s_stop;
  if (threadIdx.x == 0) s_stop = __atomic_load_n(&a.c.ctrl->status, __ATOMIC_RELAXED);
  __syncthreads();
  if (s_stop & FL_HARD) return;
  __shared__ T s_pl[NG][TM + 4][TJ + 4];
  __shared__ T s_ft[NG][TM][TJ + 1];
  __shared__ T s_fr[NG][TM + 1][TJ];
  __shared__ double s_red[NTM / 64][3];
  // FP64 gas: per-thread slots (no sharing) for the column's cell below the current plane
  // and the flux of the z face below, kept in LDS between their uses (without them the
  // face solves spill registers); the other kernels keep both in registers
  constexpr bool LR = GAS && !P32;
  __shared__ T s_rm[LR ? NG : 1][LR ? NTM : 1];
  __shared__ T s_fz[LR ? NG : 1][LR ? NTM : 1];

  const Geo& g = a.g;
  const GasC gc = gas_consts(g.gamma, g.newton_max);
  const int F0 = GAS ? 0 : 5 + 4 * species;
  const int slot = GAS ? 0 : 1 + species;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int tjb = tile % a.ntj;
  const int tib = (tile / a.ntj) % a.ntm;
  const int kcb = tile / (a.ntj * a.ntm);
  // one wavefront per radial row (TJ = 64 lanes of a 1D workgroup): the row index is
  // wavefront-uniform, and saying so puts the per-row tables in scalar registers and
  // scalar loads (without it the FP64 gas kernel spills)
  const int tid = threadIdx.x, tj = tid & (TJ - 1);
  const int ti = __builtin_amdgcn_readfirstlane(tid / TJ);
  const int j0 = tjb * TJ, i0 = tib * TM;
  const int k0 = kcb * a.tk, k1 = min(g.nz, k0 + a.tk);
  const int jg = j0 + tj;
  const int jw = jg % g.nth;
  const int ig = i0 + ti;
  const bool act = jg < g.nth && ig < g.nr;
  const int igc = min(ig, g.nr - 1);
  const bool drag = !a.gas_only && ND > 0 && !g.drag_exact;
  const void* in = a.in;
  const double dt = a.dt_idx >= 0 ? a.c.dtlog[a.dt_idx] : 0.0;

  TStat st = {0, 0, 0, 0, 0, 0, 0};
  // histogram of the Newton iteration counts (bins 0..7, 7: seven or more) over the
  // faces the thread owns (each face of the mesh is owned by one thread of the launch),
  // 16 bits a bin in LDS slots private to the thread; a thread owns at most 4 faces per
  // plane and one more
  __shared__ unsigned s_nh[GAS ? 4 : 1][GAS ? NTM : 1];
  if constexpr (GAS) {
#pragma unroll
    for (int q = 0; q < 4; ++q) s_nh[q][tid] = 0u;
  }
  auto tally = [&](bool own) {
    if constexpr (GAS) {
      const int b = min(st.last, 7);
      if (own) s_nh[b >> 1][tid] += 1u << (16 * (b & 1));
    }
  };

  // The per-plane tables of the tile's rows, staged in LDS one plane ahead (double
  // buffered): the stationary flow at the cell centres (wc) and, for the gas, at the r
  // faces i0-1/2 .. i0+TM-1/2 (wr) and the z face above the plane (wz); the cells'
  // stationary conservative state (bgc) and gravity.  Thread t stages entry t: its
  // address is tab_p0 + plane * tab_stride.
  constexpr int T_WC = 0;
  constexpr int T_WR = T_WC + TM * WB_N;
  constexpr int T_WZ = T_WR + (GAS ? (TM + 1) * WB_N : 0);
  constexpr int T_BG = T_WZ + (GAS ? TM * WB_N : 0);
  constexpr int T_GR = T_BG + TM * 5;
  constexpr int NTAB = T_GR + TM * 2;
  static_assert(NTAB <= NTM, "one table entry per thread");
  __shared__ double s_tab[2][NTAB];
  const bool tab_t = tid < NTAB;
  const double* tab_p0 = nullptr;
  size_t tab_stride = 0;
  if (tab_t) {
    const size_t nr = (size_t)g.nr;
    if (tid < T_WR) {
      const int r = tid / WB_N, e = tid % WB_N;
      tab_p0 = a.t.wc + (size_t)min(i0 + r, g.nr - 1) * WB_N + e;
      tab_stride = nr * WB_N;
    } else if (tid < T_WZ) {
      const int f = (tid - T_WR) / WB_N, e = (tid - T_WR) % WB_N;
      tab_p0 = a.t.wr + (size_t)min(i0 + f, g.nr) * WB_N + e;
      tab_stride = (nr + 1) * WB_N;
    } else if (tid < T_BG) {
      const int r = (tid - T_WZ) / WB_N, e = (tid - T_WZ) % WB_N;
      tab_p0 = a.t.wz + (nr + (size_t)min(i0 + r, g.nr - 1)) * WB_N + e;
      tab_stride = nr * WB_N;
    } else if (tid < T_GR) {
      const int r = (tid - T_BG) / 5, e = (tid - T_BG) % 5;
      tab_p0 = a.t.bgc + (size_t)min(i0 + r, g.nr - 1) * 5 + e;
      tab_stride = nr * 5;
    } else {
      const int r = (tid - T_GR) / 2, e = (tid - T_GR) % 2;
      tab_p0 = a.t.grav + (size_t)min(i0 + r, g.nr - 1) * 2 + e;
      tab_stride = nr * 2;
    }
  }
  double dtmin = 1e300;
  // the largest signal speed of the thread's new cells (dust: its square).  The thread's
  // row (so its volume and largest face area) is fixed, and the CFL bound decreases with
  // the speed, so the bound of the largest speed, formed once after the march, is the
  // smallest one
  double smax = 0.0, vmax2 = 0.0;
  double tsmin = 1e300;  // smallest stopping time of the new state (drag law 1)
  double ledger = 0.0;

  const double* rt = a.t.rt + (size_t)igc * RT_N;
  const double Vc = rt[RT_V], invV = rt[RT_INVV], Ath = rt[RT_ATH], Az = rt[RT_AZ];
  const double invrc = rt[RT_INVRC], omk = rt[RT_OMK], maxA = rt[RT_MAXA];
  const double Arlo = a.t.ar[igc], Arhi = a.t.ar[igc + 1];
  const double Ar0 = a.t.ar[0];  // inner boundary face (ledger)

  // gas face: FP64 full states, or FP32 perturbations about the face background; the
  // cells' reconstructed variables, the stationary flow at the face (bf) and at the
  // centres of the two cells next to it (bB, bC: the positivity fallback)
  auto face = [&](auto dirc, const T* wA, const T* wB, const T* wC, const T* wD, const double* coB,
                  const double* coC, const double* bf, const double* bB, const double* bC, T* F) {
    constexpr int D = decltype(dirc)::value;
    if constexpr (PG) gas_face_p32<D>(gc, wA, wB, wC, wD, coB, coC, bf, bB, bC, F, st);
    else if constexpr (GAS) gas_face<D, G75>(gc, wA, wB, wC, wD, coB, coC, bf, bB, bC, F, st);
    else dust_face<D>(wA, wB, wC, wD, coB, coC, F, st);
  };
  using DR = std::integral_constant<int, 0>;
  using DT = std::integral_constant<int, 1>;
  using DZ = std::integral_constant<int, 2>;

  // z ring of the thread's column: e_{k-1}, e_k, e_{k+1}, e_{k+2}; fluxes below/above k
  T rm[NG], r0[NG], rp[NG], rn[NG], fzlo[NG], fzhi[NG];
  const int tslot = threadIdx.x;
  const bool twod = g.twod != 0;
  if (!twod) {
    T e2[NG];
    load_recon<P32, EXT, NG>(a, in, F0, k0 - 2, ig, jw, e2);
    load_recon<P32, EXT, NG>(a, in, F0, k0 - 1, ig, jw, rm);
    load_recon<P32, EXT, NG>(a, in, F0, k0, ig, jw, r0);
    load_recon<P32, EXT, NG>(a, in, F0, k0 + 1, ig, jw, rp);
    const double* bf = a.t.wz + ((size_t)k0 * g.nr + igc) * WB_N;
    face(DZ(), e2, rm, r0, rp, nullptr, nullptr, bf, bg_ptr(a, k0 - 1, igc), bg_ptr(a, k0, igc),
         fzlo);
    if (GAS) tally(act && k0 == 0);
    if (a.second && k0 == 0 && act) {
      double fm = (double)fzlo[NG - 1];
      if (PG) fm += bf[WB_RHO] * bf[WB_W];  // background normal mass flux rho0 w0
      ledger -= Az * fm;
    }
    if constexpr (LR) {
#pragma unroll
      for (int f = 0; f < NG; ++f) { s_rm[f][tslot] = rm[f]; s_fz[f][tslot] = fzlo[f]; }
    }
  } else {
    load_recon<P32, EXT, NG>(a, in, F0, 0, ig, jw, r0);
#pragma unroll
    for (int f = 0; f < NG; ++f) {
      rm[f] = T(0); rp[f] = T(0); rn[f] = T(0); fzlo[f] = T(0); fzhi[f] = T(0);
    }
  }

  // the halo ring of the LDS plane: two rows below and above the tile, then two columns
  // on each side of its rows; slot tid for every thread, and slot tid + NTM for the first
  // threads when the ring is larger than the workgroup (4-row tiles).  PF: the first slot
  // of each plane is loaded one plane ahead, so that its latency hides behind the previous
  // plane's face solves (not in the FP32-perturbation gas kernel, where the held registers
  // cost more than they hide).
  constexpr int HW = TJ + 4, NHALO = 4 * HW + 4 * TM;
  constexpr int NH2 = NHALO > NTM ? NHALO - NTM : 0;
  static_assert(NHALO <= 2 * NTM, "two halo cells per thread at most");
  auto halo_pos = [&](int h, int& rr, int& cc) {
    if (h < 2 * HW) { rr = h / HW; cc = h % HW; }
    else if (h < 4 * HW) { rr = TM + 2 + (h - 2 * HW) / HW; cc = (h - 2 * HW) % HW; }
    else { const int e = h - 4 * HW; rr = 2 + e / 4; cc = (e & 3) < 2 ? (e & 3) : TJ + (e & 3); }
  };
  const bool halo_t = tid < NHALO;
  int h_rr = 0, h_cc = 0;
  if (halo_t) halo_pos(tid, h_rr, h_cc);
  const int h_ii = i0 + h_rr - 2;
  const int h_jj = (j0 + h_cc - 2 + g.nth) % g.nth;
  const bool halo2 = NH2 > 0 && tid < NH2;
  int h2_rr = 0, h2_cc = 0;
  if (halo2) halo_pos(tid + NTM, h2_rr, h2_cc);
  const int h2_ii = i0 + h2_rr - 2;
  const int h2_jj = (j0 + h2_cc - 2 + g.nth) % g.nth;
  constexpr bool PF = !PG;
  T hv[NG];
  // dust: the next plane's first-slot halo and the column's cell k+2 are fetched raw at
  // the top of a plane and formed after the faces (the halo after the second barrier, the
  // column cell before the z face), so that no wait for them precedes the faces
  DustRaw<P32> hraw, nraw;
  // FP32 gas (base boundary options): the column's cell k+2 the same way; the next plane's
  // halo is requested after the second barrier, ahead of the drag's dust loads (one wait
  // for both), and formed before the update's stores
  constexpr bool RAWG = PG && !EXT;
  const float gm1f = (float)(g.gamma - 1.0);
  GasRaw32 gnraw, ghraw;
  if constexpr (RAWG) {
    if (halo_t) {
      gas_fetch32(a, in, k0, h_ii, h_jj, ghraw);
      gas_finish32(ghraw, gm1f, hv);
    }
  } else if constexpr (GAS) {
    if (PF && halo_t) load_recon<P32, EXT, NG>(a, in, F0, k0, h_ii, h_jj, hv);
  } else {
    if (halo_t) {
      dust_fetch<P32, EXT>(a, in, F0, k0, h_ii, h_jj, hraw);
      dust_finish<P32>(hraw, hv);
    }
  }

  if (tab_t) s_tab[k0 & 1][tid] = tab_p0[(size_t)k0 * tab_stride];
  // the radial parabola weights and limiter bounds of rows i0-1 .. i0+TM (plane
  // invariant), read by the r faces
  __shared__ double s_rco[(TM + 2) * RC_N];
  if (tid < (TM + 2) * RC_N) s_rco[tid] = rco_ptr(a, i0 - 1 + tid / RC_N)[tid % RC_N];

  // every load of the set-up done before the march: a load still in flight at the loop's
  // entry makes the compiler wait for all memory operations at the top of every plane,
  // the previous plane's stores included
  __builtin_amdgcn_s_waitcnt(0);
  for (int k = k0; k < k1; ++k) {
    if (!twod) {
      if constexpr (RAWG) gas_fetch32(a, in, k + 2, ig, jw, gnraw);
      else if constexpr (GAS) load_recon<P32, EXT, NG>(a, in, F0, k + 2, ig, jw, rn);
      else dust_fetch<P32, EXT>(a, in, F0, k + 2, ig, jw, nraw);
    }
    const int kb = k & 1;
    double tab_next = 0.0;
    if (tab_t && k + 1 < k1) tab_next = tab_p0[(size_t)(k + 1) * tab_stride];
    // the update's base values of this plane's cell and (dust) the gas state the drag
    // needs, requested here so that their latency hides behind the face solves.  Stage 1
    // of the FP32 dust layout reads its base from r0 (the same cell of the same state).
    const size_t cell = ((size_t)k * g.nr + ig) * g.nth + jg;
    const size_t cellw = ((size_t)k * g.nr + igc) * g.nth + jw;
    const bool upd = a.mode == MODE_UPDATE && act;
    const bool base_r0 = P32 && !GAS && a.base == a.in;
    // (raw stored values: any arithmetic on them here would wait for the loads)
    using BT = typename std::conditional<PG, float, double>::type;
    BT pb[NG];
    float pvel[P32 && !GAS ? 3 : 1];  // FP32 dust layout: stored velocity deviations
    // (the FP32 gas kernel requests them after the second barrier instead, with the drag's
    // loads: held across the faces they would spill)
    auto load_base_pg = [&]() {
      if (upd) {
#pragma unroll
        for (int f = 0; f < NG; ++f) pb[f] = ((const float*)a.base)[(size_t)f * g.N + cell];
      }
    };
    if (upd && !base_r0) {
      if constexpr (PG) {
        if constexpr (!RAWG) load_base_pg();
      } else if constexpr (P32 && !GAS) {
        const float* vel = (const float*)a.base + (size_t)(5 + 3 * species) * g.N + cell;
        pb[3] = ((const double*)a.base)[p32_f64_base(g) + (size_t)species * g.N + cell];
        pvel[0] = vel[0];
        pvel[1] = vel[g.N];
        pvel[2] = vel[2 * (size_t)g.N];
      } else {
        load_cons<P32, NG>(a, a.base, F0, k, ig, jg, pb);
      }
    }
    using GT = typename std::conditional<P32, float, double>::type;
    GT pg[GAS ? 1 : 5];
    if constexpr (!GAS) {
      if (drag) {
#pragma unroll
        for (int f = 0; f < 5; ++f) pg[f] = ((const GT*)in)[(size_t)f * g.N + cellw];
      }
    }
    // ---- stage the plane (with halo) in LDS
#pragma unroll
    for (int f = 0; f < NG; ++f) s_pl[f][ti + 2][tj + 2] = r0[f];
    if (halo_t) {
      if constexpr (GAS && !RAWG) {
        if (!PF) load_recon<P32, EXT, NG>(a, in, F0, k, h_ii, h_jj, hv);
      }
#pragma unroll
      for (int f = 0; f < NG; ++f) s_pl[f][h_rr][h_cc] = hv[f];
      if constexpr (GAS) {
        if (PF && k + 1 < k1) load_recon<P32, EXT, NG>(a, in, F0, k + 1, h_ii, h_jj, hv);
      } else {
        if (k + 1 < k1) dust_fetch<P32, EXT>(a, in, F0, k + 1, h_ii, h_jj, hraw);
      }
    }
    if constexpr (NH2 > 0) {
      if (halo2) {
        T hv2[NG];
        load_recon<P32, EXT, NG>(a, in, F0, k, h2_ii, h2_jj, hv2);
#pragma unroll
        for (int f = 0; f < NG; ++f) s_pl[f][h2_rr][h2_cc] = hv2[f];
      }
    }
    __syncthreads();
    // ---- theta face j+1/2 and r face i+1/2 of this cell
    {
      T eA[NG], eB[NG], eC[NG], eD[NG], F[NG];
#pragma unroll
      for (int f = 0; f < NG; ++f) {
        eA[f] = s_pl[f][ti + 2][tj + 1]; eB[f] = s_pl[f][ti + 2][tj + 2];
        eC[f] = s_pl[f][ti + 2][tj + 3]; eD[f] = s_pl[f][ti + 2][tj + 4];
      }
      {
        const double* bf = &s_tab[kb][T_WC + ti * WB_N];
        face(DT(), eA, eB, eC, eD, nullptr, nullptr, bf, bf, bf, F);
        if (GAS) tally(act);
      }
#pragma unroll
      for (int f = 0; f < NG; ++f) s_ft[f][ti][tj + 1] = F[f];
#pragma unroll
      for (int f = 0; f < NG; ++f) {
        eA[f] = s_pl[f][ti + 1][tj + 2]; eB[f] = s_pl[f][ti + 2][tj + 2];
        eC[f] = s_pl[f][ti + 3][tj + 2]; eD[f] = s_pl[f][ti + 4][tj + 2];
      }
      {
        const double* bf = GAS ? &s_tab[kb][T_WR + (ti + 1) * WB_N] : nullptr;
        face(DR(), eA, eB, eC, eD, &s_rco[(ti + 1) * RC_N], &s_rco[(ti + 2) * RC_N], bf,
             bg_ptr(a, k, min(ig, g.nr)), bg_ptr(a, k, min(ig + 1, g.nr)), F);
        if (GAS) tally(act);
        if (a.second && act && ig == g.nr - 1) {
          double fm = (double)F[NG - 1];
          if (PG) fm += bf[WB_RHO] * bf[WB_U];  // background normal mass flux rho0 u0
          ledger += Arhi * fm;
        }
      }
#pragma unroll
      for (int f = 0; f < NG; ++f) s_fr[f][ti + 1][tj] = F[f];
    }
    // ---- lower-edge faces of the tile: r face i0-1/2 (threads 0..63) and theta face
    //      j0-1/2 of each row (threads 64..71)
    if (tid < TJ) {
      T eA[NG], eB[NG], eC[NG], eD[NG], F[NG];
      const int col = tid;
#pragma unroll
      for (int f = 0; f < NG; ++f) {
        eA[f] = s_pl[f][0][col + 2]; eB[f] = s_pl[f][1][col + 2];
        eC[f] = s_pl[f][2][col + 2]; eD[f] = s_pl[f][3][col + 2];
      }
      const double* bf = GAS ? &s_tab[kb][T_WR] : nullptr;
      face(DR(), eA, eB, eC, eD, &s_rco[0], &s_rco[RC_N], bf, bg_ptr(a, k, i0 - 1),
           bg_ptr(a, k, i0), F);
      // the tile's lower r face is the upper face of the tile below, except at the inner
      // boundary
      if (GAS) tally(i0 == 0 && j0 + col < g.nth);
#pragma unroll
      for (int f = 0; f < NG; ++f) s_fr[f][0][col] = F[f];
      if (a.second && i0 == 0 && j0 + col < g.nth) {
        double fm = (double)F[NG - 1];
        if (PG) fm += bf[WB_RHO] * bf[WB_U];
        ledger -= Ar0 * fm;
      }
    } else if (tid < TJ + TM) {
      T eA[NG], eB[NG], eC[NG], eD[NG], F[NG];
      const int row = tid - TJ;
#pragma unroll
      for (int f = 0; f < NG; ++f) {
        eA[f] = s_pl[f][row + 2][0]; eB[f] = s_pl[f][row + 2][1];
        eC[f] = s_pl[f][row + 2][2]; eD[f] = s_pl[f][row + 2][3];
      }
      const double* bf = &s_tab[kb][T_WC + row * WB_N];
      face(DT(), eA, eB, eC, eD, nullptr, nullptr, bf, bf, bf, F);
#pragma unroll
      for (int f = 0; f < NG; ++f) s_ft[f][row][0] = F[f];
    }
    // ---- z face k+1/2 from the register ring
    if (!twod) {
      if constexpr (RAWG) gas_finish32(gnraw, gm1f, rn);
      else if constexpr (!GAS) dust_finish<P32>(nraw, rn);
      if constexpr (LR) {
#pragma unroll
        for (int f = 0; f < NG; ++f) rm[f] = s_rm[f][tslot];
      }
      const double* bf = GAS ? &s_tab[kb][T_WZ + ti * WB_N] : nullptr;
      face(DZ(), rm, r0, rp, rn, nullptr, nullptr, bf, bg_ptr(a, k, igc), bg_ptr(a, k + 1, igc),
           fzhi);
      if (GAS) tally(act);
      if (a.second && act && k == g.nz - 1) {
        double fm = (double)fzhi[NG - 1];
        if (PG) fm += bf[WB_RHO] * bf[WB_W];
        ledger += Az * fm;
      }
    }
    __syncthreads();
    // ---- the next plane's tables (read after the next plane's first barrier; buffer
    //      (k + 1) & 1 was last read before this plane's first barrier) and the dust halo;
    //      both here, before this plane's stores, so that waiting for them waits for no store
    if (tab_t && k + 1 < k1) s_tab[(k + 1) & 1][tid] = tab_next;
    if constexpr (!GAS) {
      if (halo_t && k + 1 < k1) dust_finish<P32>(hraw, hv);
    }
    if constexpr (RAWG) {
      load_base_pg();
      if (halo_t && k + 1 < k1) gas_fetch32(a, in, k + 1, h_ii, h_jj, ghraw);
    }
    // ---- divergence -sum_s A_s F.n_s (Sect. 2.2), sources (App. B), drag (Sect. 2.9)
    T Gd[NG];
#pragma unroll
    for (int f = 0; f < NG; ++f) {
      T dr = T(Arhi) * s_fr[f][ti + 1][tj] - T(Arlo) * s_fr[f][ti][tj];
      T dth = T(Ath) * (s_ft[f][ti][tj + 1] - s_ft[f][ti][tj]);
      T dz = twod ? T(0) : T(Az) * (fzhi[f] - (LR ? s_fz[f][tslot] : fzlo[f]));
      Gd[f] = -((dr + dth) + dz);
    }
    const double gr = s_tab[kb][T_GR + ti * 2 + 0];
    const double gz = s_tab[kb][T_GR + ti * 2 + 1];
    const double* bgc = &s_tab[kb][T_BG + ti * 5];
    const double* bw = &s_tab[kb][T_WC + ti * WB_N];
    T S[NG];
    if constexpr (PG) {
      // source change S(E) - S(E0), every term formed from the perturbations W' (the
      // stationary flow has no radial or vertical velocity)
      const float rp = r0[4], up = r0[0], vp = r0[1], wp = r0[2], pp = r0[3];
      const float v0 = (float)bw[WB_V];
      const float rho = (float)(bw[WB_RHO] + (double)rp);
      const float ir = (float)invrc, fgr = (float)gr, fgz = (float)gz;
      const float dmv2 = rp * (float)(bw[WB_V] * bw[WB_V]) + rho * vp * (2.0f * v0 + vp);
      S[0] = (dmv2 + pp) * ir + rp * fgr;
      S[1] = -(rho * up * (v0 + vp)) * ir;
      S[2] = rp * fgz;
      S[3] = rho * (up * fgr + wp * fgz);
      S[4] = 0.0f;
      if (drag) {
        const double rg = bw[WB_RHO] + (double)rp;
        const double u = (double)up, v = bw[WB_V] + (double)vp, w2 = (double)wp;
        const double pq = (EXT && g.drag_law) ? bw[WB_P] + (double)pp : 0.0;
        double dx = 0.0, dy = 0.0, dzz = 0.0;
        // every species' density and velocities requested together (loads made
        // conditional on the density would each wait for it)
        double rds[ND > 0 ? ND : 1];
        float vds[ND > 0 ? ND : 1][3];
#pragma unroll
        for (int s2 = 0; s2 < ND; ++s2) {
          const float* vel = (const float*)in + (size_t)(5 + 3 * s2) * g.N + cellw;
          rds[s2] = ld_cell<P32>(a, in, 5 + 4 * s2 + 3, k, igc, cellw);
          vds[s2][0] = vel[0];
          vds[s2][1] = vel[g.N];
          vds[s2][2] = vel[2 * (size_t)g.N];
        }
#pragma unroll
        for (int s2 = 0; s2 < ND; ++s2) {
          // the FP32 layout stores the dust velocities as deviations from the stationary
          // flow's, as the gas W' is: the velocity difference is formed from the deviations
          const double rd = rds[s2];
          const bool full = rd > 0.0;
          const double dud = full ? (double)vds[s2][0] - (double)up : -u;
          const double dvd = full ? (double)vds[s2][1] - (double)vp : -v;
          const double dwd = full ? (double)vds[s2][2] - (double)wp : -w2;
          const double its = inv_tstop<EXT>(g, s2, omk, rg, pq);
          dx += rd * dud * its;
          dy += rd * dvd * its;
          dzz += rd * dwd * its;
        }
        S[0] += (float)dx;
        S[1] += (float)dy;
        S[2] += (float)dzz;
        S[3] += (float)(u * dx + v * dy + w2 * dzz);
      }
    } else if constexpr (GAS) {
      // the cell's primitives: stationary flow + W'
      const double rho = bw[WB_RHO] + r0[4];
      const double u = bw[WB_U] + r0[0], v = bw[WB_V] + r0[1], w = bw[WB_W] + r0[2];
      const double p = bw[WB_P] + r0[3];
      S[0] = (rho * v * v + p) * invrc + rho * gr;
      S[1] = -(rho * u * v) * invrc;
      S[2] = rho * gz;
      S[3] = rho * (u * gr + w * gz);
      S[4] = 0.0;
      if (drag) {
        double dx = 0.0, dy = 0.0, dzz = 0.0;
        // every species' variables requested together (see the FP32 branch)
        double dvar[ND > 0 ? ND : 1][4];
#pragma unroll
        for (int s2 = 0; s2 < ND; ++s2)
#pragma unroll
          for (int c = 0; c < 4; ++c) dvar[s2][c] = ld_cell<P32>(a, in, 5 + 4 * s2 + c, k, igc, cellw);
#pragma unroll
        for (int s2 = 0; s2 < ND; ++s2) {
          const double rd = dvar[s2][3];
          double ud = 0.0, vd = 0.0, wd = 0.0;
          if (rd > 0.0) {
            double id = 1.0 / rd;
            ud = dvar[s2][0] * id;
            vd = dvar[s2][1] * id;
            wd = dvar[s2][2] * id;
          }
          const double its = inv_tstop<EXT>(g, s2, omk, rho, p);
          dx += rd * (ud - u) * its;
          dy += rd * (vd - v) * its;
          dzz += rd * (wd - w) * its;
        }
        S[0] += dx;
        S[1] += dy;
        S[2] += dzz;
        S[3] += u * dx + v * dy + w * dzz;
      }
    } else {
      // the dust cell's primitives (velocity zero where the density is not positive)
      const double rd = r0[3], ud = r0[0], vd = r0[1], wd = r0[2];
      double fx = 0.0, fy = 0.0, fz = 0.0;
      if (drag) {
        double q[5];
#pragma unroll
        for (int f = 0; f < 5; ++f) q[f] = bgc[f] + (double)pg[f];
        const double inv = 1.0 / q[4];
        const double u = q[0] * inv, v = q[1] * inv, w = q[2] * inv;
        const double pq = (EXT && g.drag_law) ? gc.gm1 * (q[3] - 0.5 * (q[0] * u + q[1] * v + q[2] * w)) : 0.0;
        const double its = inv_tstop<EXT>(g, species, omk, q[4], pq);
        fx = rd * (ud - u) * its;
        fy = rd * (vd - v) * its;
        fz = rd * (wd - w) * its;
      }
      S[0] = (rd * vd * vd) * invrc + rd * gr - fx;
      S[1] = -(rd * ud * vd) * invrc - fy;
      S[2] = rd * gz - fz;
      S[3] = 0.0;
    }
    // indirect gravity (Sect. 2.10): minus the star's acceleration by the disc
    if (EXT && g.indirect && a.mode != MODE_RESID) {
      const double A = a.t.indab[0], B = a.t.indab[1];
      const double cs = a.t.trig[jw], sn = a.t.trig[g.nth + jw];
      const double ar = -g.GM * (A * cs + B * sn), at = -g.GM * (B * cs - A * sn);
      if constexpr (GAS) {
        const double rho = bw[WB_RHO] + (double)r0[4];
        const double mr = rho * (bw[WB_U] + (double)r0[0]), mt = rho * (bw[WB_V] + (double)r0[1]);
        S[0] += (T)(rho * ar);
        S[1] += (T)(rho * at);
        S[3] += (T)(mr * ar + mt * at);
      } else {
        S[0] += r0[3] * ar;
        S[1] += r0[3] * at;
      }
    }
    // boundary damping zones (Sect. 2.4): the gas deviation relaxes to the stationary flow
    if (EXT && GAS && g.damp) {
      const double kd = a.t.damp[(size_t)k * g.nr + igc];
      double e[NG];
      load_cons<P32, NG>(a, in, F0, k, igc, jw, e);
#pragma unroll
      for (int f = 0; f < NG; ++f) S[f] -= (T)(kd * e[f]);
    }
    if constexpr (RAWG) {
      if (halo_t && k + 1 < k1) gas_finish32(ghraw, gm1f, hv);
    }
    T Gt[NG];
#pragma unroll
    for (int f = 0; f < NG; ++f) Gt[f] = fma(S[f], T(Vc), Gd[f]);
    if (GAS && !P32 && a.mode != MODE_RESID) {
      const double* R0 = a.t.r0 + ((size_t)k * g.nr + igc) * 5;
#pragma unroll
      for (int f = 0; f < NG; ++f) Gt[f] -= (T)R0[f];
    }
    if (a.mode == MODE_RESID) {
      if (GAS && act && jg == 0) {
#pragma unroll
        for (int f = 0; f < NG; ++f) a.c.r0w[((size_t)k * g.nr + ig) * 5 + f] = (double)Gt[f];
      }
    } else if (a.mode == MODE_OPER) {
      if (act) {
#pragma unroll
        for (int f = 0; f < NG; ++f) {
          if (P32) ((float*)a.out)[(size_t)(F0 + f) * g.N + cell] = (float)Gt[f];
          else ((double*)a.out)[(size_t)(F0 + f) * g.N + cell] = (double)Gt[f];
        }
      }
    } else if (act) {
      // all loads before any store (the second stage updates in place).  The FP32 gas
      // kernel stores after its positivity and CFL arithmetic, so that a wait there (a
      // register reload) comes before the stores rather than waiting for them; the others
      // store first (their registers prefer it)
      double nvd[NG];
      float nv[PG ? NG : 1];
      auto store_new = [&]() {
        if constexpr (PG) {
#pragma unroll
          for (int f = 0; f < NG; ++f) ((float*)a.out)[(size_t)f * g.N + cell] = nv[f];
        } else if constexpr (!P32 || GAS) {
#pragma unroll
          for (int f = 0; f < NG; ++f) st_cell<P32>(a, a.out, F0 + f, k, ig, cell, nvd[f]);
        } else {
          // FP32 dust velocities are formed with the new density
          st_dust32(a, a.out, species, cell, nvd, bw[WB_V]);
        }
      };
      if constexpr (PG) {
        const float cdt = (float)(a.coef * dt * invV);
#pragma unroll
        for (int f = 0; f < NG; ++f) {
          nv[f] = fma(cdt, Gt[f], pb[f]);
          nvd[f] = (double)nv[f];
        }
      } else {
        const double cdt = a.coef * dt * invV;
        double bv[NG];
        if (base_r0) {
          // load_cons of the FP32 dust layout: density times (stored velocity deviation +
          // stationary velocity), the stored deviation being zero where the density is not
          // positive
          const double rd = (double)r0[3];
          const double v0 = bw[WB_V];
          bv[0] = rd * (double)r0[0];
          bv[1] = rd * (rd > 0.0 ? (double)r0[1] : v0);
          bv[2] = rd * (double)r0[2];
          bv[3] = rd;
        } else if constexpr (P32 && !GAS) {
          // load_cons of the FP32 dust layout
          bv[0] = pb[3] * (double)pvel[0];
          bv[1] = pb[3] * (bw[WB_V] + (double)pvel[1]);
          bv[2] = pb[3] * (double)pvel[2];
          bv[3] = pb[3];
        } else {
#pragma unroll
          for (int f = 0; f < NG; ++f) bv[f] = (double)pb[f];
        }
#pragma unroll
        for (int f = 0; f < NG; ++f) nvd[f] = fma(cdt, (double)Gt[f], bv[f]);
        store_new();
      }
      if (GAS) {
        // positivity of the new gas state; CFL of the new state (second stage)
        double qn[5];
#pragma unroll
        for (int f = 0; f < 5; ++f) qn[f] = bgc[f] + nvd[f];
        const double in2 = 1.0 / qn[4];
        const double un = qn[0] * in2, vn = qn[1] * in2, wn = qn[2] * in2;
        const double pn = gc.gm1 * (qn[3] - 0.5 * (qn[0] * un + qn[1] * vn + qn[2] * wn));
        if (!(qn[4] > 0.0 && pn > 0.0)) {
          atomicOr(&a.c.ctrl->status, FL_NEG);
          atomicMin(&a.c.ctrl->first_bad, (unsigned long long)cell);
          atomicCAS(&a.c.ctrl->bad_step, -1, a.step);
        } else if (a.second) {
          double spd = sqrt(un * un + vn * vn + wn * wn) + sqrt(gc.g * pn * in2);
          smax = fmax(smax, spd);
          if (EXT && g.drag_law) {
#pragma unroll
            for (int s2 = 0; s2 < ND; ++s2) tsmin = fmin(tsmin, 1.0 / inv_tstop<EXT>(g, s2, omk, qn[4], pn));
          }
        }
      } else if (a.second && nvd[3] < 0.0) {
        st.negd++;
      } else if (a.second && nvd[3] > 0.0) {
        double id = 1.0 / nvd[3];
        double a1 = nvd[0] * id, a2 = nvd[1] * id, a3 = nvd[2] * id;
        vmax2 = fmax(vmax2, a1 * a1 + a2 * a2 + a3 * a3);
      }
      if constexpr (PG) store_new();
    }
    // ---- shift the ring
#pragma unroll
    for (int f = 0; f < NG; ++f) {
      if constexpr (LR) {
        s_rm[f][tslot] = r0[f]; s_fz[f][tslot] = fzhi[f];
      } else {
        rm[f] = r0[f]; fzlo[f] = fzhi[f];
      }
      r0[f] = rp[f]; rp[f] = rn[f];
    }
  }

  // ---- block reductions: counters, CFL partial, boundary outflow partial
  if constexpr (!GAS) smax = sqrt(vmax2);
  if (smax > 0.0) dtmin = g.cfl * Vc / (smax * maxA);
  const int wv = tid / 64, ln = tid & 63;
  int nf_ = wave_isum(st.fall), nv_ = wave_isum(st.vac), mi_ = wave_imax(st.maxit);
  int nc_ = wave_imax(st.noconv), nr_ = wave_isum(st.resolve), nd_ = GAS ? 0 : wave_isum(st.negd);
  if constexpr (GAS) {
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const int hb = wave_isum((int)((s_nh[b >> 1][tid] >> (16 * (b & 1))) & 0xffffu));
      if (ln == 0 && hb) atomicAdd(&a.c.ctrl->newton_hist[b], (unsigned long long)hb);
    }
  }
  if (ln == 0) {
    if (nd_) atomicAdd(&a.c.ctrl->nnegd, (unsigned long long)nd_);
    if (nf_) atomicAdd(&a.c.ctrl->nfall, (unsigned long long)nf_);
    if (nv_) { atomicAdd(&a.c.ctrl->nvac, (unsigned long long)nv_); atomicOr(&a.c.ctrl->status, FL_VAC); }
    if (mi_) atomicMax(&a.c.ctrl->maxit, mi_);
    if (nr_) atomicAdd(&a.c.ctrl->nresolve, (unsigned long long)nr_);
    if (nc_) { atomicOr(&a.c.ctrl->status, FL_NOCONV); atomicCAS(&a.c.ctrl->bad_step, -1, a.step); }
  }
  if (a.second && a.mode == MODE_UPDATE) {
    double m = wave_min(dtmin);
    double ls = wave_sum(ledger);
    double tm = (EXT && GAS && ND > 0) ? wave_min(tsmin) : 1e300;
    if (ln == 0) { s_red[wv][0] = m; s_red[wv][1] = ls; s_red[wv][2] = tm; }
    __syncthreads();
    if (tid == 0) {
      double mm = s_red[0][0], lsum = s_red[0][1], tmm = s_red[0][2];
      for (int w2 = 1; w2 < NTM / 64; ++w2) {
        mm = fmin(mm, s_red[w2][0]);
        lsum += s_red[w2][1];
        tmm = fmin(tmm, s_red[w2][2]);
      }
      a.c.cflp[(size_t)blockIdx.x * 5 + slot] = mm;
      a.c.outp[(size_t)blockIdx.x * 5 + slot] = lsum;
      if (EXT && GAS && g.drag_law) a.c.tsp[blockIdx.x] = tmm;
    }
  }
}

// ------------------------------------------------------------------------------------
// standalone CFL of a state (start of a call) with the positivity check

template <int ND, bool P32>
__global__ void __launch_bounds__(256) k_cfl(StageArgs a, const void* state) {
  __shared__ double s_m[4];
  __shared__ double s_t[4];
  const Geo& g = a.g;
  double dtmin = 1e300, tsmin = 1e300;
  const double gm1 = g.gamma - 1.0;
  for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < g.N;
       c += (size_t)gridDim.x * blockDim.x) {
    const size_t ki = c / g.nth;
    const int i = (int)(ki % g.nr);
    const double* bgc = a.t.bgc + ki * 5;
    const int k = (int)(ki / g.nr);
    double q[5];
#pragma unroll
    for (int f = 0; f < 5; ++f) q[f] = bgc[f] + ld_cell<P32>(a, state, f, k, i, c);
    const double in2 = 1.0 / q[4];
    const double u = q[0] * in2, v = q[1] * in2, w = q[2] * in2;
    const double p = gm1 * (q[3] - 0.5 * (q[0] * u + q[1] * v + q[2] * w));
    if (!(q[4] > 0.0 && p > 0.0)) {
      atomicOr(&a.c.ctrl->status, FL_NEG);
      atomicMin(&a.c.ctrl->first_bad, (unsigned long long)c);
      atomicCAS(&a.c.ctrl->bad_step, -1, a.step);
      continue;
    }
    double spd = sqrt(u * u + v * v + w * w) + sqrt(g.gamma * p * in2);
#pragma unroll
    for (int s = 0; s < ND; ++s) {
      const int o = 5 + 4 * s;
      double rd = ld_cell<P32>(a, state, o + 3, k, i, c);
      if (rd > 0.0) {
        double id = 1.0 / rd;
        double a1 = ld_cell<P32>(a, state, o, k, i, c) * id;
        double a2 = ld_cell<P32>(a, state, o + 1, k, i, c) * id;
        double a3 = ld_cell<P32>(a, state, o + 2, k, i, c) * id;
        spd = fmax(spd, sqrt(a1 * a1 + a2 * a2 + a3 * a3));
      }
    }
    const double* rt = a.t.rt + (size_t)i * RT_N;
    dtmin = fmin(dtmin, g.cfl * rt[RT_V] / (spd * rt[RT_MAXA]));
    if (g.drag_law) {
#pragma unroll
      for (int s = 0; s < ND; ++s) tsmin = fmin(tsmin, 1.0 / inv_tstop(g, s, rt[RT_OMK], q[4], p));
    }
  }
  double m = wave_min(dtmin);
  double tm = wave_min(tsmin);
  if ((threadIdx.x & 63) == 0) { s_m[threadIdx.x / 64] = m; s_t[threadIdx.x / 64] = tm; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double mm = fmin(fmin(s_m[0], s_m[1]), fmin(s_m[2], s_m[3]));
    a.c.cflp[blockIdx.x] = mm;
    if (g.drag_law) a.c.tsp[blockIdx.x] = fmin(fmin(s_t[0], s_t[1]), fmin(s_t[2], s_t[3]));
  }
}

// ------------------------------------------------------------------------------------
// the drag alone over a part of the step, exactly (split integration of the Sect. 2.9
// forces for steps that may exceed the stopping times)
//
// With the densities and the stopping times of a cell held, the total momentum of each
// velocity component is constant and the dust-gas velocity differences d_s = u_s - u_g
// (species with rho_s > 0) obey dd/dt = B d, B_ab = -eps_b / t_b - [a == b] / t_a,
// eps_b = rho_b / rho_g, so d(tau) = exp(tau B) d(0).  exp(tau B) is taken by scaling
// and squaring: X = tau B / 2^s with |X| (largest absolute row sum) <= 1/8, the Taylor
// polynomial of degree 12 in Horner form (remainder below 1e-21), then s squarings; B's
// eigenvalues are negative, so the squarings do not amplify rounding.  New velocities:
// u_g = (P - sum rho_s d_s) / (rho_g + sum rho_s), u_s = u_g + d_s; the gas energy changes
// by the gas kinetic-energy change (the pressure is unchanged).

template <int ND>
__device__ __forceinline__ void mat_mul(const double* A, const double* B, double* C) {
#pragma unroll
  for (int r = 0; r < ND; ++r)
#pragma unroll
    for (int c = 0; c < ND; ++c) {
      double acc = 0.0;
#pragma unroll
      for (int m = 0; m < ND; ++m) acc = fma(A[r * ND + m], B[m * ND + c], acc);
      C[r * ND + c] = acc;
    }
}

template <int ND, bool P32>
__global__ void __launch_bounds__(256) k_drag(StageArgs a, void* state, double frac) {
  __shared__ int s_stop;
  if (threadIdx.x == 0) s_stop = __atomic_load_n(&a.c.ctrl->status, __ATOMIC_RELAXED);
  __syncthreads();
  if (s_stop & FL_HARD) return;
  const Geo& g = a.g;
  const double tau = frac * a.c.dtlog[a.dt_idx];
  const double gm1 = g.gamma - 1.0;
  for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < g.N;
       c += (size_t)gridDim.x * blockDim.x) {
    const size_t ki = c / g.nth;
    const int i = (int)(ki % g.nr);
    const int k = (int)(ki / g.nr);
    const double* bgc = a.t.bgc + ki * 5;
    double q[5];
#pragma unroll
    for (int f = 0; f < 5; ++f) q[f] = bgc[f] + ld_cell<P32>(a, state, f, k, i, c);
    const double rho = q[4], ir = 1.0 / rho;
    double ug[3] = {q[0] * ir, q[1] * ir, q[2] * ir};
    const double p = gm1 * (q[3] - 0.5 * (q[0] * ug[0] + q[1] * ug[1] + q[2] * ug[2]));
    const double omk = a.t.rt[(size_t)i * RT_N + RT_OMK];
    const double v0 = a.t.wc[ki * WB_N + WB_V];
    double rd[ND], ia[ND], ud[ND][3];
    double mtot = rho;
    bool any = false;
#pragma unroll
    for (int s = 0; s < ND; ++s) {
      const int o = 5 + 4 * s;
      rd[s] = ld_cell<P32>(a, state, o + 3, k, i, c);
      const bool on = rd[s] > 0.0;
      any = any || on;
      if constexpr (P32) {
        const float* vel = (const float*)state + (size_t)(5 + 3 * s) * g.N + c;
        ud[s][0] = (double)vel[0];
        ud[s][1] = v0 + (double)vel[g.N];
        ud[s][2] = (double)vel[2 * g.N];
      } else {
        const double id = on ? 1.0 / rd[s] : 0.0;
#pragma unroll
        for (int d = 0; d < 3; ++d) ud[s][d] = ((const double*)state)[(size_t)(o + d) * g.N + c] * id;
      }
      ia[s] = on ? inv_tstop<true>(g, s, omk, rho, p) : 0.0;
      if (on) mtot += rd[s];
      else rd[s] = 0.0;
    }
    if (!any) continue;
    // exp(tau B)
    double X[ND * ND], M[ND * ND], T[ND * ND];
    double nrm = 0.0;
#pragma unroll
    for (int r = 0; r < ND; ++r) {
      double row = 0.0;
#pragma unroll
      for (int b = 0; b < ND; ++b) {
        X[r * ND + b] = -(rd[b] * ir) * ia[b] - (r == b ? ia[r] : 0.0);
        row += fabs(X[r * ND + b]);
      }
      nrm = fmax(nrm, row * tau);
    }
    int sq = 0;
    while (nrm > 0.125 && sq < 1100) { nrm *= 0.5; ++sq; }  // bounded for a non-finite norm
    const double sc = ldexp(tau, -sq);
#pragma unroll
    for (int e = 0; e < ND * ND; ++e) X[e] *= sc;
    // Horner: M = I + X/12, then M = I + (X/k) M for k = 11 .. 1
#pragma unroll
    for (int e = 0; e < ND * ND; ++e) M[e] = X[e] * (1.0 / 12.0) + ((e / ND) == (e % ND) ? 1.0 : 0.0);
#pragma unroll
    for (int kk = 11; kk >= 1; --kk) {
      mat_mul<ND>(X, M, T);
      const double ik = 1.0 / (double)kk;
#pragma unroll
      for (int e = 0; e < ND * ND; ++e) M[e] = fma(T[e], ik, (e / ND) == (e % ND) ? 1.0 : 0.0);
    }
    for (int r = 0; r < sq; ++r) {
      mat_mul<ND>(M, M, T);
#pragma unroll
      for (int e = 0; e < ND * ND; ++e) M[e] = T[e];
    }
    // relax each component
    double dke = 0.0;
    const double imt = 1.0 / mtot;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      double P = q[d], d0[ND];
#pragma unroll
      for (int s = 0; s < ND; ++s) {
        P += rd[s] * ud[s][d];
        d0[s] = rd[s] > 0.0 ? ud[s][d] - ug[d] : 0.0;
      }
      double pd = 0.0, d1[ND];
#pragma unroll
      for (int s = 0; s < ND; ++s) {
        double acc = 0.0;
#pragma unroll
        for (int b = 0; b < ND; ++b) acc = fma(M[s * ND + b], d0[b], acc);
        d1[s] = acc;
        pd += rd[s] * acc;
      }
      const double ug1 = (P - pd) * imt;
      dke += 0.5 * rho * (ug1 * ug1 - ug[d] * ug[d]);
      st_cell<P32>(a, state, d, k, i, c, rho * ug1 - bgc[d]);
#pragma unroll
      for (int s = 0; s < ND; ++s) {
        if (!(rd[s] > 0.0)) continue;
        if constexpr (P32) {
          const double u1 = ug1 + d1[s] - (d == 1 ? v0 : 0.0);
          ((float*)state)[(size_t)(5 + 3 * s + d) * g.N + c] = (float)u1;
        } else {
          ((double*)state)[(size_t)(5 + 4 * s + d) * g.N + c] = rd[s] * (ug1 + d1[s]);
        }
      }
    }
    st_cell<P32>(a, state, 3, k, i, c, q[3] + dke - bgc[3]);
  }
}

// final reduction after a step: next dt (CFL), stiffness check, boundary outflow ledger
__global__ void __launch_bounds__(256) k_reduce(StageArgs a, int nparts, int dt_next, int want_dt,
                                                int want_ledger) {
  __shared__ double s_m[4];
  __shared__ double s_ts[4];
  __shared__ double s_l[4][5];
  __shared__ int s_stop;
  if (threadIdx.x == 0) s_stop = __atomic_load_n(&a.c.ctrl->status, __ATOMIC_RELAXED);
  __syncthreads();
  if (s_stop & FL_HARD) return;
  double m = 1e300, tsm = 1e300;
  double l[5] = {0, 0, 0, 0, 0};
  const bool dyn_ts = a.g.drag_law && a.g.nd > 0;
  // fixed partition and order: deterministic sums
  // stage partials: [nparts][5] (gas, dust species); standalone CFL: [nparts]
  const int per = want_ledger ? 1 + a.g.nd : 1;
  for (int b = threadIdx.x; b < nparts; b += blockDim.x) {
    if (dyn_ts) tsm = fmin(tsm, a.c.tsp[b]);
    if (want_dt)
      for (int s = 0; s < per; ++s) m = fmin(m, a.c.cflp[want_ledger ? (size_t)b * 5 + s : b]);
    if (want_ledger)
#pragma unroll
      for (int s = 0; s < 5; ++s) l[s] += a.c.outp[(size_t)b * 5 + s];
  }
  m = wave_min(m);
  tsm = wave_min(tsm);
#pragma unroll
  for (int s = 0; s < 5; ++s) l[s] = wave_sum(l[s]);
  if ((threadIdx.x & 63) == 0) {
    s_m[threadIdx.x / 64] = m;
    s_ts[threadIdx.x / 64] = tsm;
#pragma unroll
    for (int s = 0; s < 5; ++s) s_l[threadIdx.x / 64][s] = l[s];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    if (want_dt) {
      double mm = fmin(fmin(s_m[0], s_m[1]), fmin(s_m[2], s_m[3]));
      a.c.dtlog[dt_next] = mm;
    }
    if (want_ledger)
#pragma unroll
      for (int s = 0; s < 5; ++s)
        a.c.ctrl->outflow[s] = ((s_l[0][s] + s_l[1][s]) + (s_l[2][s] + s_l[3][s]));
    double dtn = a.c.dtlog[dt_next];
    // stiffness: dt against the smallest stopping time (constant law: from the tables;
    // law 1: over the cells of the state the step starts from)
    const double tsmin = dyn_ts ? fmin(fmin(s_ts[0], s_ts[1]), fmin(s_ts[2], s_ts[3]))
                                : a.c.ctrl->min_ts;
    if (a.g.nd > 0 && !a.g.drag_exact && dtn >= tsmin) {
      atomicOr(&a.c.ctrl->status, FL_STIFF);
      // dt_next 0: the first step of the call (a.step); else the step after a.step
      atomicCAS(&a.c.ctrl->bad_step, -1, dt_next == 0 ? a.step : a.step + 1);
    }
  }
}

// ------------------------------------------------------------------------------------
// tables and initial state (device side of the initialisation)

struct EqPoint {
  double rho, P, v;
};

// Stationary flow (App. A): rho0 = rho_mid(r) exp[(GM/c^2)(1/s - 1/r)], P0 = c^2 rho0 with
// the isothermal c^2 = h0^2 GM r^beta_T, and the azimuthal velocity from the radial
// balance, v^2 = GM/r + c^2 (beta_T + beta_rho) + beta_T GM (1/r - 1/s) (the analytic
// pressure gradient folded in).
__device__ EqPoint eq_point(const rb_config& c, double r, double z) {
  EqPoint e;
  const double c2 = c.h0 * c.h0 * c.GM * pow(r, c.beta_T);
  const double s = sqrt(r * r + z * z);
  const double invs = 1.0 / s, invr = 1.0 / r;
  e.rho = c.rho_mid0 * pow(r, c.beta_rho) * exp(c.GM / c2 * (invs - invr));
  e.P = c2 * e.rho;
  e.v = sqrt(c.GM * invr + c2 * (c.beta_T + c.beta_rho) + c.beta_T * c.GM * (invr - invs));
  return e;
}

__device__ void gas_cons(double g, double rho, double u, double v, double P, double* q) {
  q[0] = rho * u;
  q[1] = rho * v;
  q[2] = 0.0;
  q[3] = P / (g - 1.0) + 0.5 * rho * (u * u + v * v);
  q[4] = rho;
}

// Primitive variables of a conservative gas state q as a WB_N table entry: velocity,
// pressure, density, sound speed, E + P, 1/rho.  Zero for the Sod annulus (its split has
// no stationary reference).
__device__ void prim_entry(const rb_config& c, const double* q, double* o) {
  if (c.init_kind != RB_INIT_DISC) {
    for (int s = 0; s < WB_N; ++s) o[s] = 0.0;
    return;
  }
  const double rho = q[4];
  o[WB_U] = q[0] / rho;
  o[WB_V] = q[1] / rho;
  o[WB_W] = q[2] / rho;
  o[WB_P] = (c.gamma - 1.0) * (q[3] - 0.5 * (q[0] * o[WB_U] + q[1] * o[WB_V] + q[2] * o[WB_W]));
  o[WB_RHO] = rho;
  o[WB_C] = sqrt(c.gamma * o[WB_P] / rho);
  o[WB_H] = q[3] + o[WB_P];
  o[WB_IRHO] = 1.0 / rho;
}

// Reconstructed variables of a ghost cell whose full state is q (nf fields): the gas
// deviation W(q) - W0 (zero on a disc, whose ghosts hold the stationary flow; the
// state's own primitives for the Sod annulus), and each dust fluid's velocity (zero
// where it is empty) and density.
__device__ void ghost_recon(const rb_config& c, int nf, const double* q, double* o) {
  if (c.init_kind == RB_INIT_DISC) {
    for (int f = 0; f < 5; ++f) o[f] = 0.0;
  } else {
    const double rho = q[4];
    const double u = q[0] / rho, v = q[1] / rho, w = q[2] / rho;
    o[0] = u; o[1] = v; o[2] = w;
    o[3] = (c.gamma - 1.0) * (q[3] - 0.5 * (q[0] * u + q[1] * v + q[2] * w));
    o[4] = rho;
  }
  for (int b = 5; b < nf; b += 4) {
    const double rd = q[b + 3];
    for (int m = 0; m < 3; ++m) o[b + m] = rd > 0.0 ? q[b + m] / rd : 0.0;
    o[b + 3] = rd;
  }
}

// initial dust layer of species s: eps (H/H_d) rho_mid(r) exp(-z^2 / 2 H_d^2)
__device__ double dust_layer(const rb_config& c, int s, double r, double z) {
  const double c2 = c.h0 * c.h0 * c.GM * pow(r, c.beta_T);
  const double H = sqrt(c2) / sqrt(c.GM / (r * r * r));
  const double Hd = c.hd_over_h[s] * H;
  return c.eps_dust[s] / c.hd_over_h[s] * c.rho_mid0 * pow(r, c.beta_rho) *
         exp(-(z * z) / (2.0 * Hd * Hd));
}

// full stationary state (gas + dust layer moving with the gas) at (r, z); Sod: the
// initial state at radius r
__device__ void background_full(const InitArgs& a, double r, double z, double* q) {
  const rb_config& c = a.cfg;
  if (c.init_kind == RB_INIT_SOD) {
    const double* s = r < c.sod_r0 ? c.sod_left : c.sod_right;
    gas_cons(c.gamma, s[0], s[2], 0.0, s[1], q);
    return;
  }
  EqPoint e = eq_point(c, r, z);
  gas_cons(c.gamma, e.rho, 0.0, e.v, e.P, q);
  for (int s = 0; s < c.n_dust; ++s) {
    double rd = dust_layer(c, s, r, z);
    q[5 + 4 * s + 0] = 0.0;
    q[5 + 4 * s + 1] = rd * e.v;
    q[5 + 4 * s + 2] = 0.0;
    q[5 + 4 * s + 3] = rd;
  }
}

__device__ __forceinline__ double face_r(const rb_config& c, int i) {
  if (c.log_r) return c.r_in * pow(c.r_out / c.r_in, (double)i / c.nr);
  return c.r_in + i * ((c.r_out - c.r_in) / c.nr);
}
__device__ __forceinline__ double cell_r(const rb_config& c, int i) {
  return 0.5 * (face_r(c, i) + face_r(c, i + 1));
}

// radial tables: one block
__global__ void __launch_bounds__(256) k_tables_r(InitArgs a) {
  const rb_config& c = a.cfg;
  const Layout& L = a.L;
  double* w = a.work;
  const int nr = c.nr;
  const bool twod = c.nz == 1;
  const double dth = 2.0 * M_PI / c.ntheta;
  const double dz = twod ? 1.0 : 2.0 * c.z_half / c.nz;
  for (int i = threadIdx.x; i < nr + 4; i += blockDim.x) w[L.rcell + i] = cell_r(c, i - 2);
  for (int i = threadIdx.x; i <= nr; i += blockDim.x) w[L.rface + i] = face_r(c, i);
  for (int k = threadIdx.x; k < c.nz; k += blockDim.x)
    w[L.zc + k] = twod ? 0.0 : (k + 0.5 - 0.5 * c.nz) * dz;
  for (int j = threadIdx.x; j < c.ntheta; j += blockDim.x) {
    const double th = (j + 0.5) * dth;
    w[L.trig + j] = cos(th);
    w[L.trig + c.ntheta + j] = sin(th);
  }
  for (int i = threadIdx.x; i <= nr; i += blockDim.x) w[L.ar + i] = face_r(c, i) * dth * dz;
  for (int i = threadIdx.x; i < nr; i += blockDim.x) {
    double rm = face_r(c, i), rp = face_r(c, i + 1);
    double* rt = w + L.rt + (size_t)i * RT_N;
    double area = 0.5 * (rp * rp - rm * rm);
    rt[RT_V] = area * dth * dz;
    rt[RT_INVV] = 1.0 / rt[RT_V];
    rt[RT_ATH] = (rp - rm) * dz;
    rt[RT_AZ] = area * dth;
    double rc = 0.5 * (rm + rp);
    rt[RT_RC] = rc;
    rt[RT_INVRC] = 1.0 / rc;
    rt[RT_OMK] = sqrt(c.GM / (rc * rc * rc));
    double amax = fmax(fmax(rm * dth * dz, rp * dth * dz), rt[RT_ATH]);
    if (!twod) amax = fmax(amax, rt[RT_AZ]);
    rt[RT_MAXA] = amax;
  }
  // parabola weights and limiter bounds along r for cells -1..nr (Sect. 2.7)
  for (int cI = threadIdx.x; cI < nr + 2; cI += blockDim.x) {
    int cc = cI - 1;
    double xm = cell_r(c, cc - 1), x0 = cell_r(c, cc), xp = cell_r(c, cc + 1);
    double hm = x0 - xm, hp = xp - x0, sum = hm + hp;
    double* co = w + L.rco + (size_t)cI * RC_N;
    double d = face_r(c, cc + 1) - x0;
    co[RC_WPP] = (d * d + hm * d) / (hp * sum);
    co[RC_WPM] = (hp * d - d * d) / (hm * sum);
    co[RC_LPM] = 2.0 * d / hm;
    co[RC_LPP] = 2.0 * d / hp;
    d = face_r(c, cc) - x0;
    co[RC_WMP] = (d * d + hm * d) / (hp * sum);
    co[RC_WMM] = (hp * d - d * d) / (hm * sum);
    co[RC_LMM] = 2.0 * d / hm;
    co[RC_LMP] = 2.0 * d / hp;
  }
  if (threadIdx.x == 0) {
    Ctrl* ct = reinterpret_cast<Ctrl*>(w + L.ctrl);
    double mts = 1e300;
    for (int s = 0; s < c.n_dust && c.drag_law == 0; ++s)
      for (int i = 0; i < nr; ++i) {
        double rc = cell_r(c, i);
        mts = fmin(mts, c.stokes[s] / sqrt(c.GM / (rc * rc * rc)));
      }
    ct->min_ts = mts;
  }
}

// 2D tables over (k, i) including two ghost layers in each direction
__global__ void __launch_bounds__(256) k_tables_2d(InitArgs a) {
  const rb_config& c = a.cfg;
  const Layout& L = a.L;
  double* w = a.work;
  const int nr = c.nr, nz = c.nz, nf = a.g.nf;
  const bool twod = nz == 1;
  const double dz = twod ? 1.0 : 2.0 * c.z_half / nz;
  const int W = nr + 4, H = nz + 4;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < W * H; t += gridDim.x * blockDim.x) {
    const int ii = t % W - 2, kk = t / W - 2;
    const double zc = twod ? 0.0 : (kk + 0.5 - 0.5 * nz) * dz;
    double q[MAXF];
    const bool kin = kk >= 0 && kk < nz, iin = ii >= 0 && ii < nr;
    if (kin && iin) {
      // indirect-gravity weight V r / (r^2 + z^2)^(3/2) of the cell
      const double rm = face_r(c, ii), rp = face_r(c, ii + 1), rc = cell_r(c, ii);
      const double V = 0.5 * (rp * rp - rm * rm) * (2.0 * M_PI / c.ntheta) * dz;
      const double s2 = rc * rc + zc * zc;
      w[L.indw + (size_t)kk * nr + ii] = V * rc / (s2 * sqrt(s2));
      // boundary damping zones: rate R / tau, R the squared fraction of the way from the
      // zone edge to the boundary, tau = damp_tau orbital periods
      double rate = 0.0;
      if (c.bc_r == 1) {
        const double e_in = c.damp_r_in * c.r_in, e_out = c.damp_r_out * c.r_out;
        if (rc < e_in) {
          const double x = (e_in - rc) / (e_in - c.r_in);
          rate += x * x * sqrt(c.GM / (c.r_in * c.r_in * c.r_in)) / (2.0 * M_PI * c.damp_tau);
        }
        if (rc > e_out) {
          const double x = (rc - e_out) / (c.r_out - e_out);
          rate += x * x * sqrt(c.GM / (c.r_out * c.r_out * c.r_out)) / (2.0 * M_PI * c.damp_tau);
        }
      }
      if (c.bc_z == 2 && !twod) {
        const double e_z = c.damp_z * c.z_half, az = fabs(zc);
        if (az > e_z) {
          const double x = (az - e_z) / (c.z_half - e_z);
          rate += x * x * sqrt(c.GM / (rc * rc * rc)) / (2.0 * M_PI * c.damp_tau);
        }
      }
      w[L.damp + (size_t)kk * nr + ii] = rate;
    }
    if (kin && iin) {
      const double r = cell_r(c, ii);
      background_full(a, r, zc, q);
      for (int f = 0; f < 5; ++f) w[L.bgc + ((size_t)kk * nr + ii) * 5 + f] =
          c.init_kind == RB_INIT_DISC ? q[f] : 0.0;
      prim_entry(c, q, w + L.wc + ((size_t)kk * nr + ii) * WB_N);
      double s3 = pow(r * r + zc * zc, 1.5);
      w[L.grav + ((size_t)kk * nr + ii) * 2 + 0] = -c.GM * r / s3;
      w[L.grav + ((size_t)kk * nr + ii) * 2 + 1] = -c.GM * zc / s3;
    }
    if (kin && ii >= 0 && ii <= nr) {
      background_full(a, face_r(c, ii), zc, q);
      for (int f = 0; f < 5; ++f) w[L.bgr + ((size_t)kk * (nr + 1) + ii) * 5 + f] =
          c.init_kind == RB_INIT_DISC ? q[f] : 0.0;
      prim_entry(c, q, w + L.wr + ((size_t)kk * (nr + 1) + ii) * WB_N);
    }
    if (!twod && iin && kk >= 0 && kk <= nz) {
      background_full(a, cell_r(c, ii), (kk - 0.5 * nz) * dz, q);
      for (int f = 0; f < 5; ++f) w[L.bgz + ((size_t)kk * nr + ii) * 5 + f] =
          c.init_kind == RB_INIT_DISC ? q[f] : 0.0;
      prim_entry(c, q, w + L.wz + ((size_t)kk * nr + ii) * WB_N);
    }
    // ghost cells: reconstructed variables (gas W', dust primitives) and the stationary
    // flow's primitives
    if (kin && !iin && ii >= -2 && ii <= nr + 1) {
      const int side = ii < 0 ? 0 : 1, layer = ii < 0 ? -1 - ii : ii - nr;
      background_full(a, cell_r(c, ii), zc, q);
      ghost_recon(c, nf, q, w + L.ghr + ((size_t)(side * 2 + layer) * nz + kk) * nf);
      prim_entry(c, q, w + L.ghrw + ((size_t)(side * 2 + layer) * nz + kk) * WB_N);
    }
    if (!twod && iin && !kin && kk >= -2 && kk <= nz + 1) {
      const int side = kk < 0 ? 0 : 1, layer = kk < 0 ? -1 - kk : kk - nz;
      background_full(a, cell_r(c, ii), zc, q);
      ghost_recon(c, nf, q, w + L.ghz + ((size_t)(side * 2 + layer) * nr + ii) * nf);
      prim_entry(c, q, w + L.ghzw + ((size_t)(side * 2 + layer) * nr + ii) * WB_N);
      // outflow ghosts: stationary density of the ghost over that of the boundary cell
      const double rho_g = q[4];
      background_full(a, cell_r(c, ii), (side == 0 ? 0.5 - 0.5 * nz : nz - 0.5 - 0.5 * nz) * dz, q);
      w[L.ozr + (size_t)(side * 2 + layer) * nr + ii] = rho_g / q[4];
    }
  }
}

// store of the initial state: FP64, or the FP32 layout (dust velocity components given
// directly through dust_vel, stored as deviations from the stationary flow's velocity)
__device__ __forceinline__ void store_init(const InitArgs& a, int f, int k, int i, size_t cl,
                                           double v, double dust_vel = 0.0) {
  const Geo& g = a.g;
  if (g.p32) {
    if (f < 5) { ((float*)a.state)[(size_t)f * g.N + cl] = (float)v; return; }
    const int sp = (f - 5) >> 2, c = (f - 5) & 3;
    if (c == 3) { ((double*)a.state)[p32_f64_base(g) + (size_t)sp * g.N + cl] = v; return; }
    const double u0 = c == 1 ? a.work[a.L.wc + ((size_t)k * g.nr + i) * WB_N + WB_V] : 0.0;
    ((float*)a.state)[(size_t)(5 + 3 * sp + c) * g.N + cl] = (float)(dust_vel - u0);
  } else {
    ((double*)a.state)[(size_t)f * g.N + cl] = v;
  }
}

// Initial state: Sod annulus, or the disc with the column Gaussian vortex (streamfunction
// psi = psi0 exp(-X^2/2 sr^2 - Y^2/2 sa^2), X = r - r_v, Y = r_v wrap(theta - theta_v),
// centre vorticity 2 Ro Omega_K(r_v) with Ro = -amplitude), density noise
// rho0 (1 + a xi) at unchanged pressure, the same on each dust layer from its own noise
// field, dust moving with the gas.  Stored as E' (gas) and whole variables (dust).
__global__ void __launch_bounds__(256) k_init_state(InitArgs a) {
  const rb_config& c = a.cfg;
  const Geo& g = a.g;
  const int nr = c.nr, nth = c.ntheta, nz = c.nz;
  const bool twod = nz == 1;
  const double dz = twod ? 1.0 : 2.0 * c.z_half / nz;
  const double dth = 2.0 * M_PI / nth;
  for (size_t cl = (size_t)blockIdx.x * blockDim.x + threadIdx.x; cl < g.N;
       cl += (size_t)gridDim.x * blockDim.x) {
    const int j = (int)(cl % nth);
    const int i = (int)((cl / nth) % nr);
    const int k = (int)(cl / ((size_t)nth * nr));
    const double r = cell_r(c, i);
    const double z = twod ? 0.0 : (k + 0.5 - 0.5 * nz) * dz;
    double q[MAXF];
    if (c.init_kind == RB_INIT_SOD) {
      background_full(a, r, z, q);
      for (int f = 0; f < 5; ++f) store_init(a, f, k, i, cl, q[f]);
      continue;
    }
    EqPoint e = eq_point(c, r, z);
    double q0[5];
    gas_cons(c.gamma, e.rho, 0.0, e.v, e.P, q0);
    const double A = a.amp ? a.amp[cl] : c.vortex_amp;
    const double rv = c.vortex_r0, sr = c.vortex_sig_r, sa = c.vortex_sig_a;
    const double X = r - rv;
    double d = (j + 0.5) * dth - c.vortex_th0;
    d -= 2.0 * M_PI * floor((d + M_PI) / (2.0 * M_PI));
    const double Y = rv * d;
    const double Om = sqrt(c.GM / (rv * rv * rv));
    const double psi = -2.0 * Om / (1.0 / (sr * sr) + 1.0 / (sa * sa)) *
                       exp(-X * X / (2.0 * sr * sr) - Y * Y / (2.0 * sa * sa));
    // Rossby-wave-instability seed (Sect. 4.3): density bump B at unchanged temperature,
    // rotation from the radial balance with the bump's pressure gradient
    // (v^2 = v0^2 + r c_iso^2 B'/B, c_iso^2 = P0/rho0), m-mode radial velocity
    double B = 1.0, vr = 0.0, vt = e.v;
    if (c.rwi_delta != 0.0 || c.rwi_eps != 0.0) {
      const double x = r - c.rwi_r0, w2 = c.rwi_dr * c.rwi_dr;
      const double gx = exp(-0.5 * x * x / w2);
      B = 1.0 + c.rwi_delta * gx;
      vt = sqrt(e.v * e.v - r * (e.P / e.rho) * (c.rwi_delta * gx * x / w2) / B);
      vr = c.rwi_eps * e.v * sin(c.rwi_m * ((j + 0.5) * dth)) * gx;
    }
    const double u = A * (-psi * rv * Y / (r * sa * sa)) + vr;
    const double v = vt + A * (psi * X / (sr * sr));
    const double xi = a.noise ? a.noise[cl] : 0.0;
    const double rho = e.rho * B * (1.0 + c.noise_amp * xi);
    gas_cons(c.gamma, rho, u, v, e.P * B, q);
    for (int f = 0; f < 5; ++f) store_init(a, f, k, i, cl, q[f] - q0[f]);
    for (int s = 0; s < c.n_dust; ++s) {
      const double xd = a.noise ? a.noise[(size_t)(1 + s) * g.N + cl] : 0.0;
      const double rd = dust_layer(c, s, r, z) * (1.0 + c.noise_amp * xd);
      const int o = 5 + 4 * s;
      store_init(a, o + 0, k, i, cl, rd * u, u);
      store_init(a, o + 1, k, i, cl, rd * v, v);
      store_init(a, o + 2, k, i, cl, 0.0, 0.0);
      store_init(a, o + 3, k, i, cl, rd);
    }
  }
}

// Derivative of the initial state with respect to the per-cell vortex amplitude A,
// contracted with a state cotangent lam: u = A u_hat, v = v0 + A v_hat, so
// d(rho u, rho v, 0, E, rho)/dA = (rho u_hat, rho v_hat, 0, rho (u u_hat + v v_hat), 0)
// and d(rho_d u, rho_d v, 0, rho_d)/dA = (rho_d u_hat, rho_d v_hat, 0, 0).
__global__ void __launch_bounds__(256) k_amp_grad(InitArgs a, const double* lam, double* out) {
  const rb_config& c = a.cfg;
  const Geo& g = a.g;
  const int nr = c.nr, nth = c.ntheta, nz = c.nz;
  const bool twod = nz == 1;
  const double dz = twod ? 1.0 : 2.0 * c.z_half / nz;
  const double dth = 2.0 * M_PI / nth;
  for (size_t cl = (size_t)blockIdx.x * blockDim.x + threadIdx.x; cl < g.N;
       cl += (size_t)gridDim.x * blockDim.x) {
    const int j = (int)(cl % nth);
    const int i = (int)((cl / nth) % nr);
    const int k = (int)(cl / ((size_t)nth * nr));
    const double r = cell_r(c, i);
    const double z = twod ? 0.0 : (k + 0.5 - 0.5 * nz) * dz;
    EqPoint e = eq_point(c, r, z);
    const double A = a.amp ? a.amp[cl] : c.vortex_amp;
    const double rv = c.vortex_r0, sr = c.vortex_sig_r, sa = c.vortex_sig_a;
    const double X = r - rv;
    double d = (j + 0.5) * dth - c.vortex_th0;
    d -= 2.0 * M_PI * floor((d + M_PI) / (2.0 * M_PI));
    const double Y = rv * d;
    const double Om = sqrt(c.GM / (rv * rv * rv));
    const double psi = -2.0 * Om / (1.0 / (sr * sr) + 1.0 / (sa * sa)) *
                       exp(-X * X / (2.0 * sr * sr) - Y * Y / (2.0 * sa * sa));
    const double uh = -psi * rv * Y / (r * sa * sa);
    const double vh = psi * X / (sr * sr);
    const double u = A * uh;
    const double v = e.v + A * vh;
    const double xi = a.noise ? a.noise[cl] : 0.0;
    const double rho = e.rho * (1.0 + c.noise_amp * xi);
    double acc = lam[0 * g.N + cl] * rho * uh + lam[1 * g.N + cl] * rho * vh +
                 lam[3 * g.N + cl] * rho * (u * uh + v * vh);
    for (int s = 0; s < c.n_dust; ++s) {
      const double xd = a.noise ? a.noise[(size_t)(1 + s) * g.N + cl] : 0.0;
      const double rd = dust_layer(c, s, r, z) * (1.0 + c.noise_amp * xd);
      const int o = 5 + 4 * s;
      acc += lam[(size_t)(o + 0) * g.N + cl] * rd * uh + lam[(size_t)(o + 1) * g.N + cl] * rd * vh;
    }
    out[cl] = acc;
  }
}

// ------------------------------------------------------------------------------------
// conversions and reductions

// a fresh control block (no flags, no bad cell), for calls whose control block is not
// the context's
__global__ void k_ctrl_init(Ctrl* c) {
  if (threadIdx.x == 0) {
    c->status = 0;
    c->bad_step = -1;
    c->maxit = 0;
    c->first_bad = ~0ull;
    c->nfall = 0;
    c->nvac = 0;
    c->nresolve = 0;
    for (int b = 0; b < 8; ++b) c->newton_hist[b] = 0;
    c->nnegd = 0;
    c->min_ts = 1e300;
  }
}

// the reduced CFL step to the caller's slot, or zero when the state had a cell with a
// non-positive density or pressure
__global__ void k_cfl_out(const Ctrl* c, const double* dt, double* out) {
  if (threadIdx.x == 0) out[0] = (c->status & FL_NEG) ? 0.0 : dt[0];
}

__global__ void k_fill(double* p, size_t n, double v) {
  for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
       q += (size_t)gridDim.x * blockDim.x)
    p[q] = v;
}

// field f of the state -> full FP64 values (gas: E0 + E'; dust: momenta, densities)
template <bool P32>
__global__ void k_to_full(StageArgs a, const void* state, double* out, int f) {
  const Geo& g = a.g;
  for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < g.N;
       c += (size_t)gridDim.x * blockDim.x) {
    const size_t ki = c / g.nth;
    double v = ld_cell<P32>(a, state, f, (int)(ki / g.nr), (int)(ki % g.nr), c);
    if (f < 5) v += a.t.bgc[ki * 5 + f];
    out[c] = v;
  }
}
template <bool P32>
__global__ void k_from_full(StageArgs a, const double* in, void* state, int f) {
  const Geo& g = a.g;
  for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < g.N;
       c += (size_t)gridDim.x * blockDim.x) {
    const size_t ki = c / g.nth;
    double v = in[c];
    if (f < 5) v -= a.t.bgc[ki * 5 + f];
    st_cell<P32>(a, state, f, (int)(ki / g.nr), (int)(ki % g.nr), c, v);
  }
}

// mass of field f (density slot): per-block partial sums of rho V over fixed chunks,
// each summed by a fixed tree (deterministic, FP64)
template <bool P32>
__global__ void __launch_bounds__(256) k_mass(StageArgs a, const void* state, double* part, int f) {
  __shared__ double s_s[4];
  const Geo& g = a.g;
  const size_t chunk = (g.N + gridDim.x - 1) / gridDim.x;
  const size_t c0 = (size_t)blockIdx.x * chunk, c1 = min(g.N, c0 + chunk);
  double acc = 0.0;
  for (size_t c = c0 + threadIdx.x; c < c1; c += blockDim.x) {
    const size_t ki = c / g.nth;
    const int i = (int)(ki % g.nr);
    double v = ld_cell<P32>(a, state, f, (int)(ki / g.nr), i, c);
    if (f < 5) v += a.t.bgc[ki * 5 + f];
    acc += v * a.t.rt[(size_t)i * RT_N + RT_V];
  }
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) s_s[threadIdx.x / 64] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (s_s[0] + s_s[1]) + (s_s[2] + s_s[3]);
}

// Indirect-gravity sums A = sum m w cos(theta), B = sum m w sin(theta) over the cells,
// m = gas + dust density, w = V r / (r^2 + z^2)^(3/2): per-block partials over fixed
// chunks, then one block adds them in a fixed order (deterministic, FP64).
template <bool P32>
__global__ void __launch_bounds__(256) k_indirect(StageArgs a, const void* state, double* part) {
  __shared__ double s_s[2][4];
  const Geo& g = a.g;
  const size_t chunk = (g.N + gridDim.x - 1) / gridDim.x;
  const size_t c0 = (size_t)blockIdx.x * chunk, c1 = min(g.N, c0 + chunk);
  double sa = 0.0, sb = 0.0;
  for (size_t c = c0 + threadIdx.x; c < c1; c += blockDim.x) {
    const size_t ki = c / g.nth;
    const int j = (int)(c % g.nth), i = (int)(ki % g.nr), k = (int)(ki / g.nr);
    double m = a.t.bgc[ki * 5 + 4] + ld_cell<P32>(a, state, 4, k, i, c);
    for (int s = 0; s < g.nd; ++s) m += ld_cell<P32>(a, state, 5 + 4 * s + 3, k, i, c);
    const double mw = m * a.t.indw[ki];
    sa += mw * a.t.trig[j];
    sb += mw * a.t.trig[g.nth + j];
  }
  sa = wave_sum(sa);
  sb = wave_sum(sb);
  if ((threadIdx.x & 63) == 0) { s_s[0][threadIdx.x / 64] = sa; s_s[1][threadIdx.x / 64] = sb; }
  __syncthreads();
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = (s_s[0][0] + s_s[0][1]) + (s_s[0][2] + s_s[0][3]);
    part[2 * blockIdx.x + 1] = (s_s[1][0] + s_s[1][1]) + (s_s[1][2] + s_s[1][3]);
  }
}

__global__ void __launch_bounds__(256) k_indirect_final(const double* part, int n, double* ab) {
  __shared__ double s_s[2][4];
  double sa = 0.0, sb = 0.0;
  for (int b = threadIdx.x; b < n; b += blockDim.x) { sa += part[2 * b]; sb += part[2 * b + 1]; }
  sa = wave_sum(sa);
  sb = wave_sum(sb);
  if ((threadIdx.x & 63) == 0) { s_s[0][threadIdx.x / 64] = sa; s_s[1][threadIdx.x / 64] = sb; }
  __syncthreads();
  if (threadIdx.x == 0) {
    ab[0] = (s_s[0][0] + s_s[0][1]) + (s_s[0][2] + s_s[0][3]);
    ab[1] = (s_s[1][0] + s_s[1][1]) + (s_s[1][2] + s_s[1][3]);
  }
}

__global__ void __launch_bounds__(256) k_sum(const double* part, int n, double* out) {
  __shared__ double s_s[4];
  double acc = 0.0;
  for (int b = threadIdx.x; b < n; b += blockDim.x) acc += part[b];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) s_s[threadIdx.x / 64] = acc;
  __syncthreads();
  if (threadIdx.x == 0) *out = (s_s[0] + s_s[1]) + (s_s[2] + s_s[3]);
}

// ------------------------------------------------------------------------------------
// launchers

hipError_t launch_tables(const InitArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_tables_r, dim3(1), dim3(256), 0, s, a);
  const int cells = (a.cfg.nr + 4) * (a.cfg.nz + 4);
  const int blocks = (cells + 255) / 256;
  hipLaunchKernelGGL(k_tables_2d, dim3(blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_init_state(const InitArgs& a, hipStream_t s) {
  const int blocks = (int)std::min<size_t>((a.g.N + 255) / 256, 65536);
  hipLaunchKernelGGL(k_init_state, dim3(blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

template <int ND, bool P32, bool EXT>
static void group_nd3(const StageArgs& a, int blocks, int group, hipStream_t s) {
  if (group == 0) {
    if (a.g.gamma == 1.4)
      hipLaunchKernelGGL((k_march<true, ND, true, P32, EXT>), dim3(blocks), dim3(NTM), 0, s, a, 0);
    else
      hipLaunchKernelGGL((k_march<true, ND, false, P32, EXT>), dim3(blocks), dim3(NTM), 0, s, a, 0);
  } else {
    hipLaunchKernelGGL((k_march<false, ND, true, P32, EXT>), dim3(blocks), dim3(NTM), 0, s, a,
                       group - 1);
  }
}

// the optional physics (indirect gravity, drag law 1) and boundary options (damping zones,
// outflow ghosts) run in their own instantiation; the base one compiles them out
static bool uses_ext(const Geo& g) { return g.indirect || g.damp || g.bc_z == 1 || g.drag_law; }

template <int ND, bool P32>
static void group_nd2(const StageArgs& a, int blocks, int group, hipStream_t s) {
  if (uses_ext(a.g)) group_nd3<ND, P32, true>(a, blocks, group, s);
  else group_nd3<ND, P32, false>(a, blocks, group, s);
}

template <int ND>
static void group_nd(const StageArgs& a, int blocks, int group, hipStream_t s) {
  if (a.g.p32) group_nd2<ND, true>(a, blocks, group, s);
  else group_nd2<ND, false>(a, blocks, group, s);
}

hipError_t launch_stage_group(const StageArgs& a, int blocks, int group, hipStream_t s) {
  switch (a.g.nd) {
    case 0: group_nd<0>(a, blocks, group, s); break;
    case 1: group_nd<1>(a, blocks, group, s); break;
    case 2: group_nd<2>(a, blocks, group, s); break;
    case 3: group_nd<3>(a, blocks, group, s); break;
    case 4: group_nd<4>(a, blocks, group, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_stage(const StageArgs& a, int blocks, hipStream_t s) {
  hipError_t e = launch_stage_group(a, blocks, 0, s);
  if (e != hipSuccess || a.gas_only) return e;
  for (int sp = 0; sp < a.g.nd; ++sp) {
    e = launch_stage_group(a, blocks, 1 + sp, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int ND>
static void cfl_nd(const StageArgs& a, const void* state, int blocks, hipStream_t s) {
  if (a.g.p32) hipLaunchKernelGGL((k_cfl<ND, true>), dim3(blocks), dim3(256), 0, s, a, state);
  else hipLaunchKernelGGL((k_cfl<ND, false>), dim3(blocks), dim3(256), 0, s, a, state);
}

hipError_t launch_cfl(const StageArgs& a, const void* state, int blocks, int dt_idx,
                      hipStream_t s) {
  (void)dt_idx;
  switch (a.g.nd) {
    case 0: cfl_nd<0>(a, state, blocks, s); break;
    case 1: cfl_nd<1>(a, state, blocks, s); break;
    case 2: cfl_nd<2>(a, state, blocks, s); break;
    case 3: cfl_nd<3>(a, state, blocks, s); break;
    case 4: cfl_nd<4>(a, state, blocks, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int ND>
static void drag_nd(const StageArgs& a, void* state, double frac, int blocks, hipStream_t s) {
  if (a.g.p32) hipLaunchKernelGGL((k_drag<ND, true>), dim3(blocks), dim3(256), 0, s, a, state, frac);
  else hipLaunchKernelGGL((k_drag<ND, false>), dim3(blocks), dim3(256), 0, s, a, state, frac);
}

hipError_t launch_drag(const StageArgs& a, void* state, double frac, int blocks, hipStream_t s) {
  switch (a.g.nd) {
    case 1: drag_nd<1>(a, state, frac, blocks, s); break;
    case 2: drag_nd<2>(a, state, frac, blocks, s); break;
    case 3: drag_nd<3>(a, state, frac, blocks, s); break;
    case 4: drag_nd<4>(a, state, frac, blocks, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_reduce(const StageArgs& a, int nparts, int dt_idx_next, int want_dt,
                         int want_ledger, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(256), 0, s, a, nparts, dt_idx_next, want_dt,
                     want_ledger);
  return hipGetLastError();
}

hipError_t launch_ctrl_init(Ctrl* c, hipStream_t s) {
  hipLaunchKernelGGL(k_ctrl_init, dim3(1), dim3(64), 0, s, c);
  return hipGetLastError();
}

hipError_t launch_cfl_out(const Ctrl* c, const double* dt, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_cfl_out, dim3(1), dim3(64), 0, s, c, dt, out);
  return hipGetLastError();
}

hipError_t launch_fill(double* p, size_t n, double v, hipStream_t s) {
  const int blocks = (int)std::min<size_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(k_fill, dim3(std::max(blocks, 1)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_to_full(const StageArgs& a, const void* state, double* out, int f,
                          hipStream_t s) {
  const int blocks = (int)std::min<size_t>((a.g.N + 255) / 256, 65536);
  if (a.g.p32) hipLaunchKernelGGL(k_to_full<true>, dim3(blocks), dim3(256), 0, s, a, state, out, f);
  else hipLaunchKernelGGL(k_to_full<false>, dim3(blocks), dim3(256), 0, s, a, state, out, f);
  return hipGetLastError();
}

hipError_t launch_from_full(const StageArgs& a, const double* in, void* state, int f,
                            hipStream_t s) {
  const int blocks = (int)std::min<size_t>((a.g.N + 255) / 256, 65536);
  if (a.g.p32) hipLaunchKernelGGL(k_from_full<true>, dim3(blocks), dim3(256), 0, s, a, in, state, f);
  else hipLaunchKernelGGL(k_from_full<false>, dim3(blocks), dim3(256), 0, s, a, in, state, f);
  return hipGetLastError();
}

hipError_t launch_mass(const StageArgs& a, const void* state, double* partials, int f,
                       int blocks, hipStream_t s) {
  if (a.g.p32) hipLaunchKernelGGL(k_mass<true>, dim3(blocks), dim3(256), 0, s, a, state, partials, f);
  else hipLaunchKernelGGL(k_mass<false>, dim3(blocks), dim3(256), 0, s, a, state, partials, f);
  return hipGetLastError();
}

hipError_t launch_amp_grad(const InitArgs& a, const double* lam, double* out, hipStream_t s) {
  const int blocks = (int)std::min<size_t>((a.g.N + 255) / 256, 65536);
  hipLaunchKernelGGL(k_amp_grad, dim3(blocks), dim3(256), 0, s, a, lam, out);
  return hipGetLastError();
}

hipError_t launch_indirect(const StageArgs& a, const void* state, double* partials, int blocks,
                           double* ab, hipStream_t s) {
  if (a.g.p32) hipLaunchKernelGGL(k_indirect<true>, dim3(blocks), dim3(256), 0, s, a, state, partials);
  else hipLaunchKernelGGL(k_indirect<false>, dim3(blocks), dim3(256), 0, s, a, state, partials);
  hipLaunchKernelGGL(k_indirect_final, dim3(1), dim3(256), 0, s, partials, blocks, ab);
  return hipGetLastError();
}

hipError_t launch_sum(const double* partials, int n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, s, partials, n, out);
  return hipGetLastError();
}

}  // namespace rb
