// Fused 2D time step: one launch advances every active population set by
// one step (pull streaming, moments, isotropic stencils, anisotropy,
// forces, MRT collisions in closed form, time-stretched AAC store, history).
//
// Work decomposition: a workgroup owns a tile of nodes (StepTile: 32 x 8 with
// two halo rings, 32 x 4 with one), one node per thread.  Moments of the tile plus a halo of R rings
// (R = 2 when the flow and bubble phase are both active, else 1) are staged
// in LDS; the flow phase then evaluates D_phi (x) v0 on the tile plus one
// ring (LDS), and each thread finishes its own node from registers and LDS.
// Populations live in SoA planes (x fastest), post-collision at their source
// node, so a node pulls f_i(x) from x - c_i; a population that would cross a
// wall is read back from the node's own opposite slot (half-way bounce-back).
// FP32 and 16-bit planes hold deviations f_i - w_i m_ref from the bulk-liquid
// rest state and the collisions are written in those deviations, so that the
// bulk, where f_i is close to w_i m_ref, rounds small numbers; FP64 planes
// hold full populations.
//
// Tiles whose pulls stay inside the domain take a fast path: every load and
// store is a scalar base plus a 32-bit byte offset, one integer add per
// access.  Tiles on the domain edge use the general wrap/bounce addressing.
// A far-field side is a wall for NS and phi; the populations of psi, C and
// theta that leave across it are stored by anti-bounce-back, -f*_i +
// 2 w_i value, so the pull reads them back as from a wall; the stencil
// ghosts of psi and U there are odd about psi_l and U = 0.
#pragma once
#include "pfl_kernels.h"
#include "pfl_step2d.h"

namespace pfl {

template <int FIELDS, int QP, class ST, class HT, class CT, bool SYM, bool STREAM>
__global__ __launch_bounds__((StepTile<FIELDS, ST>::N))
__attribute__((amdgpu_waves_per_eu(StepTile<FIELDS, ST>::template waves<CT, SYM>())))
void step2d_kernel(const DevParams P,
                                                    const typename Store<ST>::raw* __restrict__ fin,
                                                    typename Store<ST>::raw* __restrict__ fout,
                                                    HT* hist, double* __restrict__ mout,
                                                    int mode) {
  constexpr bool NS = FIELDS & F_NS, PHI = FIELDS & F_PHI, PSI = FIELDS & F_PSI;
  constexpr bool CC = FIELDS & F_C, TH = FIELDS & F_TH;
  constexpr bool FLOWX = NS && PHI;          // mass-flux force needs D_phi (x) v0 on ring 1
  constexpr int R = FLOWX ? 2 : 1;
  constexpr int STX = StepTile<FIELDS, ST>::X, STY = StepTile<FIELDS, ST>::Y, SNT = StepTile<FIELDS, ST>::N;
  constexpr int RX = STX + 2 * R, RY = STY + 2 * R;
  constexpr int QN = 9, QS = 5;
  using LN = Lat<9>;
  using LS = Lat<5>;
  using LP = Lat<QP>;
  using raw = typename Store<ST>::raw;
  constexpr uint32_t S = sizeof(raw), HS = sizeof(HT);
  const KP<CT>& K = kp<CT>(P);

  __shared__ CT s_phi[RY][RX];
  __shared__ CT s_psi[RY][RX];
  __shared__ CT s_U[RY][RX];
  // psi populations of the tile and ring 1: the time-stretched store needs
  // f_i(x + c_i) at the start of the step
  __shared__ CT s_fps[PSI ? QS : 1][PSI ? RY : 1][PSI ? RX : 1];
  __shared__ CT s_jx[NS ? RY : 1][NS ? RX : 1];
  __shared__ CT s_jy[NS ? RY : 1][NS ? RX : 1];
  __shared__ CT s_X[FLOWX ? 4 : 1][FLOWX ? RY : 1][FLOWX ? RX : 1];

  const int tid = threadIdx.x;
  const int lx = tid % STX, ly = tid / STX;
  const int gtx = (P.nx + STX - 1) / STX;
  const int lt = logical_tile(blockIdx.x, gtx * ((P.ny + STY - 1) / STY));
  const int tile_x = lt % gtx, tile_y = lt / gtx;
  const int bx0 = tile_x * STX, by0 = tile_y * STY;
  const int x = bx0 + lx, y = by0 + ly;
  const bool own = (x < P.nx) && (y < P.ny);
  const long long N = P.N;
  const long long idx = (long long)y * P.nx + x;
  // every pull of the tile and its halo stays inside the domain
  const bool fast = P.fast && bx0 >= R + 1 && by0 >= R + 1 && bx0 + STX + R + 1 <= P.nx &&
                    by0 + STY + R + 1 <= P.ny;

  const raw* fin_ns = fin + (long long)(NS ? P.o_ns : 0) * N;
  const raw* fin_phi = fin + (long long)(PHI ? P.o_phi : 0) * N;
  const raw* fin_psi = fin + (long long)(PSI ? P.o_psi : 0) * N;
  const raw* fin_c = fin + (long long)(CC ? P.o_c : 0) * N;
  const raw* fin_th = fin + (long long)(TH ? P.o_th : 0) * N;

  const CT k1 = K.k1;

  // ---- phase A1: own node populations and moments
  CT fns[NS ? QN : 1], fph[PHI ? QP : 1], fps[PSI ? QS : 1], fc[CC ? QS : 1], fth[TH ? QS : 1];
  // Moments are rest value + sum of stored values: phi = r_phi + dphi, ...
  // Deviation storage (FP32, FP16, BF16) has r = (1, -1, C_ref, theta0);
  // FP64 storage holds full populations, r = 0, and keeps the plain
  // equilibrium forms below so its rounding follows the definitions.
  constexpr bool DEV = !std::is_same<ST, double>::value;
  const CT r_phi = DEV ? CT(1) : CT(0), r_psi = DEV ? CT(-1) : CT(0);
  const CT r_C = DEV ? K.C_ref : CT(0), r_H = DEV ? K.theta0 : CT(0);
  CT phi = CT(1), psi = CT(-1), C = CT(0), H = CT(0), U = K.U0, jx = CT(0), jy = CT(0);
  CT dphi = CT(0), dpsi = CT(0), dC = CT(0), dH = CT(0);
  // history and grain id of the own node, loaded early so that their latency
  // overlaps with the pulls
  const bool first = P.first != 0;
  const uint32_t hbyte = (uint32_t)idx * HS;
  const uint32_t hplane = (uint32_t)N * HS;
  const HT* hsrc = P.hist_src ? (const HT*)P.hist_src : hist;
  auto hld = [&](int plane) -> CT {
    if (P.fast) return CT(*(const HT*)((const char*)hsrc + (uint32_t)plane * hplane + hbyte));
    return CT(hsrc[(long long)plane * N + idx]);
  };
  CT h_psi = CT(0), h_S = CT(0), h_pv0 = CT(0), h_pv1 = CT(0), h_B0 = CT(0), h_B1 = CT(0);
  CT h_Hv0 = CT(0), h_Hv1 = CT(0);
  int gid = 0;
  if (own) {
    if (PSI) gid = P.grain[idx];
    if (!first && mode == 0) {
      if constexpr (PSI) { h_psi = hld(P.h_psi); h_S = hld(P.h_S); }
      if constexpr (PHI) { h_pv0 = hld(P.h_phiv); h_pv1 = hld(P.h_phiv + 1); }
      if constexpr (CC) { h_B0 = hld(P.h_B); h_B1 = hld(P.h_B + 1); }
      if constexpr (TH) { h_Hv0 = hld(P.h_Hv); h_Hv1 = hld(P.h_Hv + 1); }
    }
  }
  if (own) {
    if constexpr (NS) {
      pull<QN, ST, CT, SYM>(fast, fin_ns, P, x, y, fns);
#pragma unroll
      for (int i = 0; i < QN; ++i) { jx += CT(LN::c[i][0]) * fns[i]; jy += CT(LN::c[i][1]) * fns[i]; }
    }
    if constexpr (PHI) {
      pull<QP, ST, CT, SYM>(fast, fin_phi, P, x, y, fph);
#pragma unroll
      for (int i = 0; i < QP; ++i) dphi += fph[i];
      phi = r_phi + dphi;
    }
    if constexpr (PSI) {
      pull<QS, ST, CT, SYM>(fast, fin_psi, P, x, y, fps);
#pragma unroll
      for (int i = 0; i < QS; ++i) { dpsi += fps[i]; s_fps[i][ly + R][lx + R] = fps[i]; }
      psi = r_psi + dpsi;
    }
    if constexpr (CC) {
      pull<QS, ST, CT, SYM>(fast, fin_c, P, x, y, fc);
#pragma unroll
      for (int i = 0; i < QS; ++i) dC += fc[i];
      C = r_C + dC;
      const CT h = (psi + CT(1)) * CT(0.5);
      U = (C * rcp(CT(1) - k1 * h) - CT(1)) * K.inv_k1;
    }
    if constexpr (TH) {
      pull<QS, ST, CT, SYM>(fast, fin_th, P, x, y, fth);
#pragma unroll
      for (int i = 0; i < QS; ++i) dH += fth[i];
      H = r_H + dH;
    }
    s_phi[ly + R][lx + R] = phi;
    s_psi[ly + R][lx + R] = psi;
    s_U[ly + R][lx + R] = U;
    if constexpr (NS) { s_jx[ly + R][lx + R] = jx; s_jy[ly + R][lx + R] = jy; }
  }

  // ---- phase A2: halo (and, on edge tiles, tile positions past the domain)
  auto halo_node = [&](int rx, int ry, int gx, int gy, bool hfast) {
    const bool ring1 = rx >= R - 1 && rx <= RX - R && ry >= R - 1 && ry <= RY - R;
    CT hphi = CT(1), hpsi = CT(-1), hU = K.U0, hjx = CT(0), hjy = CT(0);
    if constexpr (PHI) {
      CT f[QP];
      pull<QP, ST, CT, SYM>(hfast, fin_phi, P, gx, gy, f);
      CT d = CT(0);
#pragma unroll
      for (int i = 0; i < QP; ++i) d += f[i];
      hphi = r_phi + d;
    }
    if (ring1) {
      if constexpr (PSI) {
        CT f[QS];
        pull<QS, ST, CT, SYM>(hfast, fin_psi, P, gx, gy, f);
        CT d = CT(0);
#pragma unroll
        for (int i = 0; i < QS; ++i) { d += f[i]; s_fps[i][ry][rx] = f[i]; }
        hpsi = r_psi + d;
      }
      if constexpr (CC) {
        CT f[QS];
        pull<QS, ST, CT, SYM>(hfast, fin_c, P, gx, gy, f);
        CT d = CT(0);
#pragma unroll
        for (int i = 0; i < QS; ++i) d += f[i];
        const CT hC = r_C + d;
        const CT h = (hpsi + CT(1)) * CT(0.5);
        hU = (hC * rcp(CT(1) - k1 * h) - CT(1)) * K.inv_k1;
      }
      if constexpr (NS) {
        CT f[QN];
        pull<QN, ST, CT, SYM>(hfast, fin_ns, P, gx, gy, f);
#pragma unroll
        for (int i = 0; i < QN; ++i) { hjx += CT(LN::c[i][0]) * f[i]; hjy += CT(LN::c[i][1]) * f[i]; }
      }
    }
    s_phi[ry][rx] = hphi;
    s_psi[ry][rx] = hpsi;
    s_U[ry][rx] = hU;
    if constexpr (NS) { s_jx[ry][rx] = hjx; s_jy[ry][rx] = hjy; }
  };
  if (fast) {
    constexpr int NH = RX * RY - STX * STY;
    for (int k = tid; k < NH; k += SNT) {
      int rx, ry;
      halo_pos<R, STX, STY>(k, rx, ry);
      halo_node(rx, ry, bx0 + rx - R, by0 + ry - R, true);
    }
  } else {
    for (int k = tid; k < RX * RY; k += SNT) {
      const int rx = k % RX, ry = k / RX;
      const int tx = rx - R, ty = ry - R;
      const int gx0 = bx0 + tx, gy0 = by0 + ty;
      const bool inner = tx >= 0 && tx < STX && ty >= 0 && ty < STY;
      if (inner && gx0 < P.nx && gy0 < P.ny) continue;   // filled in A1
      halo_node(rx, ry, map_coord(gx0, P.nx, P.wall[0]), map_coord(gy0, P.ny, P.wall[1]), false);
      if (SYM && P.far) {
        // ghost across an odd number of far-field sides: psi and U odd about
        // psi_l = -1 and U = 0 (each crossing mirrors once)
        const bool fx = gx0 < 0 ? far_side(P, 0, true) : gx0 >= P.nx && far_side(P, 0, false);
        const bool fy = gy0 < 0 ? far_side(P, 1, true) : gy0 >= P.ny && far_side(P, 1, false);
        if (fx != fy) {
          s_psi[ry][rx] = CT(-2) - s_psi[ry][rx];
          s_U[ry][rx] = -s_U[ry][rx];
        }
      }
    }
  }
  __syncthreads();

  // ---- phase B: D_phi (x) v0 on the tile and ring 1 (mass-flux force)
  FlowNode<CT> fo;
  if constexpr (FLOWX) {
    if (own) {
      flow_node<NS, PHI, CT, RX>(K, s_phi, s_psi, s_jx, s_jy, ly + R, lx + R, fo);
      s_X[0][ly + R][lx + R] = fo.Dx * fo.v0x;
      s_X[1][ly + R][lx + R] = fo.Dx * fo.v0y;
      s_X[2][ly + R][lx + R] = fo.Dy * fo.v0x;
      s_X[3][ly + R][lx + R] = fo.Dy * fo.v0y;
    }
    constexpr int AX = STX + 2, AY = STY + 2;
    for (int k = tid; k < AX * AY; k += SNT) {
      const int rx = k % AX + R - 1, ry = k / AX + R - 1;
      const int tx = rx - R, ty = ry - R;
      const int gx0 = bx0 + tx, gy0 = by0 + ty;
      const bool inner = tx >= 0 && tx < STX && ty >= 0 && ty < STY;
      if (inner && gx0 < P.nx && gy0 < P.ny) continue;
      // ghosts across a wall take minus the value at their mirror node;
      // across a symmetry plane the mirror image: the off-diagonal
      // components (one index along the normal) change sign
      int mx = rx, my = ry;
      CT sgn = CT(1), sod = CT(1);
      bool skip = false;
      if (P.wall[0] && (gx0 < 0 || gx0 >= P.nx)) {
        if (gx0 == -1) mx = rx + 1; else if (gx0 == P.nx) mx = rx - 1; else skip = true;
        if (SYM && sym_side(P, 0, gx0 < 0)) sod = -sod; else sgn = -sgn;
      }
      if (P.wall[1] && (gy0 < 0 || gy0 >= P.ny)) {
        if (gy0 == -1) my = ry + 1; else if (gy0 == P.ny) my = ry - 1; else skip = true;
        if (SYM && sym_side(P, 1, gy0 < 0)) sod = -sod; else sgn = -sgn;
      }
      CT X0 = CT(0), X1 = CT(0), X2 = CT(0), X3 = CT(0);
      if (!skip) {
        FlowNode<CT> h;
        flow_node<NS, PHI, CT, RX>(K, s_phi, s_psi, s_jx, s_jy, my, mx, h);
        X0 = sgn * h.Dx * h.v0x; X1 = sgn * sod * h.Dx * h.v0y;
        X2 = sgn * sod * h.Dy * h.v0x; X3 = sgn * h.Dy * h.v0y;
      }
      s_X[0][ry][rx] = X0; s_X[1][ry][rx] = X1; s_X[2][ry][rx] = X2; s_X[3][ry][rx] = X3;
    }
    __syncthreads();
  } else {
    if (own) flow_node<NS, PHI, CT, RX>(K, s_phi, s_psi, s_jx, s_jy, ly + R, lx + R, fo);
  }
  if (!own) return;

  // ---- phase C: the rest of the step at the own node
  const int ry = ly + R, rx = lx + R;
  // direction i of the 5-velocity sets leaves across a far-field side
  auto far_out = [&](int i) -> bool {
    if constexpr (!SYM) return false;
    if (fast || !P.far) return false;
    const int dx = LS::c[i][0], dy = LS::c[i][1];
    return (dx > 0 && x == P.nx - 1 && far_side(P, 0, false)) || (dx < 0 && x == 0 && far_side(P, 0, true)) ||
           (dy > 0 && y == P.ny - 1 && far_side(P, 1, false)) || (dy < 0 && y == 0 && far_side(P, 1, true));
  };
  const CT h = (psi + CT(1)) * CT(0.5);
  const CT q = clamp01((CT(1) - psi) * CT(0.5));
  // temperature: H = c_p theta - c_p^s h with sum g = rho H; rho, c_p, k_T
  // linear in phi between gas and liquid (liquid = solid = 1).  dtheta =
  // theta - r_H, the deviation of the non-rest equilibria; s_th the heat
  // relaxation rate from k_T.
  CT theta = K.theta0, dtheta = CT(0), s_th = K.s_th;
  if constexpr (TH) {
    if (K.varheat) {
      const CT rh = K.th_rho_g + (CT(1) - K.th_rho_g) * phi;
      const CT cp = K.th_cp_g + (CT(1) - K.th_cp_g) * phi;
      const CT kh = K.th_k_g + (CT(1) - K.th_k_g) * phi;
      const CT rc = rh * cp;
      dtheta = (dH + rh * h + r_H * (CT(1) - rc)) / rc;
      theta = r_H + dtheta;
      s_th = rcp(K.alpha_cs * kh + CT(0.5));
    } else {
      theta = H + h;
      dtheta = dH + h;
    }
  }

  // gradients of psi and U
  CT gpx = CT(0), gpy = CT(0), gUx = CT(0), gUy = CT(0);
  if constexpr (PSI) grad9<CT, RX>(s_psi, ry, rx, gpx, gpy);
  if constexpr (CC) grad9<CT, RX>(s_U, ry, rx, gUx, gUy);
  // unit normal and cubic anisotropy in the crystal frame of the nearest
  // seed: a_s = 1 + eps (4 S4 - 3 G^2) / (G + delta)^2, N' = G a_s d a_s/d g'
  const CT dn = K.dn;
  const CT invp = rsq(gpx * gpx + gpy * gpy + dn);
  const CT ex = gpx * invp, ey = gpy * invp;
  CT a_s, Nx, Ny;
  {
    const CT cth = CT(P.grain_cs[2 * gid]), sth = CT(P.grain_cs[2 * gid + 1]);
    const CT rx_ = cth * gpx + sth * gpy;
    const CT ry_ = -sth * gpx + cth * gpy;
    const CT rx2 = rx_ * rx_, ry2 = ry_ * ry_;
    const CT G = rx2 + ry2;
    const CT S4 = rx2 * rx2 + ry2 * ry2;
    const CT invGd = rcp(G + dn);
    const CT inv2 = invGd * invGd;
    const CT eps = K.eps4;
    a_s = CT(1) + eps * (CT(4) * S4 - CT(3) * G * G) * inv2;
    const CT pre = CT(4) * eps * G * a_s * inv2 * invGd;
    const CT Nrx = pre * rx_ * (CT(4) * rx2 * G + (CT(4) * rx2 - CT(3) * G) * dn - CT(4) * S4);
    const CT Nry = pre * ry_ * (CT(4) * ry2 * G + (CT(4) * ry2 - CT(3) * G) * dn - CT(4) * S4);
    Nx = cth * Nrx - sth * Nry;
    Ny = sth * Nrx + cth * Nry;
  }
  const CT as2 = a_s * a_s;

  // kinetics F(U)
  const CT lin = CT(1) + k1 * U;
  const CT F = K.inv_Le + K.Mcinf * (lin > CT(0) ? lin : CT(0));
  const CT gFx = lin > CT(0) ? K.Mcinf * k1 * gUx : CT(0);
  const CT gFy = lin > CT(0) ? K.Mcinf * k1 * gUy : CT(0);

  // psi source
  const CT om = CT(1) - phi;
  const CT ps1 = psi + CT(1);
  const CT f2p = CT(0.5) * (CT(1) - psi) * ps1 * (CT(-2) * psi);
  const CT f3psi = CT(2) * K.beta_inter * om * om * ps1;
  const CT s1m = (CT(1) - psi) * ps1;
  const CT pprime = CT(30.0 / 32.0) * s1m * s1m;
  const CT Qpsi = -(f2p + f3psi + K.lam * pprime * (theta + K.Mcinf * U));
  // rewritten form: a_n = a_s^2, F(U) in D_psi and S_psi with the grad F
  // term; form for Le = O(1): a_n = a_s^2 F(U) (Appendix B)
  CT S_psi, D_psi;
  if (P.le1) {
    S_psi = Qpsi * K.inv_tau0;
    D_psi = K.d_psi * as2;
  } else {
    const CT invF = rcp(F);
    S_psi = K.d_psi * invF * invF * (gFx * (as2 * gpx + Nx) + gFy * (as2 * gpy + Ny)) +
            Qpsi * invF * K.inv_tau0;
    D_psi = K.d_psi * as2 * invF;
  }
  const CT an = P.le1 ? as2 * F : as2;
  const CT rate_psi = rcp(D_psi * CT(3) + CT(0.5));

  // velocity, forces, pressure (pressure recovered in FP64 in every mode)
  CT vx = CT(0), vy = CT(0), Fx = CT(0), Fy = CT(0), p = CT(0);
  const CT rho = fo.rho;
  const CT grx = K.drho * fo.gx, gry = K.drho * fo.gy;
  CT Fmx = CT(0), Fmy = CT(0);
  if constexpr (NS) {
    if constexpr (FLOWX) {
      // (div X)_b = 3 sum_i w_i sum_a c_ia X_ab(x + c_i), X = D (x) v0
      const CT w1 = CT(1.0 / 9), w2 = CT(1.0 / 36);
      auto Xs = [&](int c, int dy, int dx) { return s_X[c][ry + dy][rx + dx]; };
      // a = x components (X0: D_x v0_x, X1: D_x v0_y); a = y (X2, X3)
      const CT ax0 = w1 * (Xs(0, 0, 1) - Xs(0, 0, -1)) + w2 * ((Xs(0, 1, 1) - Xs(0, 1, -1)) + (Xs(0, -1, 1) - Xs(0, -1, -1)));
      const CT ax1 = w1 * (Xs(1, 0, 1) - Xs(1, 0, -1)) + w2 * ((Xs(1, 1, 1) - Xs(1, 1, -1)) + (Xs(1, -1, 1) - Xs(1, -1, -1)));
      const CT ay2 = w1 * (Xs(2, 1, 0) - Xs(2, -1, 0)) + w2 * ((Xs(2, 1, 1) + Xs(2, 1, -1)) - (Xs(2, -1, -1) + Xs(2, -1, 1)));
      const CT ay3 = w1 * (Xs(3, 1, 0) - Xs(3, -1, 0)) + w2 * ((Xs(3, 1, 1) + Xs(3, 1, -1)) - (Xs(3, -1, -1) + Xs(3, -1, 1)));
      Fmx = K.drho * CT(3) * (ax0 + ay2);
      Fmy = K.drho * CT(3) * (ax1 + ay3);
    }
    const CT Fby = -(rho - K.rho_l) * K.g;
    const CT rvx = jx + CT(0.5) * (fo.Fsx + Fmx);
    const CT rvy = jy + CT(0.5) * (fo.Fsy + Fby + Fmy);
    const CT onechi = CT(1) - fo.chi;
    const CT irho = rcp(rho);
    vx = onechi * rvx * irho;
    vy = onechi * rvy * irho;
    Fx = fo.Fsx + Fmx - CT(2) * fo.chi * rvx;
    Fy = fo.Fsy + Fby + Fmy - CT(2) * fo.chi * rvy;
    const double vvd = (double)vx * vx + (double)vy * vy;
    const double s0 = -LN::w[0] * vvd * 1.5;
    double sum = 0.0;
#pragma unroll
    for (int i = 1; i < QN; ++i) sum += (double)fns[i];
    p = CT(LN::cs2 / (1.0 - LN::w[0]) *
           (sum + 0.5 * ((double)vx * grx + (double)vy * gry) + (double)rho * s0));
  }

  // the step's stencil results, for an adjoint sweep that does not redo them
  if (P.tape) {
    CT* t = (CT*)P.tape;
    const CT tv[TAPE_PLANES] = {fo.gx, fo.gy, fo.lap, gpx, gpy, gUx, gUy, Fmx, Fmy};
#pragma unroll
    for (int k = 0; k < TAPE_PLANES; ++k) t[(long long)k * N + idx] = tv[k];
  }

  if (mode == 1) {
    const double m9[9] = {(double)phi, (double)psi, (double)C, (double)theta, (double)U, (double)p,
                          (double)vx, (double)vy, 0.0};
    put_macros(P, mout, idx, m9);
    return;
  }

  // stores: plane i of a set at byte (o + i) * N * S + idx * S
  const uint32_t nbyte = (uint32_t)idx * S;
  // 16-bit storage: stochastic rounding keyed on (node, step, plane)
  constexpr bool LOWP = sizeof(typename Store<ST>::raw) == 2;
  constexpr int QMAX = NS ? QN : ((PHI && QP > QS) ? QP : QS);
  const RoundBits<LOWP ? (QMAX + 1) / 2 : 1> rb(LOWP ? round_seed(P, (uint32_t)idx) : 0u, LOWP && P.sr);
  // store of population i of the set whose first plane is o
  // (one address form for every grid: the plane's base is uniform, the node
  // offset one 64-bit shift-add; a run-time choice between two forms would
  // merge them into a VGPR pointer computed per store)
  auto st = [&](int o, int i, CT v) {
    typename Store<ST>::raw* p = fout + (long long)(o + i) * N + idx;
    uint32_t r = 0u;
    if constexpr (LOWP) r = rb.bits(i);
    store_pop<ST, CT, STREAM>(P, p, v, r);
  };
  auto hst = [&](int plane, CT v) {
    put<STREAM, HT>(hist + (long long)plane * N + idx, (HT)v);
  };

  // ---- NS collision: f* = feq + F/2 + (1 - s_nu) P_s (f - feq + F/2),
  // P_s the orthogonal projector on the moments c_x^2 - c_y^2 and c_x c_y
  if constexpr (NS) {
    const CT nu = (K.mu_g + (K.mu_l - K.mu_g) * phi) * rcp(rho);
    const CT s_nu = rcp(nu * CT(3) + CT(0.5));
    const CT vv = vx * vx + vy * vy;
    const CT vF = vx * Fx + vy * Fy;
    // Velocity and pressure sides (non-equilibrium extrapolation, Sec. 3
    // boundary paragraph): the slot of population i leaving across one holds
    // what the node pulls back along j = opp(i) on the next step, its own f*_j
    // plus f^eq_j(p, rho, v_in) - f^eq_j(p, rho, v) (velocity side) or
    // f^eq_j(0, rho, v) - f^eq_j(p, rho, v) = -w_j p / cs2 (pressure side);
    // a velocity side takes precedence where both are crossed.
    // nee_out: 0 none, 1 velocity side, 2 pressure side.
    auto nee_out = [&](int i) -> int {
      if constexpr (!SYM) return 0;
      if (fast || !(P.vel | P.pres)) return 0;
      const int dx = LN::c[i][0], dy = LN::c[i][1];
      auto across = [&](int m) {
        return (dx > 0 && x == P.nx - 1 && ((m >> 3) & 1)) || (dx < 0 && x == 0 && (m & 1)) ||
               (dy > 0 && y == P.ny - 1 && ((m >> 4) & 1)) || (dy < 0 && y == 0 && ((m >> 1) & 1));
      };
      return across(P.vel) ? 1 : (across(P.pres) ? 2 : 0);
    };
    auto nee = [&](int j, int kind) -> CT {
      if (kind == 2) return -CT(LN::w[j]) * p * CT(3);
      const CT cx = CT(LN::c[j][0]), cy = CT(LN::c[j][1]);
      const CT bx = CT(P.vin[0]), by = CT(P.vin[1]);
      const CT cb = cx * bx + cy * by, cv = cx * vx + cy * vy;
      return rho * CT(LN::w[j]) * ((cb - cv) * CT(3) + (cb * cb - cv * cv) * CT(4.5) - (bx * bx + by * by - vv) * CT(1.5));
    };
    if constexpr (sizeof(CT) == 4) {
      // FP32 compute: the same collision in moment form.  On the 4th-order
      // isotropic lattice the traceless stress moments of f^eq and of F/2 are
      // rho T:vv and T:(vF + cs2 v grad(rho)) (symmetrised), and for i > 0
      // f_i^eq + F_i/2 = w_i [A + c.v (3 rho + 4.5 (rho c.v + c.F) + 1.5 c.grad(rho)) + 1.5 c.F]
      // with A = 3p - 1.5 rho v.v - 1.5 v.F; f_0^eq + F_0/2 = w_0 A - 3p.
      const CT r = CT(1) - s_nu;
      const CT A = CT(3) * p - CT(1.5) * rho * vv - CT(1.5) * vF;
      CT s1 = CT(0), s2 = CT(0);
#pragma unroll
      for (int i = 1; i < QN; ++i) {
        const int t1 = LN::c[i][0] * LN::c[i][0] - LN::c[i][1] * LN::c[i][1], t2 = LN::c[i][0] * LN::c[i][1];
        if (t1 > 0) s1 += fns[i]; else if (t1 < 0) s1 -= fns[i];
        if (t2 > 0) s2 += fns[i]; else if (t2 < 0) s2 -= fns[i];
      }
      const CT m1 = s1 - rho * (vx * vx - vy * vy) + (vx * Fx - vy * Fy) + CT(1.0 / 3) * (vx * grx - vy * gry);
      const CT m2 = s2 - rho * vx * vy + CT(0.5) * (vx * Fy + vy * Fx) + CT(1.0 / 6) * (vx * gry + vy * grx);
      const CT q1 = CT(0.25) * r * m1, q2 = CT(0.25) * r * m2;
      const CT rho3 = CT(3) * rho;
      auto post = [&](int i) -> CT {
        const CT cx = CT(LN::c[i][0]), cy = CT(LN::c[i][1]);
        const CT w = CT(LN::w[i]);
        if (i == 0) return w * A - CT(3) * p;
        const CT cv = cx * vx + cy * vy, cF = cx * Fx + cy * Fy, cg = cx * grx + cy * gry;
        const CT t = cv * (rho3 + CT(4.5) * (rho * cv + cF) + CT(1.5) * cg) + CT(1.5) * cF + A;
        return w * t + ((cx * cx - cy * cy) * q1 + (cx * cy) * q2);
      };
#pragma unroll
      for (int i = 0; i < QN; ++i) {
        CT fs = post(i);
        if (const int kind = nee_out(i)) fs = post(LN::opp[i]) + nee(LN::opp[i], kind);
        st(P.o_ns, i, fs);
      }
    } else {
    CT fneq[QN], fhalf[QN];
    CT m1 = CT(0), m2 = CT(0);   // projections on c_x^2 - c_y^2 and c_x c_y
#pragma unroll
    for (int i = 0; i < QN; ++i) {
      const CT cx = CT(LN::c[i][0]), cy = CT(LN::c[i][1]);
      const CT cv = cx * vx + cy * vy;
      const CT cF = cx * Fx + cy * Fy;
      const CT w = CT(LN::w[i]);
      CT feq = w * p * CT(3) + rho * w * (cv * CT(3) + cv * cv * CT(4.5) - vv * CT(1.5));
      if (i == 0) feq -= p * CT(3);
      const CT cg = cx * grx + cy * gry;
      const CT Ft = w * (cv * cg * CT(3) + cF * CT(3) + (cv * cF - vF * CT(1.0 / 3)) * CT(9));
      fhalf[i] = feq + CT(0.5) * Ft;
      fneq[i] = fns[i] - feq + CT(0.5) * Ft;
      m1 += (cx * cx - cy * cy) * fneq[i];
      m2 += (cx * cy) * fneq[i];
    }
    const CT r = CT(1) - s_nu;
    auto post = [&](int i) -> CT {
      const CT cx = CT(LN::c[i][0]), cy = CT(LN::c[i][1]);
      return fhalf[i] + r * ((cx * cx - cy * cy) * m1 * CT(0.25) + (cx * cy) * m2 * CT(0.25));
    };
#pragma unroll
    for (int i = 0; i < QN; ++i) {
      CT fs = post(i);
      if (const int kind = nee_out(i)) fs = post(LN::opp[i]) + nee(LN::opp[i], kind);
      st(P.o_ns, i, fs);
    }
    }
  }

  // ---- CAC collision
  const CT phivx = phi * vx, phivy = phi * vy;
  if constexpr (PHI) {
    CT pvx0 = phivx, pvy0 = phivy;
    if (!first) { pvx0 = h_pv0; pvy0 = h_pv1; }
    const CT gx_ = (phivx - pvx0) + CT(LP::cs2) * fo.sharp * fo.nx;
    const CT gy_ = (phivy - pvy0) + CT(LP::cs2) * fo.sharp * fo.ny;
    const CT s1 = K.s_phi;
    CT feq[QP], G[QP];
    CT jx_ = CT(0), jy_ = CT(0), gjx = CT(0), gjy = CT(0);
#pragma unroll
    for (int i = 0; i < QP; ++i) {
      const CT cx = CT(LP::c[i][0]), cy = CT(LP::c[i][1]);
      const CT w = CT(LP::w[i]);
      // equilibrium w phi (1 + c.v/cs2), less w under deviation storage
      if constexpr (DEV) feq[i] = w * dphi + w * phi * (cx * vx + cy * vy) * CT(1.0 / LP::cs2);
      else feq[i] = w * phi * (CT(1) + (cx * vx + cy * vy) * CT(1.0 / LP::cs2));
      G[i] = w * (cx * gx_ + cy * gy_) * CT(1.0 / LP::cs2);
      jx_ += cx * (fph[i] - feq[i]); jy_ += cy * (fph[i] - feq[i]);
      gjx += cx * G[i]; gjy += cy * G[i];
    }
    const CT inv_fn = CT(1.0 / LP::flux_norm);
#pragma unroll
    for (int i = 0; i < QP; ++i) {
      const CT cx = CT(LP::c[i][0]), cy = CT(LP::c[i][1]);
      const CT Pf = (cx * jx_ + cy * jy_) * inv_fn;        // projector on the flux moments
      const CT PG = (cx * gjx + cy * gjy) * inv_fn;
      const CT fs = feq[i] + (CT(1) - s1) * Pf + CT(0.5) * G[i] + CT(0.5) * (CT(1) - s1) * PG;
      st(P.o_phi, i, fs);
    }
    hst(P.h_phiv, phivx);
    hst(P.h_phiv + 1, phivy);
  }

  // ---- AAC collision with the time-stretched store
  if constexpr (PSI) {
    CT Sprev = S_psi;
    if (!first) Sprev = h_S;
    const CT inv_an = rcp(an);
    CT jx_ = CT(0), jy_ = CT(0);
#pragma unroll
    for (int i = 0; i < QS; ++i) {
      const CT d = fps[i] - CT(LS::w[i]) * dpsi;
      jx_ += CT(LS::c[i][0]) * d; jy_ += CT(LS::c[i][1]) * d;
    }
    const CT inv_as2 = P.le1 ? rcp(as2) : inv_an;
    const CT gNx = -Nx * inv_as2, gNy = -Ny * inv_as2;  // G_i = -w_i c_i.N / a_s^2
#pragma unroll
    for (int i = 0; i < QS; ++i) {
      const CT cx = CT(LS::c[i][0]), cy = CT(LS::c[i][1]);
      const CT w = CT(LS::w[i]);
      const CT G = w * (cx * gNx + cy * gNy);
      CT fstar = w * dpsi + (CT(1) - rate_psi) * (cx * jx_ + cy * jy_) * CT(0.5) + w * S_psi +
                 CT(0.5) * w * (S_psi - Sprev) + (CT(1) - CT(0.5) * rate_psi) * G;
      // anti-bounce-back to psi_l = -1 (stored less the rest value r_psi)
      if (far_out(i)) fstar = CT(2) * w * (CT(-1) - r_psi) - fstar;
      // f_i(x + c_i) before this step; across a wall it is the own f_opp(i)
      const int dx = LS::c[i][0], dy = LS::c[i][1];
      const bool across = !fast && ((P.wall[0] && (x + dx < 0 || x + dx >= P.nx)) ||
                                    (P.wall[1] && (y + dy < 0 || y + dy >= P.ny)));
      const CT old = across ? fps[LS::opp[i]] : s_fps[i][ry + dy][rx + dx];
      const CT fs = (fstar - (CT(1) - an) * old) * inv_an;
      st(P.o_psi, i, fs);
    }
  }

  // ---- solute collision
  if constexpr (CC) {
    CT psi_prev = psi;
    if (!first) psi_prev = h_psi;
    const CT at = -K.aW0 * a_s * lin * (psi - psi_prev);
    const CT Jat_x = at * ex, Jat_y = at * ey;
    const CT jv = K.D * q * C * K.sharp * (om > CT(0) ? om : CT(0));   // sqrt(2 beta_phi)/W_phi (phi_l - phi)+
    const CT Jx = jv * fo.nx, Jy = jv * fo.ny;
    const CT m = CT(1) - k1 * h;
    const CT invm = rcp(m);
    const CT dr = K.D * q * C * k1 * invm * invm * CT(0.5);   // grad h = grad psi / 2
    const CT Bx = C * vx - dr * gpx + k1 * (Jat_x + Jx);
    const CT By = C * vy - dr * gpy + k1 * (Jat_y + Jy);
    CT Bpx = Bx, Bpy = By;
    if (!first) { Bpx = h_B0; Bpy = h_B1; }
    const CT s1 = rcp(K.D * q * invm * CT(3) + CT(0.5));
    CT jx_ = CT(0), jy_ = CT(0);
#pragma unroll
    for (int i = 0; i < QS; ++i) { jx_ += CT(LS::c[i][0]) * fc[i]; jy_ += CT(LS::c[i][1]) * fc[i]; }
    jx_ -= Bx; jy_ -= By;
    const CT dBx = Bx - Bpx, dBy = By - Bpy;
#pragma unroll
    for (int i = 0; i < QS; ++i) {
      const CT cx = CT(LS::c[i][0]), cy = CT(LS::c[i][1]);
      const CT w = CT(LS::w[i]);
      const CT feq = w * dC + w * (cx * Bx + cy * By) * CT(3);
      const CT G = w * (cx * dBx + cy * dBy) * CT(3);
      CT fs = feq + (CT(1) - s1) * (cx * jx_ + cy * jy_) * CT(0.5) + (CT(1) - CT(0.5) * s1) * G;
      if (far_out(i)) fs = CT(2) * w * (CT(1) - r_C) - fs;      // anti-bounce-back to C = 1
      st(P.o_c, i, fs);
    }
    hst(P.h_B, Bx);
    hst(P.h_B + 1, By);
  }

  // ---- heat collision
  if constexpr (TH) {
    const CT Hvx = H * vx, Hvy = H * vy;
    CT Hpx = Hvx, Hpy = Hvy;
    if (!first) { Hpx = h_Hv0; Hpy = h_Hv1; }
    const CT s1 = s_th;
    CT jx_ = CT(0), jy_ = CT(0);
#pragma unroll
    for (int i = 0; i < QS; ++i) { jx_ += CT(LS::c[i][0]) * fth[i]; jy_ += CT(LS::c[i][1]) * fth[i]; }
    jx_ -= Hvx; jy_ -= Hvy;
    const CT dx_ = Hvx - Hpx, dy_ = Hvy - Hpy;
#pragma unroll
    for (int i = 0; i < QS; ++i) {
      const CT cx = CT(LS::c[i][0]), cy = CT(LS::c[i][1]);
      const CT w = CT(LS::w[i]);
      // equilibrium less r_i = w theta0; H (the sum of g) is rho times the
      // model's H, so the rest equilibrium rho H + (w - 1) theta is
      // H + (w - 1) theta, less w theta0: dH + (w - 1) dtheta
      CT geq = w * dtheta + w * (cx * Hvx + cy * Hvy) * CT(3);
      if (i == 0) {
        if constexpr (DEV) geq = K.varheat ? dH + (w - CT(1)) * dtheta : -h + w * dtheta;
        else geq = H + (w - CT(1)) * theta;
      }
      const CT G = w * (cx * dx_ + cy * dy_) * CT(3);
      CT gs = geq + (CT(1) - s1) * (cx * jx_ + cy * jy_) * CT(0.5) + (CT(1) - CT(0.5) * s1) * G;
      if (far_out(i)) gs = CT(2) * w * (K.theta0 - r_H) - gs;   // anti-bounce-back to theta0
      st(P.o_th, i, gs);
    }
    hst(P.h_Hv, Hvx);
    hst(P.h_Hv + 1, Hvy);
  }

  if constexpr (PSI) {
    hst(P.h_psi, psi);
    hst(P.h_S, S_psi);
  }
}

// ------------------------------------------------------------------ launch
template <int FIELDS, int QP, class ST, class HT, class CT>
hipError_t launch_step2d_t(const DevParams& P, const void* fin, void* fout, void* hist,
                           double* mout, int mode, hipStream_t s) {
  constexpr int STX = StepTile<FIELDS, ST>::X, STY = StepTile<FIELDS, ST>::Y, SNT = StepTile<FIELDS, ST>::N;
  dim3 grid(((P.nx + STX - 1) / STX) * ((P.ny + STY - 1) / STY));
  using raw = typename Store<ST>::raw;
  const bool sym = P.sym || P.far;
#define PFL_LAUNCH2(SYMV, NTV)                                                                  \
  hipLaunchKernelGGL((step2d_kernel<FIELDS, QP, ST, HT, CT, SYMV, NTV>), grid, dim3(SNT), 0, s, P, \
                     (const raw*)fin, (raw*)fout, (HT*)hist, mout, mode)
  if (sym && P.nt) PFL_LAUNCH2(true, true);
  else if (sym) PFL_LAUNCH2(true, false);
  else if (P.nt) PFL_LAUNCH2(false, true);
  else PFL_LAUNCH2(false, false);
#undef PFL_LAUNCH2
  return hipGetLastError();
}

template <class ST, class HT, class CT>
static hipError_t dispatch_fields(const DevParams& P, int fields, const void* fin, void* fout,
                                  void* hist, double* mout, int mode, hipStream_t s, bool& ok) {
  ok = true;
  const bool q9 = P.q_phi == 9;
#define PFL_CASE(F)                                                                              \
  case F:                                                                                        \
    return q9 ? launch_step2d_t<F, 9, ST, HT, CT>(P, fin, fout, hist, mout, mode, s)             \
              : launch_step2d_t<F, 5, ST, HT, CT>(P, fin, fout, hist, mout, mode, s);
  switch (fields) {
    PFL_CASE(F_NS | F_PHI | F_PSI | F_C | F_TH)
    PFL_CASE(F_PSI | F_C)
    PFL_CASE(F_PSI | F_C | F_TH)
    PFL_CASE(F_NS | F_PHI)
    PFL_CASE(F_PHI | F_PSI | F_C | F_TH)
    PFL_CASE(F_PSI)
    PFL_CASE(F_PHI)
    PFL_CASE(F_NS | F_PSI | F_TH)
    PFL_CASE(F_NS | F_PSI | F_C | F_TH)
    PFL_CASE(F_PSI | F_TH)
    default:
      ok = false;
      return hipSuccess;
  }
#undef PFL_CASE
}

}  // namespace pfl
