// Kernels of the discrete adjoint of the fused 2D step, instantiated once
// per compute type: FP64 in pfl_adj2d.hip (strict IEEE arithmetic), FP32 in
// pfl_adj2d_lowp.hip (contraction and reciprocals allowed).
//
// Discrete adjoint of the fused 2D step: lambda^n = (d Phi / d x^n)^T lambda^{n+1}
// and the parameter gradient lambda^{n+1} . d Phi / d(eps4, k), with the state
// x in node form (pre-collision populations at each node, then the history
// planes: the layout of pfl_get_state).  In node form the populations a node
// pulls are its own state entries, and the value a node stores for direction
// i becomes the node-form population i of x + c_i at the next step (or of the
// node itself in direction opp(i) across a wall).
//
// Two passes per step, in the forward's compute type (FP64 for FP64 storage,
// FP32 otherwise); the adjoint state and the scratch planes are held in that
// type, the parameter-gradient sums in FP64:
//  R1 (tile kernel): recompute the forward step of the tile as the forward
//     kernel does, then reverse the node-local phase (collisions, forces,
//     anisotropy, kinetics) by hand.  Writes the adjoints of the node's own
//     populations and history, of its moments, and of the stencil inputs it
//     read (grad phi, lap phi, grad psi, grad U, the mass-flux force F_m).
//  R2 (flow with bubbles only): the transposed divergence gives the adjoint
//     of X = D_phi (x) v0 at each node; reverse X and the flow quantities
//     behind it.  Computed on the tile of R3 and its ring into LDS.
//  R3: the transposed stencils turn the stencil-input adjoints into moment
//     adjoints and U = U(C, psi; k) is reversed (a tile pass with R2, a node
//     pass otherwise).
// The moment adjoints reach every population of a set (the momentum ones
// through c_i), and the time-stretched store's reads of a neighbour's old
// value reach that neighbour's population: lambda^n is the populations part R1
// wrote plus these terms.  Within a sweep over many steps they are not added
// to lambda^n: R3 keeps them in the P_ planes (and A_OLD holds the old-value
// reads), and the next step's R1 adds them where it reads lambda^n.  The
// broadcast kernel adds them to lambda^n where a sweep ends.
// A read through a wall ghost (mirror node) is credited to the mirror node
// with the direction reflected on that axis, and for X with its sign flipped.
#pragma once
#include "pfl_kernels.h"
#include "pfl_step2d.h"

namespace pfl {

namespace {


using CT = double;

// FP64 scratch planes of N nodes (adj_scratch)
enum : int {
  AM_PHI = 0, AM_PSI, AM_C, AM_H, AM_JX, AM_JY, AM_U,                  // moment adjoints
  AS_GPHX, AS_GPHY, AS_LAP, AS_GPSX, AS_GPSY, AS_GUX, AS_GUY, AS_FMX, AS_FMY,  // stencil-input adjoints
  FW_PHI, FW_PSI, FW_C, FW_JX, FW_JY, FW_GX, FW_GY, FW_LAP,            // forward values for R2/R3
  PG_EPS, PG_K1, PG_OM,                                                // per-node parameter gradients
  A_OLD0,                                                              // 5 planes: time-stretched store reads
  P_JX = A_OLD0 + 5, P_JY, P_PHI, P_PSI, P_C, P_H,                     // moment terms of lambda^n not yet added
  A_NPLANES
};

__device__ __forceinline__ int total_pop_planes(const DevParams& P) {
  if (P.o_th >= 0) return P.o_th + P.q_sc;
  if (P.o_c >= 0) return P.o_c + P.q_sc;
  if (P.o_psi >= 0) return P.o_psi + P.q_sc;
  if (P.o_phi >= 0) return P.o_phi + P.q_phi;
  return P.o_ns + P.q_ns;
}

// Element `node` of a plane, addressed by a 32-bit byte offset from the
// plane's base (a plane holds fewer than 2^32 bytes).
template <class T>
__device__ __forceinline__ const T& at_node(const T* plane, uint32_t node) {
  return *(const T*)((const char*)plane + node * (uint32_t)sizeof(T));
}
template <class T>
__device__ __forceinline__ T& at_node(T* plane, uint32_t node) {
  return *(T*)((char*)plane + node * (uint32_t)sizeof(T));
}

// The node-form entry that receives the value a node at (x, y), flat index
// idx, stores for direction i: population j of node `node`, with j = i at
// x + c_i (`regular`), j = opp(i) at the node itself across a wall or a
// far-field side (`wall`; `far` when a far-field side was crossed), or, across
// a symmetry plane (SYM), the population with that component of c_i reversed
// at x + c_i with that coordinate kept.  c_j = (sx c_ix, sy c_iy).  A wall
// dominates at corners.  In a fast tile x + c_i lies inside the domain.
struct PushTarget {
  uint32_t node;
  int j;
  bool wall, regular, far;
  int sx, sy;
};
template <int Q, bool SYM = false>
__device__ __forceinline__ PushTarget push_to(const DevParams& P, bool fast, uint32_t idx, int x, int y, int i) {
  using L = Lat<Q>;
  PushTarget t{idx + (uint32_t)(L::c[i][0] + L::c[i][1] * P.nx), i, false, true, false, 1, 1};
  if (fast) return t;
  int tx = x + L::c[i][0], ty = y + L::c[i][1];
  bool symx = false, symy = false;
  if (tx < 0 || tx >= P.nx) {
    if (P.wall[0]) {
      const bool lo = tx < 0;
      if (SYM && sym_side(P, 0, lo)) symx = true;
      else { t.wall = true; t.far = t.far || (SYM && far_side(P, 0, lo)); }
    } else tx = tx < 0 ? tx + P.nx : tx - P.nx;
  }
  if (ty < 0 || ty >= P.ny) {
    if (P.wall[1]) {
      const bool lo = ty < 0;
      if (SYM && sym_side(P, 1, lo)) symy = true;
      else { t.wall = true; t.far = t.far || (SYM && far_side(P, 1, lo)); }
    } else ty = ty < 0 ? ty + P.ny : ty - P.ny;
  }
  if (t.wall) {
    t.node = idx; t.j = L::opp[i]; t.regular = false; t.sx = -1; t.sy = -1;
    return t;
  }
  if (SYM && (symx || symy)) {
    t.regular = false;
    if (symx) { tx = x; t.sx = -1; }
    if (symy) { ty = y; t.sy = -1; }
    t.j = symx ? (symy ? L::refl[1][L::refl[0][i]] : L::refl[0][i]) : L::refl[1][i];
  }
  t.node = (uint32_t)ty * (uint32_t)P.nx + (uint32_t)tx;
  return t;
}

// The reader of a stencil entry: node z is read by the node r = z - c at
// offset c, or, when z - c lies beyond a wall, by the mirror node at the
// offset reflected on that axis (its ghost at that offset mirrors z).
struct Reader {
  uint32_t node;
  int cx, cy;      // offset as seen from the reader
  int sign;        // (-1)^(walls and far-field sides crossed): D_phi (x) v0 is odd there
  int osign;       // (-1)^(symmetry planes crossed): its off-diagonal components are odd there
  int fsign;       // (-1)^(far-field sides crossed): psi and U ghosts are odd there
};
__device__ __forceinline__ Reader reader_of(const DevParams& P, int x, int y, int cx, int cy) {
  Reader r;
  int rx = x - cx, ry = y - cy;
  r.cx = cx; r.cy = cy; r.sign = 1; r.osign = 1; r.fsign = 1;
  if (rx < 0 || rx >= P.nx) {
    if (P.wall[0]) {
      const bool lo = rx < 0;
      rx = lo ? -1 - rx : 2 * P.nx - 1 - rx; r.cx = -cx;
      if (sym_side(P, 0, lo)) r.osign = -r.osign;
      else { r.sign = -r.sign; if (far_side(P, 0, lo)) r.fsign = -r.fsign; }
    } else rx = rx < 0 ? rx + P.nx : rx - P.nx;
  }
  if (ry < 0 || ry >= P.ny) {
    if (P.wall[1]) {
      const bool lo = ry < 0;
      ry = lo ? -1 - ry : 2 * P.ny - 1 - ry; r.cy = -cy;
      if (sym_side(P, 1, lo)) r.osign = -r.osign;
      else { r.sign = -r.sign; if (far_side(P, 1, lo)) r.fsign = -r.fsign; }
    } else ry = ry < 0 ? ry + P.ny : ry - P.ny;
  }
  r.node = (uint32_t)ry * (uint32_t)P.nx + (uint32_t)rx;
  return r;
}


// ------------------------------------------------------------------- R1
// TAPED: the step's stencil results (grad and Laplacian of phi, grad psi,
// grad U, mass-flux force) are read from the tape the forward step wrote, so
// the tile's halo and its LDS stencils are not redone.
// FP32 compute without symmetry planes or far-field sides: two waves per SIMD
// asked of the register allocator (it then fits 256 VGPRs without scratch;
// left alone it takes a few AGPRs beyond them and runs one wave per SIMD).
// The other instantiations would spill to scratch and keep one wave.
template <int FIELDS, int QP, class ST, class HT, class CT, bool TAPED, bool SYM = false>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu((SYM || sizeof(CT) == 8) ? 1 : 2)))
void adj_local_kernel(const DevParams P,
                                                       const typename Store<ST>::raw* __restrict__ fin,
                                                       const HT* __restrict__ hist,
                                                       const CT* __restrict__ tape,
                                                       const CT* __restrict__ lam_in,
                                                       CT* __restrict__ lam_out,
                                                       CT* __restrict__ S) {
  constexpr bool NS = FIELDS & F_NS, PHI = FIELDS & F_PHI, PSI = FIELDS & F_PSI;
  constexpr bool CC = FIELDS & F_C, TH = FIELDS & F_TH;
  constexpr bool FLOWX = NS && PHI;
  constexpr int R = FLOWX ? 2 : 1;
  constexpr int RX = TX + 2 * R, RY = TY + 2 * R;
  constexpr int QN = 9, QS = 5;
  using LN = Lat<9>;
  using LS = Lat<5>;
  using LP = Lat<QP>;
  using raw = typename Store<ST>::raw;
  const KP<CT>& K = kp<CT>(P);

  __shared__ CT s_phi[RY][RX];
  __shared__ CT s_psi[RY][RX];
  __shared__ CT s_U[RY][RX];
  __shared__ CT s_jx[NS ? RY : 1][NS ? RX : 1];
  __shared__ CT s_jy[NS ? RY : 1][NS ? RX : 1];
  __shared__ CT s_X[FLOWX ? 4 : 1][FLOWX ? RY : 1][FLOWX ? RX : 1];

  const int tid = threadIdx.x;
  const int lx = tid % TX, ly = tid / TX;
  const int gtx = (P.nx + TX - 1) / TX;
  const int lt = logical_tile(blockIdx.x, gtx * ((P.ny + TY - 1) / TY));
  const int bx0 = (lt % gtx) * TX, by0 = (lt / gtx) * TY;
  const int x = bx0 + lx, y = by0 + ly;
  const bool own = (x < P.nx) && (y < P.ny);
  const long long N = P.N;
  const long long idx = (long long)y * P.nx + x;
  const raw* fin_ns = fin + (long long)(NS ? P.o_ns : 0) * N;
  const raw* fin_phi = fin + (long long)(PHI ? P.o_phi : 0) * N;
  const raw* fin_psi = fin + (long long)(PSI ? P.o_psi : 0) * N;
  const raw* fin_c = fin + (long long)(CC ? P.o_c : 0) * N;
  const raw* fin_th = fin + (long long)(TH ? P.o_th : 0) * N;
  const CT k1 = K.k1;
  const bool first = P.first != 0;
  // every pull of the tile and its halo stays inside the domain
  const bool fast = P.fast && bx0 >= R + 1 && by0 >= R + 1 && bx0 + TX + R + 1 <= P.nx &&
                    by0 + TY + R + 1 <= P.ny;

  // ---- forward phase A: own node, full populations (rest values added back)
  CT fns[NS ? QN : 1], fph[PHI ? QP : 1], fps[PSI ? QS : 1], fc[CC ? QS : 1], fth[TH ? QS : 1];
  CT phi = CT(1), psi = CT(-1), C = CT(0), H = CT(0), U = K.U0, jx = CT(0), jy = CT(0);
  CT h_psi = CT(0), h_S = CT(0), h_pv0 = CT(0), h_pv1 = CT(0), h_B0 = CT(0), h_B1 = CT(0);
  CT h_Hv0 = CT(0), h_Hv1 = CT(0);
  int gid = 0;
  auto hld = [&](int plane) -> CT { return CT(hist[(long long)plane * N + idx]); };
  if (own) {
    if (PSI) gid = P.grain[idx];
    if (!first) {
      if constexpr (PSI) { h_psi = hld(P.h_psi); h_S = hld(P.h_S); }
      if constexpr (PHI) { h_pv0 = hld(P.h_phiv); h_pv1 = hld(P.h_phiv + 1); }
      if constexpr (CC) { h_B0 = hld(P.h_B); h_B1 = hld(P.h_B + 1); }
      if constexpr (TH) { h_Hv0 = hld(P.h_Hv); h_Hv1 = hld(P.h_Hv + 1); }
    }
    if constexpr (NS) {
      pull<QN, ST, CT, SYM>(fast, fin_ns, P, x, y, fns);
#pragma unroll
      for (int i = 0; i < QN; ++i) {
        fns[i] += CT(P.ref_ns[i]);
        jx += CT(LN::c[i][0]) * fns[i];
        jy += CT(LN::c[i][1]) * fns[i];
      }
    }
    if constexpr (PHI) {
      pull<QP, ST, CT, SYM>(fast, fin_phi, P, x, y, fph);
      phi = CT(0);
#pragma unroll
      for (int i = 0; i < QP; ++i) { fph[i] += CT(P.ref_phi[i]); phi += fph[i]; }
    }
    if constexpr (PSI) {
      pull<QS, ST, CT, SYM>(fast, fin_psi, P, x, y, fps);
      psi = CT(0);
#pragma unroll
      for (int i = 0; i < QS; ++i) { fps[i] += CT(P.ref_psi[i]); psi += fps[i]; }
    }
    if constexpr (CC) {
      pull<QS, ST, CT, SYM>(fast, fin_c, P, x, y, fc);
#pragma unroll
      for (int i = 0; i < QS; ++i) { fc[i] += CT(P.ref_c[i]); C += fc[i]; }
      const CT h0 = (psi + CT(1)) * CT(CT(0.5));
      U = (C / (CT(1) - k1 * h0) - CT(1)) * K.inv_k1;
    }
    if constexpr (TH) {
      pull<QS, ST, CT, SYM>(fast, fin_th, P, x, y, fth);
#pragma unroll
      for (int i = 0; i < QS; ++i) { fth[i] += CT(P.ref_th[i]); H += fth[i]; }
    }
    if constexpr (!TAPED) {
      s_phi[ly + R][lx + R] = phi;
      s_psi[ly + R][lx + R] = psi;
      s_U[ly + R][lx + R] = U;
      if constexpr (NS) { s_jx[ly + R][lx + R] = jx; s_jy[ly + R][lx + R] = jy; }
    }
  }
  if constexpr (!TAPED) {
  for (int k = tid; k < RX * RY; k += NT) {
    const int rx = k % RX, ry = k / RX;
    const int tx = rx - R, ty = ry - R;
    const int gx0 = bx0 + tx, gy0 = by0 + ty;
    const bool inner = tx >= 0 && tx < TX && ty >= 0 && ty < TY;
    if (inner && gx0 < P.nx && gy0 < P.ny) continue;
    const int gx = map_coord(gx0, P.nx, P.wall[0]), gy = map_coord(gy0, P.ny, P.wall[1]);
    const bool ring1 = rx >= R - 1 && rx <= RX - R && ry >= R - 1 && ry <= RY - R;
    CT hphi = CT(1), hpsi = CT(-1), hU = K.U0, hjx = CT(0), hjy = CT(0);
    if constexpr (PHI) {
      CT f[QP];
      pull<QP, ST, CT, SYM>(fast, fin_phi, P, gx, gy, f);
      hphi = CT(0);
#pragma unroll
      for (int i = 0; i < QP; ++i) hphi += f[i] + CT(P.ref_phi[i]);
    }
    if (ring1) {
      if constexpr (PSI) {
        CT f[QS];
        pull<QS, ST, CT, SYM>(fast, fin_psi, P, gx, gy, f);
        hpsi = CT(0);
#pragma unroll
        for (int i = 0; i < QS; ++i) hpsi += f[i] + CT(P.ref_psi[i]);
      }
      if constexpr (CC) {
        CT f[QS];
        pull<QS, ST, CT, SYM>(fast, fin_c, P, gx, gy, f);
        CT hC = CT(0);
#pragma unroll
        for (int i = 0; i < QS; ++i) hC += f[i] + CT(P.ref_c[i]);
        const CT h0 = (hpsi + CT(1)) * CT(CT(0.5));
        hU = (hC / (CT(1) - k1 * h0) - CT(1)) * K.inv_k1;
      }
      if constexpr (NS) {
        CT f[QN];
        pull<QN, ST, CT, SYM>(fast, fin_ns, P, gx, gy, f);
#pragma unroll
        for (int i = 0; i < QN; ++i) {
          f[i] += CT(P.ref_ns[i]);
          hjx += CT(LN::c[i][0]) * f[i];
          hjy += CT(LN::c[i][1]) * f[i];
        }
      }
    }
    if (SYM && P.far) {
      // ghost across an odd number of far-field sides: psi and U odd about
      // psi_l = -1 and U = 0 (as the forward step)
      const bool fx = gx0 < 0 ? far_side(P, 0, true) : gx0 >= P.nx && far_side(P, 0, false);
      const bool fy = gy0 < 0 ? far_side(P, 1, true) : gy0 >= P.ny && far_side(P, 1, false);
      if (fx != fy) { hpsi = CT(-2) - hpsi; hU = -hU; }
    }
    s_phi[ry][rx] = hphi;
    s_psi[ry][rx] = hpsi;
    s_U[ry][rx] = hU;
    if constexpr (NS) { s_jx[ry][rx] = hjx; s_jy[ry][rx] = hjy; }
  }
  __syncthreads();
  }

  // ---- forward phase B
  FlowNode<CT> fo;
  if constexpr (FLOWX && !TAPED) {
    constexpr int AX = TX + 2, AY = TY + 2;
    for (int k = tid; k < AX * AY; k += NT) {
      const int rx = k % AX + R - 1, ry = k / AX + R - 1;
      const int gx0 = bx0 + rx - R, gy0 = by0 + ry - R;
      int mx = rx, my = ry;
      CT sgn = CT(1), sod = CT(1);    // walls: all components odd; symmetry planes: off-diagonal odd
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
        FlowNode<CT> hn;
        flow_node<NS, PHI, CT, RX>(K, s_phi, s_psi, s_jx, s_jy, my, mx, hn);
        X0 = sgn * hn.Dx * hn.v0x; X1 = sgn * sod * hn.Dx * hn.v0y;
        X2 = sgn * sod * hn.Dy * hn.v0x; X3 = sgn * hn.Dy * hn.v0y;
      }
      s_X[0][ry][rx] = X0; s_X[1][ry][rx] = X1; s_X[2][ry][rx] = X2; s_X[3][ry][rx] = X3;
    }
    __syncthreads();
  }
  if (!own) return;
  const int ry = ly + R, rx = lx + R;
  auto tp = [&](int k) -> CT { return tape[(long long)k * N + idx]; };
  if constexpr (TAPED)
    flow_node_from<NS, CT>(K, phi, psi, jx, jy, tp(0), tp(1), tp(2), fo);
  else
    flow_node<NS, PHI, CT, RX>(K, s_phi, s_psi, s_jx, s_jy, ry, rx, fo);

  // forward values needed by the later passes
  S[FW_PHI * N + idx] = phi;
  S[FW_PSI * N + idx] = psi;
  S[FW_C * N + idx] = C;
  S[FW_JX * N + idx] = jx;
  S[FW_JY * N + idx] = jy;
  S[FW_GX * N + idx] = fo.gx;
  S[FW_GY * N + idx] = fo.gy;
  S[FW_LAP * N + idx] = fo.lap;

  // ---- forward phase C (every intermediate kept)
  const CT h = (psi + CT(1)) * CT(CT(0.5));
  const CT qraw = (CT(1) - psi) * CT(CT(0.5));
  const CT q = clamp01(qraw);
  // temperature (theta = (sum g / rho + h) / c_p with the heat properties
  // linear in phi; H + h when they are matched) and the heat rate
  CT theta = K.theta0, th_rh = CT(1), th_cp = CT(1), th_s1 = K.s_th;
  if constexpr (TH) {
    if (K.varheat) {
      th_rh = K.th_rho_g + (CT(1) - K.th_rho_g) * phi;
      th_cp = K.th_cp_g + (CT(1) - K.th_cp_g) * phi;
      const CT kh = K.th_k_g + (CT(1) - K.th_k_g) * phi;
      theta = (H + th_rh * h) / (th_rh * th_cp);
      th_s1 = CT(1) / (K.alpha_cs * kh + CT(0.5));
    } else {
      theta = H + h;
    }
  }
  CT gpx = CT(0), gpy = CT(0), gUx = CT(0), gUy = CT(0);
  if constexpr (TAPED) {
    gpx = tp(3); gpy = tp(4); gUx = tp(5); gUy = tp(6);
  } else {
    if constexpr (PSI) grad9<CT, RX>(s_psi, ry, rx, gpx, gpy);
    if constexpr (CC) grad9<CT, RX>(s_U, ry, rx, gUx, gUy);
  }
  const CT dn = K.dn;
  const CT invp = CT(1) / sqrt(gpx * gpx + gpy * gpy + dn);
  const CT ex = gpx * invp, ey = gpy * invp;
  const CT cth = P.grain_cs[2 * gid], sth = P.grain_cs[2 * gid + 1];
  const CT eps = K.eps4;
  const CT rxa = cth * gpx + sth * gpy, rya = -sth * gpx + cth * gpy;
  const CT rx2 = rxa * rxa, ry2 = rya * rya;
  const CT G = rx2 + ry2, S4 = rx2 * rx2 + ry2 * ry2;
  const CT iG = CT(1) / (G + dn);
  const CT a_s = CT(1) + eps * (CT(4) * S4 - CT(3) * G * G) * iG * iG;
  const CT iG3 = iG * iG * iG;
  const CT pre = CT(4) * eps * G * a_s * iG3;
  const CT Ax = CT(4) * rx2 * G + (CT(4) * rx2 - CT(3) * G) * dn - CT(4) * S4;
  const CT Ay = CT(4) * ry2 * G + (CT(4) * ry2 - CT(3) * G) * dn - CT(4) * S4;
  const CT Nrx = pre * rxa * Ax, Nry = pre * rya * Ay;
  const CT Nx = cth * Nrx - sth * Nry, Ny = sth * Nrx + cth * Nry;
  const CT an = a_s * a_s;
  const CT lin = CT(1) + k1 * U;
  const bool linp = lin > CT(0);
  const CT F = K.inv_Le + K.Mcinf * (linp ? lin : CT(0));
  const CT gFx = linp ? K.Mcinf * k1 * gUx : CT(0), gFy = linp ? K.Mcinf * k1 * gUy : CT(0);
  const CT om = CT(1) - phi;
  const CT ps1 = psi + CT(1);
  const CT f3psi = CT(2) * K.beta_inter * om * om * ps1;
  const CT s1m = (CT(1) - psi) * ps1;
  const CT pprime = CT(CT(30.0) / CT(32.0)) * s1m * s1m;
  const CT f2p = CT(CT(0.5)) * (CT(1) - psi) * ps1 * (CT(-2) * psi);
  const CT Qpsi = -(f2p + f3psi + K.lam * pprime * (theta + K.Mcinf * U));
  const CT invF = CT(1) / F;
  const CT T1 = gFx * (an * gpx + Nx) + gFy * (an * gpy + Ny);
  const CT S_psi = K.d_psi * invF * invF * T1 + Qpsi * invF * K.inv_tau0;
  const CT D_psi = K.d_psi * an * invF;
  const CT rate = CT(1) / (D_psi * CT(3) + CT(CT(0.5)));

  CT vx = CT(0), vy = CT(0), Fx = CT(0), Fy = CT(0), p = CT(0), Fmx = CT(0), Fmy = CT(0);
  CT rvx = CT(0), rvy = CT(0), Fby = CT(0);
  const CT rho = fo.rho;
  const CT grx = K.drho * fo.gx, gry = K.drho * fo.gy;
  const CT c0 = LN::cs2 / (CT(1.0) - CT(LN::w[0]));
  if constexpr (NS) {
    if constexpr (TAPED) {
      Fmx = tp(7);
      Fmy = tp(8);
    } else if constexpr (FLOWX) {
      const CT w1 = CT(CT(1.0) / 9), w2 = CT(CT(1.0) / 36);
      auto Xs = [&](int c, int dy, int dx) { return s_X[c][ry + dy][rx + dx]; };
      const CT ax0 = w1 * (Xs(0, 0, 1) - Xs(0, 0, -1)) + w2 * ((Xs(0, 1, 1) - Xs(0, 1, -1)) + (Xs(0, -1, 1) - Xs(0, -1, -1)));
      const CT ax1 = w1 * (Xs(1, 0, 1) - Xs(1, 0, -1)) + w2 * ((Xs(1, 1, 1) - Xs(1, 1, -1)) + (Xs(1, -1, 1) - Xs(1, -1, -1)));
      const CT ay2 = w1 * (Xs(2, 1, 0) - Xs(2, -1, 0)) + w2 * ((Xs(2, 1, 1) + Xs(2, 1, -1)) - (Xs(2, -1, -1) + Xs(2, -1, 1)));
      const CT ay3 = w1 * (Xs(3, 1, 0) - Xs(3, -1, 0)) + w2 * ((Xs(3, 1, 1) + Xs(3, 1, -1)) - (Xs(3, -1, -1) + Xs(3, -1, 1)));
      Fmx = K.drho * CT(3) * (ax0 + ay2);
      Fmy = K.drho * CT(3) * (ax1 + ay3);
    }
    Fby = -(rho - K.rho_l) * K.g;
    rvx = jx + CT(CT(0.5)) * (fo.Fsx + Fmx);
    rvy = jy + CT(CT(0.5)) * (fo.Fsy + Fby + Fmy);
    const CT onechi = CT(1) - fo.chi;
    vx = onechi * rvx / rho;
    vy = onechi * rvy / rho;
    Fx = fo.Fsx + Fmx - CT(2) * fo.chi * rvx;
    Fy = fo.Fsy + Fby + Fmy - CT(2) * fo.chi * rvy;
    const CT s0 = -CT(LN::w[0]) * (vx * vx + vy * vy) * CT(1.5);
    CT sum = CT(0);
#pragma unroll
    for (int i = 1; i < QN; ++i) sum += fns[i];
    p = c0 * (sum + CT(0.5) * (vx * grx + vy * gry) + rho * s0);
  }

  // ---- reverse
  const int QT = total_pop_planes(P);
  auto lam_hist = [&](int hp) -> CT { return lam_in[(long long)(QT + hp) * N + idx]; };
  // lambda^{n+1} at a push target of the set at plane `base` (without the
  // moment terms the previous reverse step left open) and those terms (zero
  // planes when lambda^{n+1} is complete)
  auto lam_at = [&](int base, const PushTarget& t) -> CT {
    return at_node(lam_in + (long long)(base + t.j) * N, t.node);
  };
  auto pend_at = [&](int plane, const PushTarget& t) -> CT { return at_node(S + (long long)plane * N, t.node); };
  auto out_pop = [&](int plane, CT v) { lam_out[(long long)plane * N + idx] = v; };
  // adjoints of node-level quantities
  CT a_phi = 0, a_psi = 0, a_C = 0, a_H = 0, a_jx = 0, a_jy = 0, a_U = 0;
  CT a_vx = 0, a_vy = 0, a_Fx = 0, a_Fy = 0, a_p = 0, a_rho = 0, a_grx = 0, a_gry = 0;
  CT a_theta = 0, a_h = 0, a_q = 0, a_as = 0, a_an = 0, a_Nx = 0, a_Ny = 0, a_lin = 0;
  CT a_S = 0, a_rate = 0, a_gpx = 0, a_gpy = 0, a_ex = 0, a_ey = 0, a_gUx = 0, a_gUy = 0;
  CT a_om = 0, a_sharp = 0, a_fnx = 0, a_fny = 0, a_chi = 0, a_Fsx = 0, a_Fsy = 0, a_Fmx = 0, a_Fmy = 0;
  CT a_eps = 0, a_k1 = 0;
  CT a_Omega = 0;  // Omega through the far-field value theta0 = -Omega of the heat set
  CT a_th_s1 = 0;  // the heat relaxation rate
  CT a_fns[NS ? QN : 1] = {}, a_fph[PHI ? QP : 1] = {}, a_fps[PSI ? QS : 1] = {};
  CT a_fc[CC ? QS : 1] = {}, a_fth[TH ? QS : 1] = {}, a_old[PSI ? QS : 1] = {};
  CT a_hpsi = 0, a_hS = 0, a_hpv0 = 0, a_hpv1 = 0, a_hB0 = 0, a_hB1 = 0, a_hHv0 = 0, a_hHv1 = 0;

  // heat
  if constexpr (TH) {
    const CT Hvx = H * vx, Hvy = H * vy;
    CT Hpx = first ? Hvx : h_Hv0, Hpy = first ? Hvy : h_Hv1;
    CT jhx = -Hvx, jhy = -Hvy;
#pragma unroll
    for (int i = 0; i < QS; ++i) { jhx += CT(LS::c[i][0]) * fth[i]; jhy += CT(LS::c[i][1]) * fth[i]; }
    const CT dx_ = Hvx - Hpx, dy_ = Hvy - Hpy;
    const CT s1 = th_s1;
    CT a_Hvx = lam_hist(P.h_Hv), a_Hvy = lam_hist(P.h_Hv + 1);
    CT a_jhx = 0, a_jhy = 0, a_dx = 0, a_dy = 0;
#pragma unroll
    for (int i = 0; i < QS; ++i) {
      const CT cx = LS::c[i][0], cy = LS::c[i][1], w = LS::w[i];
      const PushTarget t = push_to<QS, SYM>(P, fast, (uint32_t)idx, x, y, i);
      CT ao = lam_at(P.o_th, t);
      ao += pend_at(P_H, t);
      if (SYM && t.far) {             // stored by anti-bounce-back: 2 w theta0 - g*, theta0 = -Omega
        a_Omega -= CT(2) * w * ao;
        ao = -ao;
      }
      a_jhx += ao * (1 - s1) * cx * CT(0.5);
      a_jhy += ao * (1 - s1) * cy * CT(0.5);
      a_dx += ao * (1 - CT(0.5) * s1) * 3 * w * cx;
      a_dy += ao * (1 - CT(0.5) * s1) * 3 * w * cy;
      // the heat rate (per node with variable k_T)
      if (K.varheat) a_th_s1 -= ao * CT(0.5) * ((cx * jhx + cy * jhy) + 3 * w * (cx * dx_ + cy * dy_));
      if (i == 0) { a_H += ao; a_theta += ao * (w - 1); }
      else { a_theta += ao * w; a_Hvx += ao * 3 * w * cx; a_Hvy += ao * 3 * w * cy; }
    }
    a_Hvx += a_dx; a_Hvy += a_dy;
    if (first) { a_Hvx -= a_dx; a_Hvy -= a_dy; } else { a_hHv0 -= a_dx; a_hHv1 -= a_dy; }
#pragma unroll
    for (int i = 0; i < QS; ++i) a_fth[i] += CT(LS::c[i][0]) * a_jhx + CT(LS::c[i][1]) * a_jhy;
    a_Hvx -= a_jhx; a_Hvy -= a_jhy;
    a_H += a_Hvx * vx + a_Hvy * vy;
    a_vx += a_Hvx * H; a_vy += a_Hvy * H;
  }

  // solute
  if constexpr (CC) {
    const CT psi_prev = first ? psi : h_psi;
    const CT dpt = psi - psi_prev;
    const CT at = -K.aW0 * a_s * lin * dpt;
    const CT Jatx = at * ex, Jaty = at * ey;
    const CT omp = om > 0 ? om : CT(0);
    const CT jv = K.D * q * C * K.sharp * omp;
    const CT Jx = jv * fo.nx, Jy = jv * fo.ny;
    const CT m = 1 - k1 * h;
    const CT invm = 1 / m;
    const CT dr = K.D * q * C * k1 * invm * invm * CT(0.5);
    const CT Bx = C * vx - dr * gpx + k1 * (Jatx + Jx);
    const CT By = C * vy - dr * gpy + k1 * (Jaty + Jy);
    const CT Bpx = first ? Bx : h_B0, Bpy = first ? By : h_B1;
    const CT s1 = 1 / (K.D * q * invm * 3 + CT(0.5));
    CT jcx = -Bx, jcy = -By;
#pragma unroll
    for (int i = 0; i < QS; ++i) { jcx += CT(LS::c[i][0]) * fc[i]; jcy += CT(LS::c[i][1]) * fc[i]; }
    const CT dBx = Bx - Bpx, dBy = By - Bpy;
    CT a_Bx = lam_hist(P.h_B), a_By = lam_hist(P.h_B + 1);
    CT a_s1 = 0, a_jcx = 0, a_jcy = 0, a_dBx = 0, a_dBy = 0;
#pragma unroll
    for (int i = 0; i < QS; ++i) {
      const CT cx = LS::c[i][0], cy = LS::c[i][1], w = LS::w[i];
      const PushTarget t = push_to<QS, SYM>(P, fast, (uint32_t)idx, x, y, i);
      CT ao = lam_at(P.o_c, t);
      ao += pend_at(P_C, t);
      if (SYM && t.far) ao = -ao;     // stored by anti-bounce-back: 2 w - f*
      a_C += ao * w;
      a_Bx += ao * 3 * w * cx;
      a_By += ao * 3 * w * cy;
      a_s1 += ao * (-(cx * jcx + cy * jcy) * CT(0.5) - CT(0.5) * 3 * w * (cx * dBx + cy * dBy));
      a_jcx += ao * (1 - s1) * cx * CT(0.5);
      a_jcy += ao * (1 - s1) * cy * CT(0.5);
      a_dBx += ao * (1 - CT(0.5) * s1) * 3 * w * cx;
      a_dBy += ao * (1 - CT(0.5) * s1) * 3 * w * cy;
    }
    a_Bx += a_dBx; a_By += a_dBy;
    if (first) { a_Bx -= a_dBx; a_By -= a_dBy; } else { a_hB0 -= a_dBx; a_hB1 -= a_dBy; }
#pragma unroll
    for (int i = 0; i < QS; ++i) a_fc[i] += CT(LS::c[i][0]) * a_jcx + CT(LS::c[i][1]) * a_jcy;
    a_Bx -= a_jcx; a_By -= a_jcy;
    CT a_invm = a_s1 * (-3 * K.D * q * s1 * s1);
    a_q += a_s1 * (-3 * K.D * invm * s1 * s1);
    // B = C v - dr grad psi + k1 (Jat + J)
    a_C += a_Bx * vx + a_By * vy;
    a_vx += a_Bx * C; a_vy += a_By * C;
    const CT a_dr = -(a_Bx * gpx + a_By * gpy);
    a_gpx -= a_Bx * dr; a_gpy -= a_By * dr;
    a_k1 += a_Bx * (Jatx + Jx) + a_By * (Jaty + Jy);
    const CT a_Jatx = a_Bx * k1, a_Jaty = a_By * k1, a_Jx = a_Bx * k1, a_Jy = a_By * k1;
    // dr = D q C k1 invm^2 / 2
    a_q += a_dr * CT(0.5) * K.D * C * k1 * invm * invm;
    a_C += a_dr * CT(0.5) * K.D * q * k1 * invm * invm;
    a_k1 += a_dr * CT(0.5) * K.D * q * C * invm * invm;
    a_invm += a_dr * K.D * q * C * k1 * invm;
    const CT a_m = -a_invm * invm * invm;
    a_k1 -= a_m * h;
    a_h -= a_m * k1;
    // J = jv n_phi
    const CT a_jv = a_Jx * fo.nx + a_Jy * fo.ny;
    a_fnx += a_Jx * jv; a_fny += a_Jy * jv;
    a_q += a_jv * K.D * C * K.sharp * omp;
    a_C += a_jv * K.D * q * K.sharp * omp;
    if (om > 0) a_om += a_jv * K.D * q * C * K.sharp;
    // Jat = at e_psi
    const CT a_at = a_Jatx * ex + a_Jaty * ey;
    a_ex += a_Jatx * at; a_ey += a_Jaty * at;
    a_as += a_at * (-K.aW0 * lin * dpt);
    a_lin += a_at * (-K.aW0 * a_s * dpt);
    const CT a_dpt = a_at * (-K.aW0 * a_s * lin);
    if (!first) { a_psi += a_dpt; a_hpsi -= a_dpt; }
  }

  // order parameter (time-stretched store)
  if constexpr (PSI) {
    const CT Sprev = first ? S_psi : h_S;
    const CT inv_an = 1 / an;
    CT jax = 0, jay = 0;
#pragma unroll
    for (int i = 0; i < QS; ++i) {
      const CT d = fps[i] - CT(LS::w[i]) * psi;
      jax += CT(LS::c[i][0]) * d; jay += CT(LS::c[i][1]) * d;
    }
    const CT gNx = -Nx * inv_an, gNy = -Ny * inv_an;
    CT a_inv_an = 0, a_jax = 0, a_jay = 0, a_gNx = 0, a_gNy = 0, a_Sprev = 0;
#pragma unroll
    for (int i = 0; i < QS; ++i) {
      const CT cx = LS::c[i][0], cy = LS::c[i][1], w = LS::w[i];
      const CT Gi = w * (cx * gNx + cy * gNy);
      const CT fstar = w * psi + (1 - rate) * (cx * jax + cy * jay) * CT(0.5) + w * S_psi +
                       CT(0.5) * w * (S_psi - Sprev) + (1 - CT(0.5) * rate) * Gi;
      const int dx = LS::c[i][0], dy = LS::c[i][1];
      const bool across = (P.wall[0] && (x + dx < 0 || x + dx >= P.nx)) ||
                          (P.wall[1] && (y + dy < 0 || y + dy >= P.ny));
      const CT old = across ? fps[LS::opp[i]]
                            : Store<ST>::template ld<CT>(fin_psi + (long long)i * N + idx) + CT(P.ref_psi[i]);
      const PushTarget t = push_to<QS, SYM>(P, fast, (uint32_t)idx, x, y, i);
      CT ao = lam_at(P.o_psi, t);
      {
        // the previous step's old-value read of this population is the
        // node's own A_OLD entry (rewritten below by this step)
        const CT old_prev = S[(long long)(A_OLD0 + i) * N + idx];
        CT v = pend_at(P_PSI, t);
        if (t.regular) v += old_prev;
        ao += v;
      }
      // across a far-field side f* was replaced by its anti-bounce-back 2 w psi_l - f*
      const bool abb = SYM && t.far;
      const CT fst = abb ? CT(-2) * w - fstar : fstar;
      const CT a_fstar = (abb ? -ao : ao) * inv_an;
      const CT a_oldi = -ao * (1 - an) * inv_an;
      a_an += ao * old * inv_an;
      a_inv_an += ao * (fst - (1 - an) * old);
      if (across) a_fps[LS::opp[i]] += a_oldi; else a_old[i] += a_oldi;
      a_psi += a_fstar * w;
      a_rate += a_fstar * (-(cx * jax + cy * jay) * CT(0.5) - CT(0.5) * Gi);
      a_jax += a_fstar * (1 - rate) * cx * CT(0.5);
      a_jay += a_fstar * (1 - rate) * cy * CT(0.5);
      a_S += a_fstar * CT(1.5) * w;
      a_Sprev -= a_fstar * CT(0.5) * w;
      const CT a_G = a_fstar * (1 - CT(0.5) * rate);
      a_gNx += a_G * w * cx; a_gNy += a_G * w * cy;
    }
    a_Nx -= a_gNx * inv_an; a_Ny -= a_gNy * inv_an;
    a_inv_an -= a_gNx * Nx + a_gNy * Ny;
#pragma unroll
    for (int i = 0; i < QS; ++i) a_fps[i] += CT(LS::c[i][0]) * a_jax + CT(LS::c[i][1]) * a_jay;
    a_an -= a_inv_an * inv_an * inv_an;
    if (first) a_S += a_Sprev; else a_hS += a_Sprev;
    a_psi += lam_hist(P.h_psi);
    a_S += lam_hist(P.h_S);
  }

  // bubble phase
  if constexpr (PHI) {
    const CT phivx = phi * vx, phivy = phi * vy;
    const CT s1 = K.s_phi;
    CT a_phivx = lam_hist(P.h_phiv), a_phivy = lam_hist(P.h_phiv + 1);
    const CT pvx0 = first ? phivx : h_pv0, pvy0 = first ? phivy : h_pv1;
    const CT gx_ = (phivx - pvx0) + CT(LP::cs2) * fo.sharp * fo.nx;
    const CT gy_ = (phivy - pvy0) + CT(LP::cs2) * fo.sharp * fo.ny;
    CT feq[QP], Gv[QP];
    CT jfx = 0, jfy = 0, gjx = 0, gjy = 0;
#pragma unroll
    for (int i = 0; i < QP; ++i) {
      const CT cx = LP::c[i][0], cy = LP::c[i][1], w = LP::w[i];
      feq[i] = w * phi * (1 + (cx * vx + cy * vy) * CT(1.0 / LP::cs2));
      Gv[i] = w * (cx * gx_ + cy * gy_) * CT(1.0 / LP::cs2);
      jfx += cx * (fph[i] - feq[i]); jfy += cy * (fph[i] - feq[i]);
      gjx += cx * Gv[i]; gjy += cy * Gv[i];
    }
    const CT ifn = CT(1.0) / LP::flux_norm;
    CT a_feq[QP], a_G[QP];
    CT a_jfx = 0, a_jfy = 0, a_gjx = 0, a_gjy = 0;
#pragma unroll
    for (int i = 0; i < QP; ++i) {
      const CT cx = LP::c[i][0], cy = LP::c[i][1];
      const PushTarget t = push_to<QP, SYM>(P, fast, (uint32_t)idx, x, y, i);
      CT ao = lam_at(P.o_phi, t);
      ao += pend_at(P_PHI, t);
      a_feq[i] = ao;
      a_jfx += ao * (1 - s1) * cx * ifn; a_jfy += ao * (1 - s1) * cy * ifn;
      a_G[i] = ao * CT(0.5);
      a_gjx += ao * CT(0.5) * (1 - s1) * cx * ifn; a_gjy += ao * CT(0.5) * (1 - s1) * cy * ifn;
    }
    CT a_gx_ = 0, a_gy_ = 0;
#pragma unroll
    for (int i = 0; i < QP; ++i) {
      const CT cx = LP::c[i][0], cy = LP::c[i][1], w = LP::w[i];
      a_G[i] += cx * a_gjx + cy * a_gjy;
      a_fph[i] += cx * a_jfx + cy * a_jfy;
      a_feq[i] -= cx * a_jfx + cy * a_jfy;
      a_gx_ += a_G[i] * w * cx * CT(1.0 / LP::cs2);
      a_gy_ += a_G[i] * w * cy * CT(1.0 / LP::cs2);
      a_phi += a_feq[i] * w * (1 + (cx * vx + cy * vy) * CT(1.0 / LP::cs2));
      a_vx += a_feq[i] * w * phi * cx * CT(1.0 / LP::cs2);
      a_vy += a_feq[i] * w * phi * cy * CT(1.0 / LP::cs2);
    }
    if (!first) { a_phivx += a_gx_; a_phivy += a_gy_; a_hpv0 -= a_gx_; a_hpv1 -= a_gy_; }
    a_sharp += (a_gx_ * fo.nx + a_gy_ * fo.ny) * CT(LP::cs2);
    a_fnx += a_gx_ * CT(LP::cs2) * fo.sharp;
    a_fny += a_gy_ * CT(LP::cs2) * fo.sharp;
    a_phi += a_phivx * vx + a_phivy * vy;
    a_vx += a_phivx * phi; a_vy += a_phivy * phi;
  }

  // flow
  if constexpr (NS) {
    const CT nu = (K.mu_g + (K.mu_l - K.mu_g) * phi) / rho;
    const CT s_nu = 1 / (nu * 3 + CT(0.5));
    const CT vv = vx * vx + vy * vy;
    const CT vF = vx * Fx + vy * Fy;
    CT feq[QN], Ft[QN];
    CT m1 = 0, m2 = 0;
#pragma unroll
    for (int i = 0; i < QN; ++i) {
      const CT cx = LN::c[i][0], cy = LN::c[i][1], w = LN::w[i];
      const CT cv = cx * vx + cy * vy, cF = cx * Fx + cy * Fy;
      feq[i] = w * p * 3 + rho * w * (cv * 3 + cv * cv * CT(4.5) - vv * CT(1.5));
      if (i == 0) feq[i] -= p * 3;
      const CT cg = cx * grx + cy * gry;
      Ft[i] = w * (cv * cg * 3 + cF * 3 + (cv * cF - vF * CT(1.0 / 3)) * 9);
      const CT fneq = fns[i] - feq[i] + CT(0.5) * Ft[i];
      m1 += (cx * cx - cy * cy) * fneq;
      m2 += (cx * cy) * fneq;
    }
    const CT r = 1 - s_nu;
    CT a_r = 0, a_m1 = 0, a_m2 = 0, ao_[QN];
#pragma unroll
    for (int i = 0; i < QN; ++i) {
      const CT cx = LN::c[i][0], cy = LN::c[i][1];
      const PushTarget t = push_to<QN, SYM>(P, fast, (uint32_t)idx, x, y, i);
      ao_[i] = lam_at(P.o_ns, t);
      {
        // c_j . a_j at the target: c_j = -c_i across a wall, c_i with the
        // plane's component reversed across a symmetry plane
        CT v = CT(0);
        if (LN::c[i][0] != 0) v += CT(t.sx) * cx * pend_at(P_JX, t);
        if (LN::c[i][1] != 0) v += CT(t.sy) * cy * pend_at(P_JY, t);
        ao_[i] += v;
      }
      a_r += ao_[i] * CT(0.25) * ((cx * cx - cy * cy) * m1 + (cx * cy) * m2);
      a_m1 += ao_[i] * r * CT(0.25) * (cx * cx - cy * cy);
      a_m2 += ao_[i] * r * CT(0.25) * (cx * cy);
    }
    CT a_vF = 0, a_vv = 0;
#pragma unroll
    for (int i = 0; i < QN; ++i) {
      const CT cx = LN::c[i][0], cy = LN::c[i][1], w = LN::w[i];
      const CT cv = cx * vx + cy * vy, cF = cx * Fx + cy * Fy, cg = cx * grx + cy * gry;
      const CT a_fneq = (cx * cx - cy * cy) * a_m1 + (cx * cy) * a_m2;
      a_fns[i] += a_fneq;
      const CT a_feq = ao_[i] - a_fneq;
      const CT a_Ft = CT(0.5) * a_fneq + CT(0.5) * ao_[i];
      const CT a_cg = a_Ft * w * 3 * cv;
      a_grx += a_cg * cx; a_gry += a_cg * cy;
      const CT a_cF = a_Ft * w * (3 + 9 * cv);
      CT a_cv = a_Ft * w * (9 * cF + 3 * cg);
      a_vF -= 3 * w * a_Ft;
      a_p += a_feq * (3 * w - (i == 0 ? CT(3.0) : CT(0.0)));
      a_rho += a_feq * w * (cv * 3 + cv * cv * CT(4.5) - vv * CT(1.5));
      a_cv += a_feq * rho * w * (3 + 9 * cv);
      a_vv -= a_feq * rho * w * CT(1.5);
      a_vx += a_cv * cx; a_vy += a_cv * cy;
      a_Fx += a_cF * cx; a_Fy += a_cF * cy;
    }
    a_vx += a_vF * Fx; a_vy += a_vF * Fy; a_Fx += a_vF * vx; a_Fy += a_vF * vy;
    a_vx += 2 * a_vv * vx; a_vy += 2 * a_vv * vy;
    const CT a_snu = -a_r;
    const CT a_nu = a_snu * (-3 * s_nu * s_nu);
    a_phi += a_nu * (K.mu_l - K.mu_g) / rho;
    a_rho -= a_nu * nu / rho;
    // pressure
    const CT a_sum = a_p * c0;
#pragma unroll
    for (int i = 1; i < QN; ++i) a_fns[i] += a_sum;
    a_vx += a_p * c0 * (CT(0.5) * grx - rho * CT(LN::w[0]) * 3 * vx);
    a_vy += a_p * c0 * (CT(0.5) * gry - rho * CT(LN::w[0]) * 3 * vy);
    a_grx += a_p * c0 * CT(0.5) * vx; a_gry += a_p * c0 * CT(0.5) * vy;
    a_rho += a_p * c0 * (-CT(LN::w[0]) * (vx * vx + vy * vy) * CT(1.5));
    // forces and velocity
    const CT onechi = 1 - fo.chi;
    a_Fsx += a_Fx; a_Fmx += a_Fx; a_chi -= 2 * rvx * a_Fx;
    CT a_rvx = -2 * fo.chi * a_Fx;
    a_Fsy += a_Fy; CT a_Fby = a_Fy; a_Fmy += a_Fy; a_chi -= 2 * rvy * a_Fy;
    CT a_rvy = -2 * fo.chi * a_Fy;
    const CT irho = 1 / rho;
    const CT a_onechi = (a_vx * rvx + a_vy * rvy) * irho;
    a_rvx += a_vx * onechi * irho; a_rvy += a_vy * onechi * irho;
    const CT a_irho = (a_vx * rvx + a_vy * rvy) * onechi;
    a_rho -= a_irho * irho * irho;
    a_chi -= a_onechi;
    a_jx += a_rvx; a_Fsx += CT(0.5) * a_rvx; a_Fmx += CT(0.5) * a_rvx;
    a_jy += a_rvy; a_Fsy += CT(0.5) * a_rvy; a_Fby += CT(0.5) * a_rvy; a_Fmy += CT(0.5) * a_rvy;
    a_rho -= K.g * a_Fby;
  }

  // source, kinetics, rates of the order parameter
  {
    const CT a_Dpsi = a_rate * (-3 * rate * rate);
    a_an += a_Dpsi * K.d_psi * invF;
    CT a_invF = a_Dpsi * K.d_psi * an;
    a_invF += a_S * (2 * K.d_psi * invF * T1 + Qpsi * K.inv_tau0);
    const CT a_T1 = a_S * K.d_psi * invF * invF;
    const CT a_Q = a_S * invF * K.inv_tau0;
    const CT a_gFx = a_T1 * (an * gpx + Nx), a_gFy = a_T1 * (an * gpy + Ny);
    a_an += a_T1 * (gFx * gpx + gFy * gpy);
    a_gpx += a_T1 * gFx * an; a_gpy += a_T1 * gFy * an;
    a_Nx += a_T1 * gFx; a_Ny += a_T1 * gFy;
    const CT a_F = -a_invF * invF * invF;
    const CT a_pp = -a_Q * K.lam * (theta + K.Mcinf * U);
    a_theta -= a_Q * K.lam * pprime;
    a_U -= a_Q * K.lam * pprime * K.Mcinf;
    const CT a_s1m = a_pp * (CT(30.0) / CT(32.0)) * 2 * s1m;
    a_psi += a_s1m * (-2 * psi);
    const CT a_f3 = -a_Q;
    a_om += a_f3 * 4 * K.beta_inter * om * ps1;
    a_psi += a_f3 * 2 * K.beta_inter * om * om;
    const CT a_f2 = -a_Q;
    a_psi += a_f2 * (3 * psi * psi - 1);
    a_phi -= a_om;
    // kinetics
    if (linp) {
      a_lin += a_F * K.Mcinf;
      a_k1 += K.Mcinf * (a_gFx * gUx + a_gFy * gUy);
      a_gUx += a_gFx * K.Mcinf * k1; a_gUy += a_gFy * K.Mcinf * k1;
    }
    a_k1 += a_lin * U;
    a_U += a_lin * k1;
  }

  // anisotropy
  {
    a_as += 2 * a_s * a_an;
    const CT a_Nrx = cth * a_Nx + sth * a_Ny, a_Nry = -sth * a_Nx + cth * a_Ny;
    const CT a_pre = a_Nrx * rxa * Ax + a_Nry * rya * Ay;
    CT a_rx = a_Nrx * pre * Ax, a_ry = a_Nry * pre * Ay;
    const CT a_Ax = a_Nrx * pre * rxa, a_Ay = a_Nry * pre * rya;
    CT a_rx2 = a_Ax * (4 * G + 4 * dn), a_ry2 = a_Ay * (4 * G + 4 * dn);
    CT a_G = a_Ax * (4 * rx2 - 3 * dn) + a_Ay * (4 * ry2 - 3 * dn);
    CT a_S4 = -4 * (a_Ax + a_Ay);
    a_eps += a_pre * 4 * G * a_s * iG3;
    a_G += a_pre * 4 * eps * a_s * iG3;
    a_as += a_pre * 4 * eps * G * iG3;
    CT a_iG = a_pre * 4 * eps * G * a_s * 3 * iG * iG;
    a_eps += a_as * (4 * S4 - 3 * G * G) * iG * iG;
    a_S4 += a_as * eps * 4 * iG * iG;
    a_G += a_as * eps * (-6 * G) * iG * iG;
    a_iG += a_as * eps * (4 * S4 - 3 * G * G) * 2 * iG;
    a_G -= a_iG * iG * iG;
    a_rx2 += 2 * rx2 * a_S4 + a_G; a_ry2 += 2 * ry2 * a_S4 + a_G;
    a_rx += 2 * rxa * a_rx2; a_ry += 2 * rya * a_ry2;
    a_gpx += cth * a_rx - sth * a_ry;
    a_gpy += sth * a_rx + cth * a_ry;
  }

  // h, q, theta (= H + h with the heat equation, the constant theta0 without), e_psi
  if constexpr (TH) {
    if (K.varheat) {
      // theta = (H / rho + h) / c_p; rho, c_p, k_T (through the rate) linear in phi
      a_H += a_theta / (th_rh * th_cp);
      a_h += a_theta / th_cp;
      a_phi += a_theta * (-(H / (th_rh * th_rh * th_cp)) * (CT(1) - K.th_rho_g) -
                          theta / th_cp * (CT(1) - K.th_cp_g));
      a_phi -= a_th_s1 * th_s1 * th_s1 * K.alpha_cs * (CT(1) - K.th_k_g);
    } else {
      a_H += a_theta;
      a_h += a_theta;
    }
  }
  a_psi += CT(0.5) * a_h;
  if (qraw > 0 && qraw < 1) a_psi -= CT(0.5) * a_q;
  {
    a_gpx += a_ex * invp; a_gpy += a_ey * invp;
    const CT a_invp = a_ex * gpx + a_ey * gpy;
    const CT i3 = invp * invp * invp;
    a_gpx -= a_invp * gpx * i3; a_gpy -= a_invp * gpy * i3;
  }

  // own flow quantities (rho, chi, surface tension, sharpening, normal, grad rho)
  CT a_gphx = a_grx * K.drho, a_gphy = a_gry * K.drho, a_lap = 0;
  {
    a_phi += a_rho * K.drho;
    const CT ps1o = psi + 1;
    const CT omo = 1 - phi;
    const CT f1p = CT(0.5) * omo * phi * (1 - 2 * phi);
    const CT f3p = -2 * K.beta_inter * omo * ps1o * ps1o;
    const CT mu = f1p + f3p - K.Wphi2 * fo.lap;
    if constexpr (NS) {
      const CT a_mu = K.k_s * (a_Fsx * fo.gx + a_Fsy * fo.gy);
      a_gphx += a_Fsx * K.k_s * mu; a_gphy += a_Fsy * K.k_s * mu;
      a_lap -= K.Wphi2 * a_mu;
      a_phi += a_mu * (-2 * K.beta_inter) * (-1) * ps1o * ps1o;
      a_psi += a_mu * (-2 * K.beta_inter) * omo * 2 * ps1o;
      a_phi += a_mu * CT(0.5) * (1 - 6 * phi + 6 * phi * phi);
    }
    const CT ho = (psi + 1) * CT(0.5);
    if (ho > 0 && ho < 1) a_psi += CT(0.5) * a_chi;
    const CT dw = omo * phi;
    if (dw > 0) a_phi += a_sharp * K.sharp * (1 - 2 * phi);
    const CT inv = 1 / sqrt(fo.gx * fo.gx + fo.gy * fo.gy + dn);
    a_gphx += a_fnx * inv; a_gphy += a_fny * inv;
    const CT a_inv = a_fnx * fo.gx + a_fny * fo.gy;
    a_gphx -= a_inv * fo.gx * inv * inv * inv;
    a_gphy -= a_inv * fo.gy * inv * inv * inv;
  }

  // ---- writes: population adjoints (moment parts follow in R3), history,
  // moment and stencil adjoints, parameter gradients
  if constexpr (NS) {
#pragma unroll
    for (int i = 0; i < QN; ++i) out_pop(P.o_ns + i, a_fns[i]);
  }
  if constexpr (PHI) {
#pragma unroll
    for (int i = 0; i < QP; ++i) out_pop(P.o_phi + i, a_fph[i]);
  }
  if constexpr (PSI) {
#pragma unroll
    for (int i = 0; i < QS; ++i) { out_pop(P.o_psi + i, a_fps[i]); S[(long long)(A_OLD0 + i) * N + idx] = a_old[i]; }
  }
  if constexpr (CC) {
#pragma unroll
    for (int i = 0; i < QS; ++i) out_pop(P.o_c + i, a_fc[i]);
  }
  if constexpr (TH) {
#pragma unroll
    for (int i = 0; i < QS; ++i) out_pop(P.o_th + i, a_fth[i]);
  }
  auto out_hist = [&](int hp, CT v) { lam_out[(long long)(QT + hp) * N + idx] = v; };
  if constexpr (PSI) { out_hist(P.h_psi, a_hpsi); out_hist(P.h_S, a_hS); }
  if constexpr (PHI) { out_hist(P.h_phiv, a_hpv0); out_hist(P.h_phiv + 1, a_hpv1); }
  if constexpr (CC) { out_hist(P.h_B, a_hB0); out_hist(P.h_B + 1, a_hB1); }
  if constexpr (TH) { out_hist(P.h_Hv, a_hHv0); out_hist(P.h_Hv + 1, a_hHv1); }
  S[AM_PHI * N + idx] = a_phi;
  S[AM_PSI * N + idx] = a_psi;
  S[AM_C * N + idx] = a_C;
  S[AM_H * N + idx] = a_H;
  S[AM_JX * N + idx] = a_jx;
  S[AM_JY * N + idx] = a_jy;
  S[AM_U * N + idx] = a_U;
  S[AS_GPHX * N + idx] = a_gphx;
  S[AS_GPHY * N + idx] = a_gphy;
  S[AS_LAP * N + idx] = a_lap;
  S[AS_GPSX * N + idx] = a_gpx;
  S[AS_GPSY * N + idx] = a_gpy;
  S[AS_GUX * N + idx] = a_gUx;
  S[AS_GUY * N + idx] = a_gUy;
  S[AS_FMX * N + idx] = a_Fmx;
  S[AS_FMY * N + idx] = a_Fmy;
  S[PG_EPS * N + idx] = a_eps;
  S[PG_K1 * N + idx] = a_k1;
  if constexpr (SYM) S[PG_OM * N + idx] = a_Omega;
}

// ------------------------------------------------------------------- R2
// Adjoint of X = D_phi (x) v0 at node n, from the transposed divergence of
// the mass-flux force adjoints, reversed through the node's flow quantities:
// the increments of the stencil-input and moment adjoints at n.
template <class CT>
struct FlowDelta {
  CT gx, gy, lap, phi, psi, jx, jy;
};
template <class CT>
__device__ __forceinline__ FlowDelta<CT> flow_delta(const DevParams& P, const CT* __restrict__ S, uint32_t n,
                                                    int x, int y) {
  using LN = Lat<9>;
  const long long N = P.N;
  const KP<CT>& K = kp<CT>(P);
  auto pl = [&](int k) -> const CT* { return S + (long long)k * N; };
  // X-bar_ab(z) = sum over readers 3 drho w c'_a Fm-bar_b(reader) (odd ghosts)
  CT aX0 = CT(0), aX1 = CT(0), aX2 = CT(0), aX3 = CT(0);
#pragma unroll
  for (int i = 1; i < 9; ++i) {
    const Reader r = reader_of(P, x, y, LN::c[i][0], LN::c[i][1]);
    const CT f = CT(3.0 * LN::w[i]) * K.drho * CT(r.sign);
    const CT fo = f * CT(r.osign);    // off-diagonal components: odd across symmetry planes
    const CT fmx = at_node(pl(AS_FMX), r.node), fmy = at_node(pl(AS_FMY), r.node);
    aX0 += f * CT(r.cx) * fmx;   // X_xx feeds Fm_x through c_x
    aX1 += fo * CT(r.cx) * fmy;  // X_xy feeds Fm_y through c_x
    aX2 += fo * CT(r.cy) * fmx;  // X_yx feeds Fm_x through c_y
    aX3 += f * CT(r.cy) * fmy;   // X_yy feeds Fm_y through c_y
  }
  const CT phi = at_node(pl(FW_PHI), n), psi = at_node(pl(FW_PSI), n);
  const CT jx = at_node(pl(FW_JX), n), jy = at_node(pl(FW_JY), n);
  const CT gx = at_node(pl(FW_GX), n), gy = at_node(pl(FW_GY), n), lap = at_node(pl(FW_LAP), n);
  // forward flow quantities at the node
  const CT inv = CT(1) / sqrt(gx * gx + gy * gy + K.dn);
  const CT nx = gx * inv, ny = gy * inv;
  const CT om = CT(1) - phi, dw = om * phi;
  const CT sharp = K.sharp * (dw > CT(0) ? dw : CT(0));
  const CT Dx = K.M_phi * (gx - sharp * nx), Dy = K.M_phi * (gy - sharp * ny);
  const CT h = (psi + CT(1)) * CT(0.5);
  const CT chi = clamp01(h);
  const CT rho = K.rho_g + K.drho * phi;
  const CT ps1 = psi + CT(1);
  const CT mu = CT(0.5) * om * phi * (CT(1) - CT(2) * phi) - CT(2) * K.beta_inter * om * ps1 * ps1 - K.Wphi2 * lap;
  const CT Fsx = K.k_s * mu * gx, Fsy = K.k_s * mu * gy;
  const CT Fby = -(rho - K.rho_l) * K.g;
  const CT sc = (CT(1) - chi) / rho;
  const CT ux = jx + CT(0.5) * Fsx, uy = jy + CT(0.5) * (Fsy + Fby);
  const CT v0x = sc * ux, v0y = sc * uy;
  // X = D (x) v0
  const CT a_Dx = aX0 * v0x + aX1 * v0y, a_Dy = aX2 * v0x + aX3 * v0y;
  const CT a_v0x = aX0 * Dx + aX2 * Dy, a_v0y = aX1 * Dx + aX3 * Dy;
  // v0 = s (j + (Fs + Fb)/2)
  const CT a_s = a_v0x * ux + a_v0y * uy;
  FlowDelta<CT> d;
  d.jx = sc * a_v0x;
  d.jy = sc * a_v0y;
  const CT a_Fsx = CT(0.5) * sc * a_v0x, a_Fsy = CT(0.5) * sc * a_v0y, a_Fby = CT(0.5) * sc * a_v0y;
  const CT a_chi = -a_s / rho;
  CT a_rho = -a_s * (CT(1) - chi) / (rho * rho) - K.g * a_Fby;
  const CT a_mu = K.k_s * (a_Fsx * gx + a_Fsy * gy);
  CT a_gx = a_Fsx * K.k_s * mu + K.M_phi * a_Dx;
  CT a_gy = a_Fsy * K.k_s * mu + K.M_phi * a_Dy;
  d.lap = -K.Wphi2 * a_mu;
  CT a_phi = a_mu * (CT(0.5) * (CT(1) - CT(6) * phi + CT(6) * phi * phi) + CT(2) * K.beta_inter * ps1 * ps1);
  CT a_psi = a_mu * (CT(-4) * K.beta_inter * om * ps1);
  // D = M (g - sharp n)
  const CT a_sharp = -K.M_phi * (a_Dx * nx + a_Dy * ny);
  const CT a_nx = -K.M_phi * sharp * a_Dx, a_ny = -K.M_phi * sharp * a_Dy;
  if (dw > CT(0)) a_phi += a_sharp * K.sharp * (CT(1) - CT(2) * phi);
  a_gx += a_nx * inv; a_gy += a_ny * inv;
  const CT a_inv = a_nx * gx + a_ny * gy;
  a_gx -= a_inv * gx * inv * inv * inv;
  a_gy -= a_inv * gy * inv * inv * inv;
  a_phi += a_rho * K.drho;
  if (h > CT(0) && h < CT(1)) a_psi += CT(0.5) * a_chi;
  d.gx = a_gx; d.gy = a_gy; d.phi = a_phi; d.psi = a_psi;
  return d;
}

// ------------------------------------------------------------------- R3
// Transposed stencils and U(C, psi; k) at node n: writes the moment terms of
// lambda^n to the P_ planes and the block's parameter partials (slot `slot`).
// Dl supplies the R2 increments not yet in the planes: at the node (own) and
// at the reader of direction i (at), or nothing (Dl::active false).
struct NoDelta {
  static constexpr bool active = false;
};
template <int FIELDS, int QP, class CT, class Dl>
__device__ __forceinline__ void assemble_node(const DevParams& P, CT* __restrict__ S, uint32_t n, int x, int y,
                                              bool live, double* __restrict__ part, int slot, int accumulate,
                                              const Dl& dl) {
  constexpr bool NS = FIELDS & F_NS, PHI = FIELDS & F_PHI, PSI = FIELDS & F_PSI;
  constexpr bool CC = FIELDS & F_C, TH = FIELDS & F_TH;
  using LN = Lat<9>;
  const long long N = P.N;
  const KP<CT>& K = kp<CT>(P);
  auto pl = [&](int k) -> const CT* { return S + (long long)k * N; };
  CT am_phi = at_node(pl(AM_PHI), n), as_lap = at_node(pl(AS_LAP), n), am_psi = at_node(pl(AM_PSI), n);
  CT am_jx = at_node(pl(AM_JX), n), am_jy = at_node(pl(AM_JY), n);
  if constexpr (Dl::active) {
    const FlowDelta<CT> d = dl.own();
    am_phi += d.phi; as_lap += d.lap; am_psi += d.psi; am_jx += d.jx; am_jy += d.jy;
  }
  // transposed isotropic stencils (gradient 3 sum w c f, Laplacian 6 sum w (f - f0))
  CT a_phi = am_phi - CT(6.0 * (1.0 - LN::w[0])) * as_lap;
  CT a_psi = am_psi, a_U = at_node(pl(AM_U), n);
#pragma unroll
  for (int i = 1; i < 9; ++i) {
    const Reader r = reader_of(P, x, y, LN::c[i][0], LN::c[i][1]);
    const CT w3 = CT(3.0 * LN::w[i]), w6 = CT(6.0 * LN::w[i]);
    const CT cx = CT(r.cx), cy = CT(r.cy);
    if constexpr (PHI) {
      CT gpx = at_node(pl(AS_GPHX), r.node), gpy = at_node(pl(AS_GPHY), r.node), lp = at_node(pl(AS_LAP), r.node);
      if constexpr (Dl::active) {
        const FlowDelta<CT> d = dl.at(i);
        gpx += d.gx; gpy += d.gy; lp += d.lap;
      }
      a_phi += w3 * (cx * gpx + cy * gpy) + w6 * lp;
    }
    // psi and U ghosts across a far-field side are odd about their far-field values
    const CT wf = w3 * CT(r.fsign);
    if constexpr (PSI) a_psi += wf * (cx * at_node(pl(AS_GPSX), r.node) + cy * at_node(pl(AS_GPSY), r.node));
    if constexpr (CC) a_U += wf * (cx * at_node(pl(AS_GUX), r.node) + cy * at_node(pl(AS_GUY), r.node));
  }
  CT a_C = at_node(pl(AM_C), n);
  CT a_k1 = at_node(pl(PG_K1), n);
  if constexpr (CC) {
    const CT psi = at_node(pl(FW_PSI), n), C = at_node(pl(FW_C), n);
    const CT h = (psi + CT(1)) * CT(0.5);
    const CT k1 = K.k1;
    const CT m0 = CT(1) - k1 * h;
    const CT U = (C / m0 - CT(1)) / k1;
    a_C += a_U / (k1 * m0);
    a_psi += a_U * C / (CT(2) * m0 * m0);
    a_k1 += a_U * (C * h / (m0 * m0) - U) / k1;
  }
  // per-block partial sums of the parameter gradients (FP64, fixed order)
  {
    __shared__ double s_e[256], s_k[256], s_o[256];
    s_e[threadIdx.x] = live ? (double)at_node(pl(PG_EPS), n) : 0.0;
    s_k[threadIdx.x] = live ? (double)a_k1 : 0.0;
    // Omega through the far-field temperature (written by the reverse that handles far-field sides)
    s_o[threadIdx.x] = (live && P.far) ? (double)at_node(pl(PG_OM), n) : 0.0;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
      if (threadIdx.x < off) {
        s_e[threadIdx.x] += s_e[threadIdx.x + off];
        s_k[threadIdx.x] += s_k[threadIdx.x + off];
        s_o[threadIdx.x] += s_o[threadIdx.x + off];
      }
      __syncthreads();
    }
    // accumulate: a sweep over several steps adds each block's partials in
    // step order (each block owns its slots), summed once at the end
    if (threadIdx.x == 0) {
      double* pb = part + 3 * slot;
      pb[0] = (accumulate ? pb[0] : 0.0) + s_e[0];
      pb[1] = (accumulate ? pb[1] : 0.0) + s_k[0];
      pb[2] = (accumulate ? pb[2] : 0.0) + s_o[0];
    }
  }
  if (!live) return;
  auto put = [&](int plane, CT v) { at_node(S + (long long)plane * N, n) = v; };
  if constexpr (NS) { put(P_JX, am_jx); put(P_JY, am_jy); }
  if constexpr (PHI) put(P_PHI, a_phi);
  if constexpr (PSI) put(P_PSI, a_psi);
  if constexpr (CC) put(P_C, a_C);
  if constexpr (TH) put(P_H, at_node(pl(AM_H), n));
}

template <int FIELDS, int QP, class CT>
__global__ __launch_bounds__(256) void adj_assemble_kernel(const DevParams P, CT* __restrict__ S,
                                                           double* __restrict__ part, int accumulate) {
  const long long n0 = (long long)blockIdx.x * 256 + threadIdx.x;
  const bool live = n0 < P.N;
  const uint32_t n = (uint32_t)(live ? n0 : P.N - 1);
  const int x = (int)(n % (uint32_t)P.nx), y = (int)(n / (uint32_t)P.nx);
  assemble_node<FIELDS, QP, CT>(P, S, n, x, y, live, part, (int)blockIdx.x, accumulate, NoDelta{});
}

// R2 and R3 in one tile pass (flow with bubbles): the R2 increments of the
// tile and its ring are computed into LDS (a ring slot holds the node its
// coordinates map to: periodic wrap, or the mirror node across a wall,
// symmetry plane or far-field side, which is the node the transposed stencil
// reads), then R3 runs on the tile; the increments are never written.
template <class CT>
struct TileDelta {
  static constexpr bool active = true;
  const CT (*s)[TY + 2][TX + 2];
  int ly, lx;
  __device__ FlowDelta<CT> get(int yy, int xx) const {
    FlowDelta<CT> d;
    d.gx = s[0][yy][xx]; d.gy = s[1][yy][xx]; d.lap = s[2][yy][xx]; d.phi = s[3][yy][xx];
    d.psi = s[4][yy][xx]; d.jx = s[5][yy][xx]; d.jy = s[6][yy][xx];
    return d;
  }
  __device__ FlowDelta<CT> own() const { return get(ly + 1, lx + 1); }
  // the reader of direction i sits at x - c_i
  __device__ FlowDelta<CT> at(int i) const { return get(ly + 1 - Lat<9>::c[i][1], lx + 1 - Lat<9>::c[i][0]); }
};
template <int FIELDS, int QP, class CT>
__global__ __launch_bounds__(NT) void adj_flow_assemble_kernel(const DevParams P, CT* __restrict__ S,
                                                               double* __restrict__ part, int accumulate) {
  constexpr int RX = TX + 2, RY = TY + 2;
  __shared__ CT s_d[7][RY][RX];
  const int tid = threadIdx.x;
  const int gtx = (P.nx + TX - 1) / TX;
  const int lt = logical_tile(blockIdx.x, gtx * ((P.ny + TY - 1) / TY));
  const int bx0 = (lt % gtx) * TX, by0 = (lt / gtx) * TY;
  for (int k = tid; k < RX * RY; k += NT) {
    const int rx = k % RX, ry = k / RX;
    const int mx = map_coord(bx0 + rx - 1, P.nx, P.wall[0]), my = map_coord(by0 + ry - 1, P.ny, P.wall[1]);
    const FlowDelta<CT> d = flow_delta<CT>(P, S, (uint32_t)my * (uint32_t)P.nx + (uint32_t)mx, mx, my);
    s_d[0][ry][rx] = d.gx; s_d[1][ry][rx] = d.gy; s_d[2][ry][rx] = d.lap; s_d[3][ry][rx] = d.phi;
    s_d[4][ry][rx] = d.psi; s_d[5][ry][rx] = d.jx; s_d[6][ry][rx] = d.jy;
  }
  __syncthreads();
  const int lx = tid % TX, ly = tid / TX;
  const int x = bx0 + lx, y = by0 + ly;
  const bool live = x < P.nx && y < P.ny;
  const int xc = live ? x : 0, yc = live ? y : 0;
  const uint32_t n = (uint32_t)yc * (uint32_t)P.nx + (uint32_t)xc;
  TileDelta<CT> dl{(const CT(*)[RY][RX])s_d, ly, lx};
  assemble_node<FIELDS, QP, CT>(P, S, n, xc, yc, live, part, (int)blockIdx.x, accumulate, dl);
}

// Zeroes the planes of open moment terms (P_ and A_OLD): lambda^{n+1} is
// complete.
template <class CT>
__global__ __launch_bounds__(256) void adj_clear_pending_kernel(CT* __restrict__ S, long long N) {
  const long long n0 = (long long)blockIdx.x * 256 + threadIdx.x;
  if (n0 >= N) return;
#pragma unroll
  for (int k = A_OLD0; k < A_NPLANES; ++k) S[(long long)k * N + n0] = CT(0);
}

// ------------------------------------------------------------ broadcast
// Adds the moment terms R3 left in the P_ planes (and the old-value reads in
// A_OLD) to the populations of lambda^n: where a sweep ends.
template <int FIELDS, int QP, class CT>
__global__ __launch_bounds__(256) void adj_broadcast_kernel(const DevParams P, const CT* __restrict__ S,
                                                            CT* __restrict__ lam) {
  constexpr bool NS = FIELDS & F_NS, PHI = FIELDS & F_PHI, PSI = FIELDS & F_PSI;
  constexpr bool CC = FIELDS & F_C, TH = FIELDS & F_TH;
  using LN = Lat<9>;
  using LS = Lat<5>;
  const long long n0 = (long long)blockIdx.x * 256 + threadIdx.x;
  if (n0 >= P.N) return;
  const uint32_t n = (uint32_t)n0;
  const long long N = P.N;
  const int x = (int)(n % (uint32_t)P.nx), y = (int)(n / (uint32_t)P.nx);
  auto pl = [&](int k) -> const CT* { return S + (long long)k * N; };
  auto add = [&](int plane, CT v) { at_node(lam + (long long)plane * N, n) += v; };
  if constexpr (NS) {
    const CT ajx = at_node(pl(P_JX), n), ajy = at_node(pl(P_JY), n);
#pragma unroll
    for (int i = 0; i < 9; ++i) add(P.o_ns + i, CT(LN::c[i][0]) * ajx + CT(LN::c[i][1]) * ajy);
  }
  if constexpr (PHI) {
    const CT a_phi = at_node(pl(P_PHI), n);
#pragma unroll
    for (int i = 0; i < QP; ++i) add(P.o_phi + i, a_phi);
  }
  if constexpr (PSI) {
    const CT a_psi = at_node(pl(P_PSI), n);
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      CT v = a_psi;
      // the neighbour at x - c_i read this population as the old value of
      // its time-stretched store (none across a wall)
      int sx = x - LS::c[i][0], sy = y - LS::c[i][1];
      bool ok = true;
      if (sx < 0 || sx >= P.nx) { if (P.wall[0]) ok = false; else sx = sx < 0 ? sx + P.nx : sx - P.nx; }
      if (sy < 0 || sy >= P.ny) { if (P.wall[1]) ok = false; else sy = sy < 0 ? sy + P.ny : sy - P.ny; }
      if (ok) v += at_node(pl(A_OLD0 + i), (uint32_t)sy * (uint32_t)P.nx + (uint32_t)sx);
      add(P.o_psi + i, v);
    }
  }
  if constexpr (CC) {
    const CT a_C = at_node(pl(P_C), n);
#pragma unroll
    for (int i = 0; i < 5; ++i) add(P.o_c + i, a_C);
  }
  if constexpr (TH) {
    const CT aH = at_node(pl(P_H), n);
#pragma unroll
    for (int i = 0; i < 5; ++i) add(P.o_th + i, aH);
  }
}

// Step parameter gradients from the per-block partials of the assembly pass:
// 256 threads take fixed strided subsets, then a fixed-order tree; thread 0
// adds the eps4 sum to dparams[0], minus the k1 sum to dparams[1]
// (k = 1 - k1) and the Omega sum to dparams[2].  Deterministic.
__global__ __launch_bounds__(256) void adj_param_sum_kernel(int nblocks, const double* __restrict__ part,
                                                            double* __restrict__ dparams) {
  __shared__ double s_e[256], s_k[256], s_o[256];
  double e = 0.0, k = 0.0, o = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += 256) { e += part[3 * b]; k += part[3 * b + 1]; o += part[3 * b + 2]; }
  s_e[threadIdx.x] = e;
  s_k[threadIdx.x] = k;
  s_o[threadIdx.x] = o;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      s_e[threadIdx.x] += s_e[threadIdx.x + off];
      s_k[threadIdx.x] += s_k[threadIdx.x + off];
      s_o[threadIdx.x] += s_o[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) { dparams[0] += s_e[0]; dparams[1] -= s_k[0]; dparams[2] += s_o[0]; }
}

// Byte offset of the per-block partials in the scratch buffer, after the
// A_NPLANES planes of the compute type.
inline size_t part_offset(long long N, size_t elem) {
  return ((size_t)A_NPLANES * (size_t)N * elem + 255) & ~(size_t)255;
}

template <int FIELDS, int QP, class ST, class HT>
hipError_t adj_step_t(const DevParams& P, const void* fin, const void* hist, const void* tape_v,
                      const void* lam_in_v, void* lam_out_v, void* scratch, double* dparams, hipStream_t s,
                      const AdjOpts& o) {
  const long long N = P.N;
  const unsigned tiles = (unsigned)(((P.nx + TX - 1) / TX) * ((P.ny + TY - 1) / TY));
  const unsigned nb = (unsigned)((N + 255) / 256);
  constexpr bool FLOWX = (FIELDS & F_NS) && (FIELDS & F_PHI);
  // the reverse runs in the forward's compute type, which is also the type
  // of the adjoint state and of the scratch planes
  using RT = typename std::conditional<std::is_same<ST, double>::value, double, float>::type;
  const RT* lam_in = (const RT*)lam_in_v;
  RT* lam_out = (RT*)lam_out_v;
  RT* S = (RT*)scratch;
  double* part = (double*)((char*)scratch + part_offset(N, sizeof(RT)));
  const RT* tape = (const RT*)tape_v;
  hipError_t e = hipSuccess;
  if (o.step) {
    if (!o.pend_in) {
      hipLaunchKernelGGL((adj_clear_pending_kernel<RT>), dim3(nb), dim3(256), 0, s, S, N);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    // symmetry planes and far-field sides: a separate instantiation
    const bool sym = P.sym || P.far;
    if (tape && sym)
      hipLaunchKernelGGL((adj_local_kernel<FIELDS, QP, ST, HT, RT, true, true>), dim3(tiles), dim3(NT), 0, s, P,
                         (const typename Store<ST>::raw*)fin, (const HT*)hist, tape, lam_in, lam_out, S);
    else if (tape)
      hipLaunchKernelGGL((adj_local_kernel<FIELDS, QP, ST, HT, RT, true>), dim3(tiles), dim3(NT), 0, s, P,
                         (const typename Store<ST>::raw*)fin, (const HT*)hist, tape, lam_in, lam_out, S);
    else if (sym)
      hipLaunchKernelGGL((adj_local_kernel<FIELDS, QP, ST, HT, RT, false, true>), dim3(tiles), dim3(NT), 0, s, P,
                         (const typename Store<ST>::raw*)fin, (const HT*)hist, tape, lam_in, lam_out, S);
    else
      hipLaunchKernelGGL((adj_local_kernel<FIELDS, QP, ST, HT, RT, false>), dim3(tiles), dim3(NT), 0, s, P,
                         (const typename Store<ST>::raw*)fin, (const HT*)hist, tape, lam_in, lam_out, S);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if constexpr (FLOWX)   // R2 and R3 in one tile pass, partials per tile
      hipLaunchKernelGGL((adj_flow_assemble_kernel<FIELDS, QP, RT>), dim3(tiles), dim3(NT), 0, s, P, S, part,
                         o.accumulate ? 1 : 0);
    else
      hipLaunchKernelGGL((adj_assemble_kernel<FIELDS, QP, RT>), dim3(nb), dim3(256), 0, s, P, S, part,
                         o.accumulate ? 1 : 0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (!o.pend_out) {
    hipLaunchKernelGGL((adj_broadcast_kernel<FIELDS, QP, RT>), dim3(nb), dim3(256), 0, s, P, (const RT*)S,
                       lam_out);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (!o.sum) return hipSuccess;
  hipLaunchKernelGGL(adj_param_sum_kernel, dim3(1), dim3(256), 0, s, (int)(FLOWX ? tiles : nb), part, dparams);
  return hipGetLastError();
}

template <class ST, class HT>
hipError_t adj_dispatch(const DevParams& P, int fields, const void* fin, const void* hist, const void* tape,
                        const void* lam_in, void* lam_out, void* S, double* dparams, hipStream_t s,
                        const AdjOpts& o, bool& ok) {
  ok = true;
  const bool q9 = P.q_phi == 9;
  // the lattice of phi matters only where phi is evolved: one instantiation otherwise
#define PFL_ADJ(F)                                                                                        \
  case F:                                                                                                 \
    return (q9 && ((F) & F_PHI))                                                                          \
               ? adj_step_t<F, ((F) & F_PHI) ? 9 : 5, ST, HT>(P, fin, hist, tape, lam_in, lam_out, S,     \
                                                               dparams, s, o)                             \
               : adj_step_t<F, 5, ST, HT>(P, fin, hist, tape, lam_in, lam_out, S, dparams, s, o);
  switch (fields) {
    PFL_ADJ(F_NS | F_PHI | F_PSI | F_C | F_TH)
    PFL_ADJ(F_PSI | F_C)
    PFL_ADJ(F_PSI | F_C | F_TH)
    PFL_ADJ(F_NS | F_PHI)
    PFL_ADJ(F_PSI)
    PFL_ADJ(F_PHI | F_PSI | F_C | F_TH)
    PFL_ADJ(F_PHI)
    PFL_ADJ(F_NS | F_PSI | F_TH)
    PFL_ADJ(F_PSI | F_TH)
    default:
      ok = false;
      return hipSuccess;
  }
#undef PFL_ADJ
}

}  // namespace

}  // namespace pfl
