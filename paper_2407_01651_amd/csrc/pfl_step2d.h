// 2D step building blocks shared by the forward step and its adjoint: tile
// shape, pulls (general and 32-bit fast addressing), halo enumeration,
// isotropic D2Q9 stencils on an LDS tile, and the flow quantities of one
// tile position.
#pragma once
#include "pfl_util.h"

namespace pfl {

constexpr int TX = 32, TY = 8, NT = TX * TY;
// The step kernel's tile, one node per thread: with the flow and the bubble
// phase both active (two halo rings), 32 x 8 nodes, or 64 x 4 with 16-bit
// storage (a wave's row is then one whole 128-byte line; coupled 2048^2 FP16
// 17.6k -> 18.1k MLUPS, BF16 17.5k -> 17.9k); otherwise 32 x 4.  The shapes
// measured fastest: with one ring 32 x 4 against 32 x 2, 32 x 8, 32 x 16,
// 64 x 4 and 16 x 8; with two rings 32 x 8 against 32 x 4, 32 x 16 and
// 16 x 16.  FP32 and FP64 storage keep 32 x 8: FP32 at 64 x 4 was 1.6%
// faster but exceeded its error bound against FP64 on one variable-heat
// case (its compiled contraction and reassociation differ per instantiation).
template <int FIELDS, class ST>
struct StepTile {
  static constexpr bool FLOWX = (FIELDS & F_NS) && (FIELDS & F_PHI);
  static constexpr int X = (FLOWX && sizeof(typename Store<ST>::raw) == 2) ? 64 : 32;
  static constexpr int Y = FLOWX ? (X == 64 ? 4 : 8) : 4;
  static constexpr int N = X * Y;
  // Minimum waves per SIMD asked of the register allocator.  The FP32-compute
  // step without flow, bubble phase or heat needs 64 VGPRs but over 100 SGPRs,
  // which would hold it at 7 waves; asking for 8 moves a few SGPRs into VGPR
  // lanes (no scratch) and gives 8 (alloy FP32 step 43.4k -> 46.0k MLUPS on
  // 1024^2).  Larger kernels spill to scratch when pushed and get slower
  // (coupled FP16 at 5 instead of 4 waves: 17.6k -> 14.0k), so they keep
  // the default (1 = no minimum).
  template <class CT, bool SYM>
  static constexpr int waves() {
    if (SYM) return 1;
    if (sizeof(CT) == 4 && !(FIELDS & (F_NS | F_PHI | F_TH))) return 8;
    return 1;
  }
};

// Pull the pre-collision population deviations of one set at node (x, y), general
// addressing: periodic wrap, half-way bounce-back at a wall (the node's own
// opposite population), or specular reflection at a symmetry plane (the
// mirror node's population with the normal component reversed) on each axis.
// SYM: the grid has symmetry planes or far-field sides (a separate
// instantiation, so that grids without them carry none of that code).
template <int Q, class ST, class CT, bool SYM = false>
__device__ __forceinline__ void pull_general(const typename Store<ST>::raw* __restrict__ base,
                                             const DevParams& P, int x, int y, CT f[Q]) {
  using L = Lat<Q>;
  const long long N = P.N;
  AxisSrc ax, ay;
  axis_src(x, P.nx, P.wall[0], SYM && sym_side(P, 0, true), SYM && sym_side(P, 0, false), 1, ax);
  axis_src(y, P.ny, P.wall[1], SYM && sym_side(P, 1, true), SYM && sym_side(P, 1, false), P.nx, ay);
  const int m = SYM ? sym_touch(P, x, y, 0) : 0;
  const long long own = (long long)y * P.nx + x;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int cx = L::c[i][0] + 1, cy = L::c[i][1] + 1;
    const bool b = ax.wall[cx] || ay.wall[cy];
    const int j = SYM ? pulled_population<Q>(i, m) : i;
    const long long e = b ? (long long)L::opp[i] * N + own : (long long)j * N + own + ax.off[cx] + ay.off[cy];
    f[i] = Store<ST>::template ld<CT>(base + e);
  }
}

// Pull at an interior node: source x - c_i lies inside the domain.
template <int Q, class ST, class CT>
__device__ __forceinline__ void pull_fast(const typename Store<ST>::raw* __restrict__ base,
                                          const DevParams& P, uint32_t nbyte, CT f[Q]) {
  using L = Lat<Q>;
  constexpr uint32_t S = sizeof(typename Store<ST>::raw);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const uint32_t rel = ((uint32_t)i * (uint32_t)P.N - (uint32_t)(L::c[i][0] + L::c[i][1] * P.nx)) * S;
    f[i] = Store<ST>::template ld<CT>(at_byte<ST>(base, rel + nbyte));
  }
}

template <int Q, class ST, class CT, bool SYM = false>
__device__ __forceinline__ void pull(bool fast, const typename Store<ST>::raw* __restrict__ base,
                                     const DevParams& P, int x, int y, CT f[Q]) {
  if (fast) {
    const uint32_t nbyte = ((uint32_t)y * (uint32_t)P.nx + (uint32_t)x) * (uint32_t)sizeof(typename Store<ST>::raw);
    pull_fast<Q, ST, CT>(base, P, nbyte, f);
  } else {
    pull_general<Q, ST, CT, SYM>(base, P, x, y, f);
  }
}

// Halo position k (0 <= k < RX*RY - TW*TH) of an R-ring TW x TH tile: the R top
// rows, the R bottom rows, then the side columns.
template <int R, int TW, int TH>
__device__ __forceinline__ void halo_pos(int k, int& rx, int& ry) {
  constexpr int RX = TW + 2 * R, RY = TH + 2 * R;
  if (k < R * RX) { ry = k / RX; rx = k % RX; return; }
  k -= R * RX;
  if (k < R * RX) { ry = RY - R + k / RX; rx = k % RX; return; }
  k -= R * RX;
  ry = R + k / (2 * R);
  const int c = k % (2 * R);
  rx = c < R ? c : TW + c;
}

// Isotropic D2Q9 gradient and Laplacian from an LDS array.
template <class CT, int RX>
__device__ __forceinline__ void grad9(const CT (*s)[RX], int ry, int rx, CT& gx, CT& gy) {
  const CT e = s[ry][rx + 1], wv = s[ry][rx - 1], n = s[ry + 1][rx], so = s[ry - 1][rx];
  const CT ne = s[ry + 1][rx + 1], nw = s[ry + 1][rx - 1], sw = s[ry - 1][rx - 1], se = s[ry - 1][rx + 1];
  gx = CT(3) * (CT(1.0 / 9) * (e - wv) + CT(1.0 / 36) * ((ne - nw) + (se - sw)));
  gy = CT(3) * (CT(1.0 / 9) * (n - so) + CT(1.0 / 36) * ((ne + nw) - (sw + se)));
}
template <class CT, int RX>
__device__ __forceinline__ CT lap9(const CT (*s)[RX], int ry, int rx) {
  const CT c = s[ry][rx];
  const CT ax = (s[ry][rx + 1] - c) + (s[ry][rx - 1] - c) + (s[ry + 1][rx] - c) + (s[ry - 1][rx] - c);
  const CT dg = (s[ry + 1][rx + 1] - c) + (s[ry + 1][rx - 1] - c) + (s[ry - 1][rx - 1] - c) + (s[ry - 1][rx + 1] - c);
  return CT(6) * (CT(1.0 / 9) * ax + CT(1.0 / 36) * dg);
}

// Flow quantities at one LDS position (node or ring 1): chemical potential,
// surface tension, phi diffusion flux, velocity without the mass-flux force.
template <class CT>
struct FlowNode {
  CT gx, gy, lap, nx, ny, Fsx, Fsy, Dx, Dy, rho, chi, v0x, v0y, sharp;
};

// The flow quantities from the node's phi, psi, momentum and the phi stencils.
template <bool NS, class CT>
__device__ __forceinline__ void flow_node_from(const KP<CT>& K, CT phi, CT psi, CT jx, CT jy, CT gx, CT gy, CT lap,
                                               FlowNode<CT>& o) {
  o.gx = gx;
  o.gy = gy;
  o.lap = lap;
  // unit normal, regularised where the gradient vanishes
  const CT inv = rsq(o.gx * o.gx + o.gy * o.gy + K.dn);
  o.nx = o.gx * inv;
  o.ny = o.gy * inv;
  // phi_l = 1, phi_g = 0, psi_l = -1, beta_phi = 1/4
  const CT one_m = CT(1) - phi;
  // double-well factor of the sharpening flux, zero outside [phi_g, phi_l]
  const CT dw = one_m * phi;
  o.sharp = K.sharp * (dw > CT(0) ? dw : CT(0));
  o.Dx = K.M_phi * (o.gx - o.sharp * o.nx);
  o.Dy = K.M_phi * (o.gy - o.sharp * o.ny);
  const CT h = (psi + CT(1)) * CT(0.5);
  o.chi = clamp01(h);
  o.rho = K.rho_g + K.drho * phi;
  if constexpr (NS) {
    const CT f1p = CT(0.5) * one_m * phi * (CT(1) - CT(2) * phi);
    const CT ps1 = psi + CT(1);
    const CT f3p = CT(-2) * K.beta_inter * one_m * ps1 * ps1;
    const CT mu = f1p + f3p - K.Wphi2 * o.lap;
    o.Fsx = K.k_s * mu * o.gx;
    o.Fsy = K.k_s * mu * o.gy;
    // buoyancy relative to the liquid: its hydrostatic head is carried by p
    const CT Fbx = CT(0), Fby = -(o.rho - K.rho_l) * K.g;
    const CT s = (CT(1) - o.chi) * rcp(o.rho);
    o.v0x = s * (jx + CT(0.5) * (o.Fsx + Fbx));
    o.v0y = s * (jy + CT(0.5) * (o.Fsy + Fby));
  } else {
    o.Fsx = o.Fsy = o.v0x = o.v0y = CT(0);
  }
}

template <bool NS, bool PHI, class CT, int RX, class JA>
__device__ __forceinline__ void flow_node(const KP<CT>& K, const CT (*s_phi)[RX], const CT (*s_psi)[RX],
                                          const JA& s_jx, const JA& s_jy, int ry, int rx, FlowNode<CT>& o) {
  CT gx = CT(0), gy = CT(0), lap = CT(0);
  if constexpr (PHI) {
    grad9<CT, RX>(s_phi, ry, rx, gx, gy);
    lap = lap9<CT, RX>(s_phi, ry, rx);
  }
  CT jx = CT(0), jy = CT(0);
  if constexpr (NS) {
    jx = s_jx[ry][rx];
    jy = s_jy[ry][rx];
  }
  flow_node_from<NS, CT>(K, s_phi[ry][rx], s_psi[ry][rx], jx, jy, gx, gy, lap, o);
}

}  // namespace pfl
