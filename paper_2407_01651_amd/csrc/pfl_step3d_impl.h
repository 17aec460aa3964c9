// Fused 3D time step: D3Q19 flow, D3Q7 bubble phase, order parameter, solute
// and heat, advanced by one step in one launch.  The scheme is the 2D step's
// with the 3D lattices: isotropic D3Q19 stencils (Appendix B), the cubic
// anisotropy with the crystal rotated about z (Sec. 3.3), the D3Q19 MRT
// collision relaxing the five traceless stress moments, D3Q7 collisions
// relaxing the three flux moments.
//
// Work decomposition (2.5-D): a workgroup owns a TX x TY column of nodes, one
// node per thread, and marches it through a chunk of z planes.  The stencil
// inputs live in LDS rings of planes, each plane loaded once per chunk: phi on
// the tile plus two rings in x and y over four planes (the mass-flux force
// needs D_phi (x) v0 one node out in every direction, and D_phi needs grad
// phi there) when flow and bubble phase are both active, otherwise one ring
// over three planes; psi and U on the tile plus one ring over three planes;
// the momentum on the tile plus one ring for the plane whose D_phi and v0 are
// being formed; D_phi and v0 on the tile plus one ring over three planes.  At
// plane t the workgroup loads phi at t + 2 (t + 1 without the mass-flux
// force) and psi, U, momentum at t + 1, forms D_phi and v0 at t + 1, and
// then steps its own nodes of plane t, pulling their populations again (the
// pulls of plane t + 1 one iteration before are still in the L2).
//
// Storage is the 2D step's: SoA planes (x fastest, then y, then z), pull
// form, half-way bounce-back from the node's own opposite slot, FP32/16-bit
// planes holding deviations from the bulk rest state.  Each plane is
// addressed from a 64-bit plane base plus a 32-bit in-plane byte offset, so
// population buffers beyond 4 GiB (256^3 in FP64) keep the cheap addressing.
#pragma once
#include "pfl_kernels.h"
#include "pfl_util.h"

namespace pfl {

namespace {

// Column tile: 32 x 8 nodes, 256 threads (rows of 32 nodes keep each wave's
// loads and stores in whole or half 128-byte lines).  FP64 runs one wave per
// SIMD either way; against 32 x 4 the taller column spreads the ring pulls
// over more nodes (coupled 256^3 FP64 2.65k -> 2.75k MLUPS) and fits the
// LDS (55 KB).
template <class CT>
struct Col3 {
  static constexpr int TX = 32, TY = sizeof(CT) == 8 ? 8 : 16;
  static constexpr int NT = TX * TY;
};

// One LDS plane of the tile plus R rings in x and y.
template <class CT, int R>
struct Pl {
  static constexpr int X = Col3<CT>::TX + 2 * R, Y = Col3<CT>::TY + 2 * R;
  static constexpr int N = X * Y;
  __device__ static constexpr int at(int y, int x) { return y * X + x; }
};

// Ring slot of plane p among n slots.
__device__ __forceinline__ int ring_slot(int p, int n) {
  const int s = p % n;
  return s < 0 ? s + n : s;
}

// Pull the stored values of one set at node (x, y, z), general addressing:
// periodic wrap, half-way bounce-back at a wall or specular reflection at a
// symmetry plane on each axis, from per-axis source offsets computed once
// per node.
template <int Q, class ST, class CT, bool SYM>
__device__ __forceinline__ void pull3_general(const typename Store<ST>::raw* __restrict__ base,
                                              const DevParams& P, int x, int y, int z, CT f[Q]) {
  using L = Lat<Q>;
  AxisSrc ax, ay, az;
  axis_src(x, P.nx, P.wall[0], SYM && sym_side(P, 0, true), SYM && sym_side(P, 0, false), 1, ax);
  axis_src(y, P.ny, P.wall[1], SYM && sym_side(P, 1, true), SYM && sym_side(P, 1, false), P.nx, ay);
  axis_src(z, P.nz, P.wall[2], SYM && sym_side(P, 2, true), SYM && sym_side(P, 2, false), P.nx * P.ny, az);
  const int m = SYM ? sym_touch(P, x, y, z) : 0;
  const long long own = ((long long)z * P.ny + y) * P.nx + x;
  const long long N = P.N;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int cx = L::c[i][0] + 1, cy = L::c[i][1] + 1, cz = L::c[i][2] + 1;
    const bool b = ax.wall[cx] || ay.wall[cy] || az.wall[cz];
    const int j = SYM ? pulled_population<Q>(i, m) : i;
    const long long e = b ? (long long)L::opp[i] * N + own
                          : (long long)j * N + (own + ax.off[cx] + ay.off[cy] + az.off[cz]);
    f[i] = Store<ST>::template ld<CT>(base + e);
  }
}

// Pull at a node whose sources x - c_i all lie inside the domain: a 64-bit
// plane base per population and one 32-bit in-plane byte offset (the source
// node's offset is non-negative and below N S < 2^32).
template <int Q, class ST, class CT>
__device__ __forceinline__ void pull3_fast(const typename Store<ST>::raw* __restrict__ base,
                                           const DevParams& P, uint32_t nbyte, CT f[Q]) {
  using L = Lat<Q>;
  constexpr uint32_t S = sizeof(typename Store<ST>::raw);
  const uint32_t sxy = (uint32_t)P.nx * (uint32_t)P.ny;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const uint32_t shift = ((uint32_t)L::c[i][0] + (uint32_t)L::c[i][1] * (uint32_t)P.nx +
                            (uint32_t)L::c[i][2] * sxy) * S;
    f[i] = Store<ST>::template ld<CT>(at_byte<ST>(base + (size_t)i * (size_t)P.N, nbyte - shift));
  }
}

template <int Q, class ST, class CT, bool SYM>
__device__ __forceinline__ void pull3(bool fast, const typename Store<ST>::raw* __restrict__ base,
                                      const DevParams& P, int x, int y, int z, CT f[Q]) {
  if (fast) {
    const uint32_t nbyte = (uint32_t)((z * P.ny + y) * P.nx + x) * (uint32_t)sizeof(typename Store<ST>::raw);
    pull3_fast<Q, ST, CT>(base, P, nbyte, f);
  } else {
    pull3_general<Q, ST, CT, SYM>(base, P, x, y, z, f);
  }
}

// Isotropic D3Q19 gradient (1/cs2) sum_i w_i c_i f(x + c_i) and Laplacian
// (2/cs2) sum_i w_i [f(x + c_i) - f(x)] from three LDS planes (below, at,
// above the node), (y, x) in the plane geometry PL.
template <class CT, class PL>
__device__ __forceinline__ void grad19p(const CT* const pl[3], int y, int x, CT g[3]) {
  using L = Lat<19>;
  CT a0 = CT(0), a1 = CT(0), a2 = CT(0);
#pragma unroll
  for (int i = 1; i < 19; ++i) {
    const CT v = CT(L::w[i]) * pl[L::c[i][2] + 1][PL::at(y + L::c[i][1], x + L::c[i][0])];
    if (L::c[i][0]) a0 += CT(L::c[i][0]) * v;
    if (L::c[i][1]) a1 += CT(L::c[i][1]) * v;
    if (L::c[i][2]) a2 += CT(L::c[i][2]) * v;
  }
  g[0] = CT(3) * a0;
  g[1] = CT(3) * a1;
  g[2] = CT(3) * a2;
}
template <class CT, class PL>
__device__ __forceinline__ CT lap19p(const CT* const pl[3], int y, int x) {
  using L = Lat<19>;
  const CT c = pl[1][PL::at(y, x)];
  CT a = CT(0);
#pragma unroll
  for (int i = 1; i < 19; ++i) a += CT(L::w[i]) * (pl[L::c[i][2] + 1][PL::at(y + L::c[i][1], x + L::c[i][0])] - c);
  return CT(6) * a;
}

template <class CT>
struct FlowNode3 {
  CT g[3], lap, n[3], Fs[3], D[3], rho, chi, v0[3], sharp;
};

// Flow quantities at one LDS position of a plane (node or ring 1); (y, x) in
// ring-1 plane coordinates; ph: the phi planes below, at and above; ps: psi
// of the plane; sj: momentum of the plane (null: v0 not formed).
template <bool NS, bool PHI, int R, class CT>
__device__ __forceinline__ void flow_node3(const KP<CT>& K, const CT* const ph[3], const CT* ps, const CT* sj,
                                           int y, int x, FlowNode3<CT>& o) {
  using PR = Pl<CT, R>;
  using P1 = Pl<CT, 1>;
  constexpr int d = R - 1;
  const CT phi = ph[1][PR::at(y + d, x + d)];
  const CT psi = ps[P1::at(y, x)];
  if constexpr (PHI) {
    grad19p<CT, PR>(ph, y + d, x + d, o.g);
    o.lap = lap19p<CT, PR>(ph, y + d, x + d);
  } else {
    o.g[0] = o.g[1] = o.g[2] = o.lap = CT(0);
  }
  const CT inv = rsq(o.g[0] * o.g[0] + o.g[1] * o.g[1] + o.g[2] * o.g[2] + K.dn);
  const CT one_m = CT(1) - phi;
  const CT dw = one_m * phi;
  o.sharp = K.sharp * (dw > CT(0) ? dw : CT(0));
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    o.n[a] = o.g[a] * inv;
    o.D[a] = K.M_phi * (o.g[a] - o.sharp * o.n[a]);
  }
  const CT h = (psi + CT(1)) * CT(0.5);
  o.chi = clamp01(h);
  o.rho = K.rho_g + K.drho * phi;
  if constexpr (NS) {
    const CT f1p = CT(0.5) * one_m * phi * (CT(1) - CT(2) * phi);
    const CT ps1 = psi + CT(1);
    const CT f3p = CT(-2) * K.beta_inter * one_m * ps1 * ps1;
    const CT mu = f1p + f3p - K.Wphi2 * o.lap;
    const CT s = (CT(1) - o.chi) * rcp(o.rho);
    const CT Fb[3] = {CT(0), -(o.rho - K.rho_l) * K.g, CT(0)};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      o.Fs[a] = K.k_s * mu * o.g[a];
      o.v0[a] = sj ? s * (sj[a * P1::N + P1::at(y, x)] + CT(0.5) * (o.Fs[a] + Fb[a])) : CT(0);
    }
  } else {
#pragma unroll
    for (int a = 0; a < 3; ++a) o.Fs[a] = o.v0[a] = CT(0);
  }
}

template <int FIELDS, class ST, class HT, class CT, bool SYM, bool STREAM>
// FP32 compute: two waves per SIMD (256 threads per workgroup)
__global__ __launch_bounds__(Col3<CT>::NT, 1) void step3d_kernel(const DevParams P,
                                                               const typename Store<ST>::raw* __restrict__ fin,
                                                               typename Store<ST>::raw* __restrict__ fout,
                                                               HT* hist, double* __restrict__ mout,
                                                               int mode) {
  constexpr bool NS = FIELDS & F_NS, PHI = FIELDS & F_PHI, PSI = FIELDS & F_PSI;
  constexpr bool CC = FIELDS & F_C, TH = FIELDS & F_TH;
  constexpr bool FLOWX = NS && PHI;
  constexpr int R = FLOWX ? 2 : 1;
  constexpr int TX = Col3<CT>::TX, TY = Col3<CT>::TY, NT = Col3<CT>::NT;
  using PR = Pl<CT, R>;
  using P1 = Pl<CT, 1>;
  // LDS plane slots.  Phase C of plane t reads the phi, psi and U planes t - 1,
  // t, t + 1; phase A of plane t + 1, which a thread may reach while others
  // are still in that phase C (no barrier between them), writes phi at
  // t + 1 + (FLOWX ? 2 : 1) and psi, U at t + 2: with these slot counts those
  // land on planes nobody reads then.
  constexpr int NPH = FLOWX ? 5 : 4;       // phi plane slots
  constexpr int NPS = 4;                   // psi and U plane slots
  constexpr int QN = 19, QS = 7, QP = 7;
  using LN = Lat<19>;
  using LS = Lat<7>;
  using LP = Lat<7>;
  using raw = typename Store<ST>::raw;
  constexpr uint32_t S = sizeof(raw), HS = sizeof(HT);
  const KP<CT>& K = kp<CT>(P);

  __shared__ CT s_phi[NPH * PR::N];
  __shared__ CT s_psi[NPS * P1::N];
  __shared__ CT s_U[CC ? NPS * P1::N : 1];
  __shared__ CT s_j[NS ? 3 * P1::N : 1];
  // D_phi and v0 of the plane formed last, tile + ring 1: [component][position]
  __shared__ CT s_D[FLOWX ? 3 * P1::N : 1];
  __shared__ CT s_v0[FLOWX ? 3 * P1::N : 1];

  const int tid = threadIdx.x;
  const int lx = tid % TX, ly = tid / TX;
  const int gtx = (P.nx + TX - 1) / TX, gty = (P.ny + TY - 1) / TY;
  const int zc = P.zc, nch = (P.nz + zc - 1) / zc;
  const int lt = logical_tile(blockIdx.x, gtx * gty * nch);
  const int bx0 = (lt % gtx) * TX, by0 = ((lt / gtx) % gty) * TY;
  const int z0 = (lt / (gtx * gty)) * zc;
  const int z1 = z0 + zc < P.nz ? z0 + zc : P.nz;
  const int x = bx0 + lx, y = by0 + ly;
  const bool own_xy = x < P.nx && y < P.ny;
  const long long N = P.N;
  // pulls of every position the tile loads stay inside the domain in x and
  // y; at plane p they stay inside in z when 1 <= p <= nz - 2
  const bool fast_xy = P.plane32 && bx0 >= R + 1 && by0 >= R + 1 && bx0 + TX + R + 1 <= P.nx &&
                       by0 + TY + R + 1 <= P.ny;
  auto fast_at = [&](int p) -> bool { return fast_xy && p >= 1 && p + 2 <= P.nz; };
  const bool zwall = P.wall[2] != 0;

  const raw* fin_ns = fin + (size_t)(NS ? P.o_ns : 0) * (size_t)N;
  const raw* fin_phi = fin + (size_t)(PHI ? P.o_phi : 0) * (size_t)N;
  const raw* fin_psi = fin + (size_t)(PSI ? P.o_psi : 0) * (size_t)N;
  const raw* fin_c = fin + (size_t)(CC ? P.o_c : 0) * (size_t)N;
  const raw* fin_th = fin + (size_t)(TH ? P.o_th : 0) * (size_t)N;
  const CT k1 = K.k1;
  constexpr bool DEV = !std::is_same<ST, double>::value;
  const CT r_phi = DEV ? CT(1) : CT(0), r_psi = DEV ? CT(-1) : CT(0);
  const CT r_C = DEV ? K.C_ref : CT(0), r_H = DEV ? K.theta0 : CT(0);
  const bool first = P.first != 0;

  // FP64 and FP32 storage with flow and bubble phase: a thread keeps the
  // flow, psi and C populations it pulls for its own node in phase A, for the
  // plane's phase C one step later (two planes in registers), so that phase C
  // pulls only phi and theta.  The FP64 kernel runs one wave per SIMD with
  // room to spare, the FP32 one still fits two (256^3 FP64 2.55k -> 2.65k,
  // FP32 6.03k -> 6.42k MLUPS); with 16-bit storage the kept values spill
  // (FP16 6.34k -> 6.18k), and the other field combinations would lose a
  // wave per SIMD.
  constexpr bool KEEP = FLOWX && sizeof(raw) >= 4;
  // FP64 storage (one wave per SIMD, registers to spare) also keeps the own
  // node's phi populations; phase A pulls phi two planes ahead, so three
  // planes are held: kph0 for this step's phase C (plane t), kph1 (t + 1),
  // kph2 (t + 2, pulled in this step's phase A)
  constexpr bool KEEPPHI = KEEP && PHI && sizeof(raw) == 8;
  constexpr int KP = KEEPPHI ? QP : 1;
  CT kph0[KP], kph1[KP], kph2[KP];
  auto rot_phi = [&]() {
    if constexpr (KEEPPHI) {
#pragma unroll
      for (int i = 0; i < KP; ++i) { kph0[i] = kph1[i]; kph1[i] = kph2[i]; }
    }
  };
  // ---- phase A: phi of plane p on the tile and R rings
  auto load_phi = [&](int p) {
    const bool fast = fast_at(p);
    CT* dst = s_phi + ring_slot(p, NPH) * PR::N;
    auto one = [&](int k, bool keep) {
      const int tx = k % PR::X - R, ty = k / PR::X - R;
      int gx = bx0 + tx, gy = by0 + ty, gz = p;
      if (!fast) {
        gx = map_coord(gx, P.nx, P.wall[0]);
        gy = map_coord(gy, P.ny, P.wall[1]);
        gz = map_coord(gz, P.nz, P.wall[2]);
      }
      CT hphi = CT(1);
      if constexpr (PHI) {
        CT f[QP];
        pull3<QP, ST, CT, SYM>(fast, fin_phi, P, gx, gy, gz, f);
        CT d = CT(0);
#pragma unroll
        for (int i = 0; i < QP; ++i) d += f[i];
        hphi = r_phi + d;
        if constexpr (KEEPPHI) {
          if (keep) {
#pragma unroll
            for (int i = 0; i < QP; ++i) kph2[i] = f[i];
          }
        }
      }
      dst[k] = hphi;
    };
    if constexpr (KEEPPHI) {
      // the own interior position first, then the ring positions (the R top
      // rows, the R bottom rows, then the side columns), those on the last
      // threads as below
      constexpr int NPASS = 1 + (PR::N - NT + NT - 1) / NT;
#pragma unroll 1
      for (int it = 0; it < NPASS; ++it) {
        int k;
        if (it == 0) {
          k = PR::at(ly + R, lx + R);
        } else {
          const int r = (it - 1) * NT + (NT - 1 - tid);
          if (r >= PR::N - NT) continue;
          if (r < R * PR::X) {
            k = r;
          } else if (r < 2 * R * PR::X) {
            k = (PR::Y - R) * PR::X + (r - R * PR::X);
          } else {
            const int q = r - 2 * R * PR::X, c = q % (2 * R);
            k = (R + q / (2 * R)) * PR::X + (c < R ? c : PR::X - 2 * R + c);
          }
        }
        one(k, it == 0);
      }
    } else if constexpr (KEEP) {
      // positions beyond the first NT go to the last threads (the first ones
      // take the extra ring positions of load_rest), so no wave does both
      // (A/B on one box: 256^3 FP64 2.82k -> 2.88k, FP32 7.31k -> 7.39k
      // MLUPS; the kernels without kept populations measured slower with
      // this loop and keep the plain one)
      constexpr int NPASS = (PR::N + NT - 1) / NT;
#pragma unroll 1
      for (int it = 0; it < NPASS; ++it) {
        const int k = it == 0 ? tid : it * NT + (NT - 1 - tid);
        if (k < PR::N) one(k, false);
      }
    } else {
      for (int k = tid; k < PR::N; k += NT) {
        const int tx = k % PR::X - R, ty = k / PR::X - R;
        int gx = bx0 + tx, gy = by0 + ty, gz = p;
        if (!fast) {
          gx = map_coord(gx, P.nx, P.wall[0]);
          gy = map_coord(gy, P.ny, P.wall[1]);
          gz = map_coord(gz, P.nz, P.wall[2]);
        }
        CT hphi = CT(1);
        if constexpr (PHI) {
          CT f[QP];
          pull3<QP, ST, CT, SYM>(fast, fin_phi, P, gx, gy, gz, f);
          CT d = CT(0);
#pragma unroll
          for (int i = 0; i < QP; ++i) d += f[i];
          hphi = r_phi + d;
        }
        dst[k] = hphi;
      }
    }
  };
  constexpr int KN = KEEP && NS ? QN : 1, KS = KEEP && PSI ? QS : 1, KC = KEEP && CC ? QS : 1;
  CT kA_ns[KN], kA_ps[KS], kA_c[KC];       // plane t (phase C of this step)
  CT kB_ns[KN], kB_ps[KS], kB_c[KC];       // plane t + 1 (pulled in this step's phase A)
  // FP16 storage keeps the flow populations only, as their stored bits two to
  // a register (252 VGPRs, no scratch; 256^3 FP16 7.17k -> 7.35k MLUPS, A/B
  // on one box; BF16 measured slower with it, 6.71k -> 6.37k, and pulls)
  constexpr bool KEEP16 = FLOWX && std::is_same<ST, half_dev>::value;
  constexpr bool OWN1 = KEEP || KEEP16;     // load_rest takes the own position first
  constexpr int KW = KEEP16 ? (QN + 1) / 2 : 1;
  uint32_t kA16[KW], kB16[KW];
  // ---- phase A: psi, U and the momentum of plane p on the tile and one ring
  auto load_rest = [&](int p) {
    const bool fast = fast_at(p);
    CT* dpsi_ = s_psi + ring_slot(p, NPS) * P1::N;
    CT* dU = s_U + (CC ? ring_slot(p, NPS) * P1::N : 0);
    // KEEP: the own interior position first, then the ring positions
    // (top row, bottom row, then the two side columns)
    constexpr int NPOS = OWN1 ? 1 + (P1::N - NT + NT - 1) / NT : (P1::N + NT - 1) / NT;
#pragma unroll 1
    for (int it = 0; it < NPOS; ++it) {
      int k;
      const bool keep = OWN1 && it == 0;
      if constexpr (OWN1) {
        if (it == 0) {
          k = P1::at(ly + 1, lx + 1);
        } else {
          const int r = tid + (it - 1) * NT;
          if (r >= P1::N - NT) break;
          if (r < P1::X) k = r;
          else if (r < 2 * P1::X) k = (P1::Y - 1) * P1::X + (r - P1::X);
          else k = (1 + (r - 2 * P1::X) / 2) * P1::X + ((r - 2 * P1::X) % 2 ? P1::X - 1 : 0);
        }
      } else {
        k = tid + it * NT;
        if (k >= P1::N) break;
      }
      const int tx = k % P1::X - 1, ty = k / P1::X - 1;
      const int gx0 = bx0 + tx, gy0 = by0 + ty;
      int gx = gx0, gy = gy0, gz = p;
      if (!fast) {
        gx = map_coord(gx, P.nx, P.wall[0]);
        gy = map_coord(gy, P.ny, P.wall[1]);
        gz = map_coord(gz, P.nz, P.wall[2]);
      }
      CT hpsi = CT(-1), hU = K.U0, hj[3] = {CT(0), CT(0), CT(0)};
      if constexpr (PSI) {
        CT f[QS];
        pull3<QS, ST, CT, SYM>(fast, fin_psi, P, gx, gy, gz, f);
        CT d = CT(0);
#pragma unroll
        for (int i = 0; i < QS; ++i) d += f[i];
        hpsi = r_psi + d;
        if constexpr (KEEP) {
          if (keep) {
#pragma unroll
            for (int i = 0; i < QS; ++i) kB_ps[i] = f[i];
          }
        }
      }
      if constexpr (CC) {
        CT f[QS];
        pull3<QS, ST, CT, SYM>(fast, fin_c, P, gx, gy, gz, f);
        CT d = CT(0);
#pragma unroll
        for (int i = 0; i < QS; ++i) d += f[i];
        if constexpr (KEEP) {
          if (keep) {
#pragma unroll
            for (int i = 0; i < QS; ++i) kB_c[i] = f[i];
          }
        }
        const CT hC = r_C + d;
        const CT h = (hpsi + CT(1)) * CT(0.5);
        hU = (hC * rcp(CT(1) - k1 * h) - CT(1)) * K.inv_k1;
      }
      if constexpr (NS) {
        CT f[QN];
        pull3<QN, ST, CT, SYM>(fast, fin_ns, P, gx, gy, gz, f);
#pragma unroll
        for (int i = 0; i < QN; ++i) {
          if (LN::c[i][0]) hj[0] += CT(LN::c[i][0]) * f[i];
          if (LN::c[i][1]) hj[1] += CT(LN::c[i][1]) * f[i];
          if (LN::c[i][2]) hj[2] += CT(LN::c[i][2]) * f[i];
        }
        if constexpr (KEEP) {
          if (keep) {
#pragma unroll
            for (int i = 0; i < QN; ++i) kB_ns[i] = f[i];
          }
        }
        if constexpr (KEEP16) {
          if (keep) {
#pragma unroll
            for (int w = 0; w < KW; ++w)
              kB16[w] = keep16<ST>(f[2 * w], 2 * w + 1 < QN ? f[2 * w + 1] : CT(0));
          }
        }
      }
      if (SYM && !fast && P.far) {
        // ghost across an odd number of far-field sides: psi and U odd about
        // psi_l = -1 and U = 0 (each crossing mirrors once)
        const bool fx = gx0 < 0 ? far_side(P, 0, true) : gx0 >= P.nx && far_side(P, 0, false);
        const bool fy = gy0 < 0 ? far_side(P, 1, true) : gy0 >= P.ny && far_side(P, 1, false);
        const bool fz = p < 0 ? far_side(P, 2, true) : p >= P.nz && far_side(P, 2, false);
        if (fx ^ fy ^ fz) {
          hpsi = CT(-2) - hpsi;
          hU = -hU;
        }
      }
      dpsi_[k] = hpsi;
      if constexpr (CC) dU[k] = hU;
      if constexpr (NS) {
#pragma unroll
        for (int a = 0; a < 3; ++a) s_j[a * P1::N + k] = hj[a];
      }
    }
  };
  // LDS planes of phi around plane p
  auto phi_planes = [&](int p, const CT* pl[3]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) pl[c] = s_phi + ring_slot(p - 1 + c, NPH) * PR::N;
  };
  // ---- phase B: D_phi and v0 of plane q on the tile and ring 1, from the
  // flow quantities at plane m (q itself, or the plane q mirrors across a
  // wall or symmetry plane in z; flip_z: q is such a ghost plane).  Ghosts
  // across a wall: D (x) v0 is odd across the wall; D takes minus the value
  // at the mirror node once per wall crossed, v0 the value.  Across a
  // symmetry plane the ghost is the mirror image: the normal components of D
  // and v0 change sign.
  auto form_dv = [&](int q, int m, bool flip_z) {
    const CT* ph[3];
    phi_planes(m, ph);
    const CT* ps = s_psi + ring_slot(m, NPS) * P1::N;
    CT* dD = s_D;
    CT* dv = s_v0;
    for (int k = tid; k < P1::N; k += NT) {
      const int rx = k % P1::X, ry = k / P1::X;
      const int g[2] = {bx0 + rx - 1, by0 + ry - 1};
      int mm[2] = {rx, ry};
      const int n[2] = {P.nx, P.ny};
      CT sgn = CT(1), sc[3] = {CT(1), CT(1), CT(1)};
      bool skip = false;
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        if (P.wall[a] && (g[a] < 0 || g[a] >= n[a])) {
          if (g[a] == -1) mm[a] += 1; else if (g[a] == n[a]) mm[a] -= 1; else skip = true;
          if (SYM && sym_side(P, a, g[a] < 0)) sc[a] = -sc[a]; else sgn = -sgn;
        }
      }
      if (flip_z) {
        if (SYM && sym_side(P, 2, q < 0)) sc[2] = -sc[2]; else sgn = -sgn;
      }
      CT D[3] = {CT(0), CT(0), CT(0)}, v0[3] = {CT(0), CT(0), CT(0)};
      if (!skip) {
        FlowNode3<CT> hn;
        flow_node3<NS, PHI, R, CT>(K, ph, ps, s_j, mm[1], mm[0], hn);
#pragma unroll
        for (int a = 0; a < 3; ++a) { D[a] = sgn * sc[a] * hn.D[a]; v0[a] = sc[a] * hn.v0[a]; }
      }
#pragma unroll
      for (int a = 0; a < 3; ++a) { dD[a * P1::N + k] = D[a]; dv[a * P1::N + k] = v0[a]; }
    }
  };

  // The mass-flux force of the own node at plane z is the divergence
  // (1/cs2) sum_i w_i (c_i . D(x + c_i)) v0(x + c_i) over the planes z - 1, z,
  // z + 1.  Each plane's D and v0 are in LDS once, right after they are
  // formed; the own thread then adds that plane's terms to the sums of the
  // nodes below (c_i,z = +1), at (c_i,z = 0) and above it (c_i,z = -1):
  // div_part returns the three groups.
  auto div_part = [&](CT (&up)[3], CT (&mid)[3], CT (&dn)[3]) {
#pragma unroll
    for (int b = 0; b < 3; ++b) up[b] = mid[b] = dn[b] = CT(0);
#pragma unroll
    for (int i = 1; i < QN; ++i) {
      const int q1 = P1::at(ly + 1 + LN::c[i][1], lx + 1 + LN::c[i][0]);
      CT cD = CT(0);
      if (LN::c[i][0]) cD += CT(LN::c[i][0]) * s_D[q1];
      if (LN::c[i][1]) cD += CT(LN::c[i][1]) * s_D[P1::N + q1];
      if (LN::c[i][2]) cD += CT(LN::c[i][2]) * s_D[2 * P1::N + q1];
      const CT wc = CT(LN::w[i]) * cD;
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        const CT term = wc * s_v0[b * P1::N + q1];
        if (LN::c[i][2] > 0) up[b] += term;
        else if (LN::c[i][2] < 0) dn[b] += term;
        else mid[b] += term;
      }
    }
  };
  // running sums for the own node at planes t and t + 1
  CT dv_t[3] = {CT(0), CT(0), CT(0)}, dv_t1[3] = {CT(0), CT(0), CT(0)};

  // phi planes z0 - 2, z0 - 1 before the march when phi runs two planes ahead
  if constexpr (FLOWX) {
    load_phi(z0 - 2);
    rot_phi();
    load_phi(z0 - 1);
    rot_phi();
  }
  for (int t = z0 - 2; t < z1; ++t) {
    load_phi(t + (FLOWX ? 2 : 1));
    load_rest(t + 1);
    __syncthreads();
    CT dv_t2[3] = {CT(0), CT(0), CT(0)};     // the own node at plane t + 2
    if constexpr (FLOWX) {
      const int q = t + 1;
      CT up[3], mid[3], dn[3];
      if (zwall && q == 0) {
        // the ghost plane -1 (plane t): its terms reach plane t + 1 = 0
        form_dv(-1, 0, true);
        __syncthreads();
        if (own_xy) {
          div_part(up, mid, dn);
#pragma unroll
          for (int b = 0; b < 3; ++b) dv_t1[b] += dn[b];
        }
        __syncthreads();
      }
      if (!zwall || (q >= 0 && q < P.nz)) form_dv(q, q, false);   // a ghost plane waits for its mirror
      if (zwall && q == P.nz) form_dv(q, P.nz - 1, true);
      __syncthreads();
      if (own_xy && (!zwall || (q >= 0 && q <= P.nz))) {
        div_part(up, mid, dn);
#pragma unroll
        for (int b = 0; b < 3; ++b) {
          dv_t[b] += up[b];
          dv_t1[b] += mid[b];
          dv_t2[b] = dn[b];
        }
      }
    }
    if (t >= z0 && own_xy) {
      auto node = [&]() {
        const int z = t;
        const bool fast = fast_at(t);
        const long long idx = ((long long)z * P.ny + y) * P.nx + x;
        const uint32_t hbyte = (uint32_t)idx * HS;
        const HT* hsrc = P.hist_src ? (const HT*)P.hist_src : hist;
        auto hld = [&](int plane) -> CT {
          if (P.plane32) return CT(*(const HT*)((const char*)(hsrc + (size_t)plane * (size_t)N) + hbyte));
          return CT(hsrc[(long long)plane * N + idx]);
        };
        // own populations and moments
        CT fns[NS ? QN : 1], fph[PHI ? QP : 1], fps[PSI ? QS : 1], fc[CC ? QS : 1], fth[TH ? QS : 1];
        CT phi = CT(1), psi = CT(-1), C = CT(0), H = CT(0), U = K.U0, j[3] = {CT(0), CT(0), CT(0)};
        CT dphi = CT(0), dpsi = CT(0), dC = CT(0), dH = CT(0);
        CT h_psi = CT(0), h_S = CT(0), h_pv[3] = {CT(0), CT(0), CT(0)}, h_B[3] = {CT(0), CT(0), CT(0)};
        CT h_Hv[3] = {CT(0), CT(0), CT(0)};
        int gid = 0;
        if (PSI) gid = P.grain[idx];
        if (!first && mode == 0) {
          if constexpr (PSI) { h_psi = hld(P.h_psi); h_S = hld(P.h_S); }
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            if constexpr (PHI) h_pv[a] = hld(P.h_phiv + a);
            if constexpr (CC) h_B[a] = hld(P.h_B + a);
            if constexpr (TH) h_Hv[a] = hld(P.h_Hv + a);
          }
        }
        if constexpr (NS) {
          if constexpr (KEEP) {
#pragma unroll
            for (int i = 0; i < QN; ++i) fns[i] = kA_ns[i];
          } else if constexpr (KEEP16) {
#pragma unroll
            for (int i = 0; i < QN; ++i) fns[i] = unkeep16<ST>(kA16[i / 2], i % 2);
          } else {
            pull3<QN, ST, CT, SYM>(fast, fin_ns, P, x, y, z, fns);
          }
#pragma unroll
          for (int i = 0; i < QN; ++i) {
            if (LN::c[i][0]) j[0] += CT(LN::c[i][0]) * fns[i];
            if (LN::c[i][1]) j[1] += CT(LN::c[i][1]) * fns[i];
            if (LN::c[i][2]) j[2] += CT(LN::c[i][2]) * fns[i];
          }
        }
        if constexpr (PHI) {
          if constexpr (KEEPPHI) {
#pragma unroll
            for (int i = 0; i < QP; ++i) fph[i] = kph0[i];
          } else {
            pull3<QP, ST, CT, SYM>(fast, fin_phi, P, x, y, z, fph);
          }
#pragma unroll
          for (int i = 0; i < QP; ++i) dphi += fph[i];
          phi = r_phi + dphi;
        }
        if constexpr (PSI) {
          if constexpr (KEEP) {
#pragma unroll
            for (int i = 0; i < QS; ++i) fps[i] = kA_ps[i];
          } else {
            pull3<QS, ST, CT, SYM>(fast, fin_psi, P, x, y, z, fps);
          }
#pragma unroll
          for (int i = 0; i < QS; ++i) dpsi += fps[i];
          psi = r_psi + dpsi;
        }
        if constexpr (CC) {
          if constexpr (KEEP) {
#pragma unroll
            for (int i = 0; i < QS; ++i) fc[i] = kA_c[i];
          } else {
            pull3<QS, ST, CT, SYM>(fast, fin_c, P, x, y, z, fc);
          }
#pragma unroll
          for (int i = 0; i < QS; ++i) dC += fc[i];
          C = r_C + dC;
          const CT h = (psi + CT(1)) * CT(0.5);
          U = (C * rcp(CT(1) - k1 * h) - CT(1)) * K.inv_k1;
        }
        if constexpr (TH) {
          pull3<QS, ST, CT, SYM>(fast, fin_th, P, x, y, z, fth);
#pragma unroll
          for (int i = 0; i < QS; ++i) dH += fth[i];
          H = r_H + dH;
        }
        // flow quantities of the own node (its v0 is not needed) and the
        // stencil planes around it
        FlowNode3<CT> fo;
        const CT* ph[3];
        phi_planes(z, ph);
        flow_node3<NS, PHI, R, CT>(K, ph, s_psi + ring_slot(z, NPS) * P1::N, nullptr, ly + 1, lx + 1, fo);
        const CT* psp[3];
        const CT* Up[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          psp[c] = s_psi + ring_slot(z - 1 + c, NPS) * P1::N;
          Up[c] = s_U + (CC ? ring_slot(z - 1 + c, NPS) * P1::N : 0);
        }
          // ---- phase C: the rest of the step at the own node
          // direction i of the 7-velocity sets leaves across a far-field side, whose
          // populations come back by anti-bounce-back, -f*_i + 2 w_i value
          auto far_out = [&](int i) -> bool {
            if constexpr (!SYM) return false;
            if (fast || !P.far) return false;
            const int n3[3] = {P.nx, P.ny, P.nz};
            const int xyz[3] = {x, y, z};
            bool out = false;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
              const int ca = LS::c[i][a];
              if (ca > 0 && xyz[a] == n3[a] - 1 && far_side(P, a, false)) out = true;
              if (ca < 0 && xyz[a] == 0 && far_side(P, a, true)) out = true;
            }
            return out;
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
          CT gp[3] = {CT(0), CT(0), CT(0)}, gU[3] = {CT(0), CT(0), CT(0)};
          if constexpr (PSI) grad19p<CT, P1>(psp, ly + 1, lx + 1, gp);
          if constexpr (CC) grad19p<CT, P1>(Up, ly + 1, lx + 1, gU);
          const CT dn = K.dn;
          const CT invp = rsq(gp[0] * gp[0] + gp[1] * gp[1] + gp[2] * gp[2] + dn);
          // cubic anisotropy in the crystal frame (rotation about z):
          // a_s = 1 + eps (4 S4 - 3 G^2) / (G + delta)^2, N' = G a_s d a_s / d g'
          CT a_s, Nv[3];
          {
            const CT cth = CT(P.grain_cs[2 * gid]), sth = CT(P.grain_cs[2 * gid + 1]);
            const CT r[3] = {cth * gp[0] + sth * gp[1], -sth * gp[0] + cth * gp[1], gp[2]};
            const CT r2[3] = {r[0] * r[0], r[1] * r[1], r[2] * r[2]};
            const CT G = r2[0] + r2[1] + r2[2];
            const CT S4 = r2[0] * r2[0] + r2[1] * r2[1] + r2[2] * r2[2];
            const CT invGd = rcp(G + dn);
            const CT inv2 = invGd * invGd;
            const CT eps = K.eps4;
            a_s = CT(1) + eps * (CT(4) * S4 - CT(3) * G * G) * inv2;
            const CT pre = CT(4) * eps * G * a_s * inv2 * invGd;
            CT Nr[3];
#pragma unroll
            for (int a = 0; a < 3; ++a)
              Nr[a] = pre * r[a] * (CT(4) * r2[a] * G + (CT(4) * r2[a] - CT(3) * G) * dn - CT(4) * S4);
            Nv[0] = cth * Nr[0] - sth * Nr[1];
            Nv[1] = sth * Nr[0] + cth * Nr[1];
            Nv[2] = Nr[2];
          }
          const CT as2 = a_s * a_s;

          const CT lin = CT(1) + k1 * U;
          const CT F = K.inv_Le + K.Mcinf * (lin > CT(0) ? lin : CT(0));
          const CT gFs = lin > CT(0) ? K.Mcinf * k1 : CT(0);

          const CT om = CT(1) - phi;
          const CT ps1 = psi + CT(1);
          const CT f2p = CT(0.5) * (CT(1) - psi) * ps1 * (CT(-2) * psi);
          const CT f3psi = CT(2) * K.beta_inter * om * om * ps1;
          const CT s1m = (CT(1) - psi) * ps1;
          const CT pprime = CT(30.0 / 32.0) * s1m * s1m;
          const CT Qpsi = -(f2p + f3psi + K.lam * pprime * (theta + K.Mcinf * U));
          // rewritten form: a_n = a_s^2, F(U) in D_psi and S_psi with the
          // grad F term; form for Le = O(1): a_n = a_s^2 F(U) (Appendix B)
          CT S_psi, D_psi;
          if (P.le1) {
            S_psi = Qpsi * K.inv_tau0;
            D_psi = K.d_psi * as2;
          } else {
            const CT invF = rcp(F);
            CT gdot = CT(0);
#pragma unroll
            for (int a = 0; a < 3; ++a) gdot += gFs * gU[a] * (as2 * gp[a] + Nv[a]);
            S_psi = K.d_psi * invF * invF * gdot + Qpsi * invF * K.inv_tau0;
            D_psi = K.d_psi * as2 * invF;
          }
          const CT an = P.le1 ? as2 * F : as2;
          const CT rate_psi = rcp(D_psi * CT(1.0 / LS::cs2) + CT(0.5));

          // velocity, forces, pressure (pressure recovered in FP64 in every mode)
          CT v[3] = {CT(0), CT(0), CT(0)}, Ft[3] = {CT(0), CT(0), CT(0)}, p = CT(0);
          const CT rho = fo.rho;
          const CT gr[3] = {K.drho * fo.g[0], K.drho * fo.g[1], K.drho * fo.g[2]};
          if constexpr (NS) {
            CT Fm[3] = {CT(0), CT(0), CT(0)};
            if constexpr (FLOWX) {
              // (div X)_b = (1/cs2) sum_i w_i (c_i . D(x + c_i)) v0_b(x + c_i), summed
              // plane by plane as the planes were formed
#pragma unroll
              for (int b = 0; b < 3; ++b) Fm[b] = K.drho * CT(3) * dv_t[b];
            }
            const CT Fb[3] = {CT(0), -(rho - K.rho_l) * K.g, CT(0)};
            const CT onechi = CT(1) - fo.chi;
            const CT irho = rcp(rho);
#pragma unroll
            for (int a = 0; a < 3; ++a) {
              const CT rv = j[a] + CT(0.5) * (fo.Fs[a] + Fb[a] + Fm[a]);
              v[a] = onechi * rv * irho;
              Ft[a] = fo.Fs[a] + Fb[a] + Fm[a] - CT(2) * fo.chi * rv;
            }
            const double vvd = (double)v[0] * v[0] + (double)v[1] * v[1] + (double)v[2] * v[2];
            const double s0 = -LN::w[0] * vvd * 1.5;
            double sum = 0.0;
#pragma unroll
            for (int i = 1; i < QN; ++i) sum += (double)fns[i];
            const double vg = (double)v[0] * gr[0] + (double)v[1] * gr[1] + (double)v[2] * gr[2];
            p = CT(LN::cs2 / (1.0 - LN::w[0]) * (sum + 0.5 * vg + (double)rho * s0));
          }

          if (mode == 1) {
            const double m9[9] = {(double)phi, (double)psi, (double)C, (double)theta, (double)U, (double)p,
                                  (double)v[0], (double)v[1], (double)v[2]};
            put_macros(P, mout, idx, m9);
            return;
          }

          const uint32_t nbyte = (uint32_t)idx * S;
          constexpr bool LOWP = sizeof(raw) == 2;
          constexpr int QMAX = NS ? QN : QS;
          const RoundBits<LOWP ? (QMAX + 1) / 2 : 1> rb(LOWP ? round_seed(P, (uint32_t)idx) : 0u, LOWP && P.sr);
          // store of population i of the set whose first plane is o
          auto st = [&](int o, int i, CT val) {
            const int plane = o + i;
            raw* ptr = P.plane32 ? at_byte<ST>(fout + (size_t)plane * (size_t)N, nbyte) : fout + (long long)plane * N + idx;
            uint32_t r = 0u;
            if constexpr (LOWP) r = rb.bits(i);
            store_pop<ST, CT, STREAM>(P, ptr, val, r);
          };
          auto hst = [&](int plane, CT val) {
            HT* q = P.plane32 ? (HT*)((char*)(hist + (size_t)plane * (size_t)N) + hbyte) : hist + (long long)plane * N + idx;
            put<STREAM, HT>(q, (HT)val);
          };

          // ---- NS collision: f* = feq + F/2 + (1 - s_nu) P_s (f - feq + F/2), P_s
          // the orthogonal projector on the five traceless stress moments
          // 2cx^2 - cy^2 - cz^2, cy^2 - cz^2, cx cy, cy cz, cx cz (squared norms over
          // D3Q19: 36, 12, 4, 4, 4)
          if constexpr (NS) {
            const CT nu = (K.mu_g + (K.mu_l - K.mu_g) * phi) * rcp(rho);
            const CT s_nu = rcp(nu * CT(3) + CT(0.5));
            const CT vv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
            const CT vF = v[0] * Ft[0] + v[1] * Ft[1] + v[2] * Ft[2];
            {
              // the collision in moment form (D3Q19 is 4th-order
              // isotropic, so each traceless stress moment T of f^eq + F/2 is
              // rho T:vv + T:(vF + cs2 v grad(rho)) symmetrised; for i > 0
              // f_i^eq + F_i/2 = w_i [A + c.v (3 rho + 4.5 (rho c.v + c.F) + 1.5 c.grad(rho)) + 1.5 c.F]
              // with A = 3p - 1.5 rho v.v - 1.5 v.F, and w_0 A - 3p at rest)
              const CT r = CT(1) - s_nu;
              const CT A = CT(3) * p - CT(1.5) * rho * vv - CT(1.5) * vF;
              CT s9 = CT(0), s11 = CT(0), sxy = CT(0), syz = CT(0), sxz = CT(0);
#pragma unroll
              for (int i = 1; i < QN; ++i) {
                const int cx = LN::c[i][0], cy = LN::c[i][1], cz = LN::c[i][2];
                s9 += CT(2 * cx * cx - cy * cy - cz * cz) * fns[i];
                s11 += CT(cy * cy - cz * cz) * fns[i];
                sxy += CT(cx * cy) * fns[i];
                syz += CT(cy * cz) * fns[i];
                sxz += CT(cx * cz) * fns[i];
              }
              const CT vx = v[0], vy = v[1], vz = v[2], Fx = Ft[0], Fy = Ft[1], Fz = Ft[2];
              const CT gx = gr[0], gy = gr[1], gz = gr[2];
              constexpr CT c3 = CT(1.0 / 3), c6 = CT(1.0 / 6);
              const CT q9 = (r * CT(1.0 / 36)) * (s9 - rho * (CT(2) * vx * vx - vy * vy - vz * vz) +
                                                  (CT(2) * vx * Fx - vy * Fy - vz * Fz) +
                                                  c3 * (CT(2) * vx * gx - vy * gy - vz * gz));
              const CT q11 = (r * CT(1.0 / 12)) * (s11 - rho * (vy * vy - vz * vz) + (vy * Fy - vz * Fz) +
                                                   c3 * (vy * gy - vz * gz));
              const CT qxy = (r * CT(0.25)) * (sxy - rho * vx * vy + CT(0.5) * (vx * Fy + vy * Fx) + c6 * (vx * gy + vy * gx));
              const CT qyz = (r * CT(0.25)) * (syz - rho * vy * vz + CT(0.5) * (vy * Fz + vz * Fy) + c6 * (vy * gz + vz * gy));
              const CT qxz = (r * CT(0.25)) * (sxz - rho * vx * vz + CT(0.5) * (vx * Fz + vz * Fx) + c6 * (vx * gz + vz * gx));
              const CT rho3 = CT(3) * rho;
              auto post = [&](int i) -> CT {
                const int cx = LN::c[i][0], cy = LN::c[i][1], cz = LN::c[i][2];
                const CT w = CT(LN::w[i]);
                if (i == 0) return w * A - CT(3) * p;
                const CT cv = CT(cx) * vx + CT(cy) * vy + CT(cz) * vz;
                const CT cF = CT(cx) * Fx + CT(cy) * Fy + CT(cz) * Fz;
                const CT cg = CT(cx) * gx + CT(cy) * gy + CT(cz) * gz;
                const CT t = cv * (rho3 + CT(4.5) * (rho * cv + cF) + CT(1.5) * cg) + CT(1.5) * cF + A;
                return w * t + (CT(2 * cx * cx - cy * cy - cz * cz) * q9 + CT(cy * cy - cz * cz) * q11 +
                                CT(cx * cy) * qxy + CT(cy * cz) * qyz + CT(cx * cz) * qxz);
              };
              // Velocity and pressure sides (non-equilibrium extrapolation, Sec. 3
              // boundary paragraph): the slot of population i leaving across one
              // holds what the node pulls back along j = opp(i) next step, its own
              // f*_j plus f^eq_j(p, rho, v_in) - f^eq_j(p, rho, v) (velocity side)
              // or f^eq_j(0, rho, v) - f^eq_j(p, rho, v) = -w_j p / cs2 (pressure
              // side); a velocity side takes precedence where both are crossed.
              auto nee_out = [&](int i) -> int {
                if constexpr (!SYM) return 0;
                if (fast || !(P.vel | P.pres)) return 0;
                const int dx = LN::c[i][0], dy = LN::c[i][1], dz = LN::c[i][2];
                auto across = [&](int m) {
                  return (dx > 0 && x == P.nx - 1 && ((m >> 3) & 1)) || (dx < 0 && x == 0 && (m & 1)) ||
                         (dy > 0 && y == P.ny - 1 && ((m >> 4) & 1)) || (dy < 0 && y == 0 && ((m >> 1) & 1)) ||
                         (dz > 0 && z == P.nz - 1 && ((m >> 5) & 1)) || (dz < 0 && z == 0 && ((m >> 2) & 1));
                };
                return across(P.vel) ? 1 : (across(P.pres) ? 2 : 0);
              };
              auto nee = [&](int j, int kind) -> CT {
                if (kind == 2) return -CT(LN::w[j]) * p * CT(3);
                const CT cx = CT(LN::c[j][0]), cy = CT(LN::c[j][1]), cz = CT(LN::c[j][2]);
                const CT bx = CT(P.vin[0]), by = CT(P.vin[1]), bz = CT(P.vin[2]);
                const CT cb = cx * bx + cy * by + cz * bz, cv = cx * vx + cy * vy + cz * vz;
                return rho * CT(LN::w[j]) *
                       ((cb - cv) * CT(3) + (cb * cb - cv * cv) * CT(4.5) - (bx * bx + by * by + bz * bz - vv) * CT(1.5));
              };
#pragma unroll
              for (int i = 0; i < QN; ++i) {
                CT fs = post(i);
                if (const int kind = nee_out(i)) fs = post(LN::opp[i]) + nee(LN::opp[i], kind);
                st(P.o_ns, i, fs);
              }
            }
          }

          // ---- CAC collision (flux moments relaxed, squared norm 2 on D3Q7)
          const CT phiv[3] = {phi * v[0], phi * v[1], phi * v[2]};
          if constexpr (PHI) {
            CT fl[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
              const CT prev = first ? phiv[a] : h_pv[a];
              fl[a] = (phiv[a] - prev) + CT(LP::cs2) * fo.sharp * fo.n[a];
            }
            const CT s1 = K.s_phi;
            CT feq[QP], G[QP];
            CT jf[3] = {CT(0), CT(0), CT(0)}, gj[3] = {CT(0), CT(0), CT(0)};
#pragma unroll
            for (int i = 0; i < QP; ++i) {
              const CT cx = CT(LP::c[i][0]), cy = CT(LP::c[i][1]), cz = CT(LP::c[i][2]);
              const CT w = CT(LP::w[i]);
              const CT cv = cx * v[0] + cy * v[1] + cz * v[2];
              if constexpr (DEV) feq[i] = w * dphi + w * phi * cv * CT(1.0 / LP::cs2);
              else feq[i] = w * phi * (CT(1) + cv * CT(1.0 / LP::cs2));
              G[i] = w * (cx * fl[0] + cy * fl[1] + cz * fl[2]) * CT(1.0 / LP::cs2);
              const CT d = fph[i] - feq[i];
              jf[0] += cx * d; jf[1] += cy * d; jf[2] += cz * d;
              gj[0] += cx * G[i]; gj[1] += cy * G[i]; gj[2] += cz * G[i];
            }
            const CT inv_fn = CT(1.0 / LP::flux_norm);
#pragma unroll
            for (int i = 0; i < QP; ++i) {
              const CT cx = CT(LP::c[i][0]), cy = CT(LP::c[i][1]), cz = CT(LP::c[i][2]);
              const CT Pf = (cx * jf[0] + cy * jf[1] + cz * jf[2]) * inv_fn;
              const CT PG = (cx * gj[0] + cy * gj[1] + cz * gj[2]) * inv_fn;
              st(P.o_phi, i, feq[i] + (CT(1) - s1) * Pf + CT(0.5) * G[i] + CT(0.5) * (CT(1) - s1) * PG);
            }
#pragma unroll
            for (int a = 0; a < 3; ++a) hst(P.h_phiv + a, phiv[a]);
          }

          // ---- AAC collision with the time-stretched store.  The population i at
          // x + c_i before this step is the stored value of plane i at x itself
          // (pull form); across a wall it is the own f_opp(i).
          if constexpr (PSI) {
            const CT Sprev = first ? S_psi : h_S;
            const CT inv_an = rcp(an);
            CT jf[3] = {CT(0), CT(0), CT(0)};
#pragma unroll
            for (int i = 0; i < QS; ++i) {
              const CT d = fps[i] - CT(LS::w[i]) * dpsi;
              if (LS::c[i][0]) jf[0] += CT(LS::c[i][0]) * d;
              if (LS::c[i][1]) jf[1] += CT(LS::c[i][1]) * d;
              if (LS::c[i][2]) jf[2] += CT(LS::c[i][2]) * d;
            }
            const CT inv_as2 = P.le1 ? rcp(as2) : inv_an;
            const CT gN[3] = {-Nv[0] * inv_as2, -Nv[1] * inv_as2, -Nv[2] * inv_as2};
            const raw* own_psi = fin_psi + idx;
            const int n3[3] = {P.nx, P.ny, P.nz};
            const int xyz[3] = {x, y, z};
#pragma unroll
            for (int i = 0; i < QS; ++i) {
              const CT cx = CT(LS::c[i][0]), cy = CT(LS::c[i][1]), cz = CT(LS::c[i][2]);
              const CT w = CT(LS::w[i]);
              const CT G = w * (cx * gN[0] + cy * gN[1] + cz * gN[2]);
              CT fstar = w * dpsi + (CT(1) - rate_psi) * (cx * jf[0] + cy * jf[1] + cz * jf[2]) * CT(0.5) +
                         w * S_psi + CT(0.5) * w * (S_psi - Sprev) + (CT(1) - CT(0.5) * rate_psi) * G;
              // anti-bounce-back to psi_l = -1 (stored less the rest value r_psi)
              if (far_out(i)) fstar = CT(2) * w * (CT(-1) - r_psi) - fstar;
              bool across = false;
#pragma unroll
              for (int a = 0; a < 3; ++a) {
                const int ca = LS::c[i][a];
                if (ca && P.wall[a] && (xyz[a] + ca < 0 || xyz[a] + ca >= n3[a])) across = true;
              }
              const CT old = across ? fps[LS::opp[i]]
                                    : Store<ST>::template ld<CT>(own_psi + (long long)i * N);
              st(P.o_psi, i, (fstar - (CT(1) - an) * old) * inv_an);
            }
          }

          // ---- solute collision
          if constexpr (CC) {
            const CT psi_prev = first ? psi : h_psi;
            const CT at = -K.aW0 * a_s * lin * (psi - psi_prev);
            const CT jv = K.D * q * C * K.sharp * (om > CT(0) ? om : CT(0));
            const CT m = CT(1) - k1 * h;
            const CT invm = rcp(m);
            const CT dr = K.D * q * C * k1 * invm * invm * CT(0.5);
            CT B[3], dB[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
              B[a] = C * v[a] - dr * gp[a] + k1 * (at * gp[a] * invp + jv * fo.n[a]);
              dB[a] = B[a] - (first ? B[a] : h_B[a]);
            }
            const CT s1 = rcp(K.D * q * invm * CT(1.0 / LS::cs2) + CT(0.5));
            CT jf[3] = {-B[0], -B[1], -B[2]};
#pragma unroll
            for (int i = 0; i < QS; ++i) {
              if (LS::c[i][0]) jf[0] += CT(LS::c[i][0]) * fc[i];
              if (LS::c[i][1]) jf[1] += CT(LS::c[i][1]) * fc[i];
              if (LS::c[i][2]) jf[2] += CT(LS::c[i][2]) * fc[i];
            }
#pragma unroll
            for (int i = 0; i < QS; ++i) {
              const CT cx = CT(LS::c[i][0]), cy = CT(LS::c[i][1]), cz = CT(LS::c[i][2]);
              const CT w = CT(LS::w[i]);
              const CT feq = w * dC + w * (cx * B[0] + cy * B[1] + cz * B[2]) * CT(1.0 / LS::cs2);
              const CT G = w * (cx * dB[0] + cy * dB[1] + cz * dB[2]) * CT(1.0 / LS::cs2);
              CT fs = feq + (CT(1) - s1) * (cx * jf[0] + cy * jf[1] + cz * jf[2]) * CT(0.5) + (CT(1) - CT(0.5) * s1) * G;
              if (far_out(i)) fs = CT(2) * w * (CT(1) - r_C) - fs;      // anti-bounce-back to C = 1
              st(P.o_c, i, fs);
            }
#pragma unroll
            for (int a = 0; a < 3; ++a) hst(P.h_B + a, B[a]);
          }

          // ---- heat collision
          if constexpr (TH) {
            const CT Hv[3] = {H * v[0], H * v[1], H * v[2]};
            CT dHv[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) dHv[a] = Hv[a] - (first ? Hv[a] : h_Hv[a]);
            const CT s1 = s_th;
            CT jf[3] = {-Hv[0], -Hv[1], -Hv[2]};
#pragma unroll
            for (int i = 0; i < QS; ++i) {
              if (LS::c[i][0]) jf[0] += CT(LS::c[i][0]) * fth[i];
              if (LS::c[i][1]) jf[1] += CT(LS::c[i][1]) * fth[i];
              if (LS::c[i][2]) jf[2] += CT(LS::c[i][2]) * fth[i];
            }
#pragma unroll
            for (int i = 0; i < QS; ++i) {
              const CT cx = CT(LS::c[i][0]), cy = CT(LS::c[i][1]), cz = CT(LS::c[i][2]);
              const CT w = CT(LS::w[i]);
              CT geq = w * dtheta + w * (cx * Hv[0] + cy * Hv[1] + cz * Hv[2]) * CT(1.0 / LS::cs2);
              // H (the sum of g) is rho times the model's H: the rest equilibrium
              // rho H + (w - 1) theta less w theta0 is dH + (w - 1) dtheta
              if (i == 0) {
                if constexpr (DEV) geq = K.varheat ? dH + (w - CT(1)) * dtheta : -h + w * dtheta;
                else geq = H + (w - CT(1)) * theta;
              }
              const CT G = w * (cx * dHv[0] + cy * dHv[1] + cz * dHv[2]) * CT(1.0 / LS::cs2);
              CT gs = geq + (CT(1) - s1) * (cx * jf[0] + cy * jf[1] + cz * jf[2]) * CT(0.5) + (CT(1) - CT(0.5) * s1) * G;
              if (far_out(i)) gs = CT(2) * w * (K.theta0 - r_H) - gs;   // anti-bounce-back to theta0
              st(P.o_th, i, gs);
            }
#pragma unroll
            for (int a = 0; a < 3; ++a) hst(P.h_Hv + a, Hv[a]);
          }

          if constexpr (PSI) {
            hst(P.h_psi, psi);
            hst(P.h_S, S_psi);
          }
      };
      node();
    }
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      dv_t[b] = dv_t1[b];
      dv_t1[b] = dv_t2[b];
    }
    if constexpr (KEEP) {
#pragma unroll
      for (int i = 0; i < KN; ++i) kA_ns[i] = kB_ns[i];
#pragma unroll
      for (int i = 0; i < KS; ++i) kA_ps[i] = kB_ps[i];
#pragma unroll
      for (int i = 0; i < KC; ++i) kA_c[i] = kB_c[i];
    }
    if constexpr (KEEP16) {
#pragma unroll
      for (int w = 0; w < KW; ++w) kA16[w] = kB16[w];
    }
    rot_phi();
    // no barrier here: the next phase A writes slots this phase C does not
    // read (the slot counts above), the D_phi/v0 plane is read before the
    // barrier after phase B, and the momentum plane only in phase B
  }
}

template <int FIELDS, class ST, class HT, class CT>
hipError_t launch_step3d_t(const DevParams& P, const void* fin, void* fout, void* hist, double* mout,
                           int mode, hipStream_t s) {
  using T = Col3<CT>;
  const long long tiles = (long long)((P.nx + T::TX - 1) / T::TX) * ((P.ny + T::TY - 1) / T::TY) *
                          ((P.nz + P.zc - 1) / P.zc);
  using raw = typename Store<ST>::raw;
  const bool sym = P.sym || P.far;
#define PFL_LAUNCH3(SYMV, NTV)                                                                    \
  hipLaunchKernelGGL((step3d_kernel<FIELDS, ST, HT, CT, SYMV, NTV>), dim3((unsigned)tiles), dim3(T::NT), 0, s, \
                     P, (const raw*)fin, (raw*)fout, (HT*)hist, mout, mode)
  if (sym && P.nt) PFL_LAUNCH3(true, true);
  else if (sym) PFL_LAUNCH3(true, false);
  else if (P.nt) PFL_LAUNCH3(false, true);
  else PFL_LAUNCH3(false, false);
#undef PFL_LAUNCH3
  return hipGetLastError();
}

template <class ST, class HT, class CT>
hipError_t dispatch3(const DevParams& P, int fields, const void* fin, void* fout, void* hist, double* mout,
                     int mode, hipStream_t s, bool& ok) {
  ok = true;
  switch (fields) {
    case F_NS | F_PHI | F_PSI | F_C | F_TH:
      return launch_step3d_t<F_NS | F_PHI | F_PSI | F_C | F_TH, ST, HT, CT>(P, fin, fout, hist, mout, mode, s);
    case F_PSI | F_C:
      return launch_step3d_t<F_PSI | F_C, ST, HT, CT>(P, fin, fout, hist, mout, mode, s);
    case F_PSI | F_C | F_TH:
      return launch_step3d_t<F_PSI | F_C | F_TH, ST, HT, CT>(P, fin, fout, hist, mout, mode, s);
    case F_NS | F_PHI:
      return launch_step3d_t<F_NS | F_PHI, ST, HT, CT>(P, fin, fout, hist, mout, mode, s);
    case F_PSI:
      return launch_step3d_t<F_PSI, ST, HT, CT>(P, fin, fout, hist, mout, mode, s);
    case F_PHI:
      return launch_step3d_t<F_PHI, ST, HT, CT>(P, fin, fout, hist, mout, mode, s);
    case F_NS | F_PSI | F_TH:
      return launch_step3d_t<F_NS | F_PSI | F_TH, ST, HT, CT>(P, fin, fout, hist, mout, mode, s);
    default:
      ok = false;
      return hipSuccess;
  }
}

}  // namespace

}  // namespace pfl
