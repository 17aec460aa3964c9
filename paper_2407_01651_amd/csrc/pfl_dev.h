// Device-side definitions shared by the step, init, export and reduction
// kernels: lattice tables, the parameter block passed by value to every
// kernel, storage conversions.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <hip/hip_bf16.h>
#include <cstdint>
#include <type_traits>

namespace pfl {

enum : int { F_NS = 1, F_PHI = 2, F_PSI = 4, F_C = 8, F_TH = 16 };

constexpr int MAX_SEEDS = 256;
constexpr int MAX_BUBBLES = 256;

// ---------------------------------------------------------------- lattices
// D2Q5 / D2Q9 / D3Q7 / D3Q19 with the velocity order of pfl.h.
template <int Q> struct Lat;

template <> struct Lat<5> {
  static constexpr int Q = 5, D = 2;
  static constexpr int c[5][3] = {{0,0,0},{1,0,0},{0,1,0},{-1,0,0},{0,-1,0}};
  static constexpr int opp[5] = {0, 3, 4, 1, 2};
  // refl[a][i]: c_i with its component on axis a reversed (specular reflection)
  static constexpr int refl[3][5] = {{0,3,2,1,4}, {0,1,4,3,2}, {0,1,2,3,4}};
  static constexpr double w[5] = {1.0/3, 1.0/6, 1.0/6, 1.0/6, 1.0/6};
  static constexpr double cs2 = 1.0/3;
  static constexpr double flux_norm = 2.0;   // sum_i c_ia^2
};

template <> struct Lat<9> {
  static constexpr int Q = 9, D = 2;
  static constexpr int c[9][3] = {{0,0,0},{1,0,0},{0,1,0},{-1,0,0},{0,-1,0},
                                  {1,1,0},{-1,1,0},{-1,-1,0},{1,-1,0}};
  static constexpr int opp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
  // refl[a][i]: c_i with its component on axis a reversed (specular reflection)
  static constexpr int refl[3][9] = {{0,3,2,1,4,6,5,8,7}, {0,1,4,3,2,8,7,6,5}, {0,1,2,3,4,5,6,7,8}};
  static constexpr double w[9] = {4.0/9, 1.0/9, 1.0/9, 1.0/9, 1.0/9,
                                  1.0/36, 1.0/36, 1.0/36, 1.0/36};
  static constexpr double cs2 = 1.0/3;
  static constexpr double flux_norm = 6.0;
};

template <> struct Lat<7> {
  static constexpr int Q = 7, D = 3;
  static constexpr int c[7][3] = {{0,0,0},{1,0,0},{-1,0,0},{0,1,0},{0,-1,0},{0,0,1},{0,0,-1}};
  static constexpr int opp[7] = {0, 2, 1, 4, 3, 6, 5};
  // refl[a][i]: c_i with its component on axis a reversed (specular reflection)
  static constexpr int refl[3][7] = {{0,2,1,3,4,5,6}, {0,1,2,4,3,5,6}, {0,1,2,3,4,6,5}};
  static constexpr double w[7] = {0.25, 0.125, 0.125, 0.125, 0.125, 0.125, 0.125};
  static constexpr double cs2 = 0.25;
  static constexpr double flux_norm = 2.0;
};

template <> struct Lat<19> {
  static constexpr int Q = 19, D = 3;
  static constexpr int c[19][3] = {{0,0,0},{1,0,0},{-1,0,0},{0,1,0},{0,-1,0},{0,0,1},{0,0,-1},
                                   {1,1,0},{-1,-1,0},{1,-1,0},{-1,1,0},
                                   {1,0,1},{-1,0,-1},{1,0,-1},{-1,0,1},
                                   {0,1,1},{0,-1,-1},{0,1,-1},{0,-1,1}};
  static constexpr int opp[19] = {0,2,1,4,3,6,5,8,7,10,9,12,11,14,13,16,15,18,17};
  // refl[a][i]: c_i with its component on axis a reversed (specular reflection)
  static constexpr int refl[3][19] = {{0,2,1,3,4,5,6,10,9,8,7,14,13,12,11,15,16,17,18},
                                    {0,1,2,4,3,5,6,9,10,7,8,11,12,13,14,18,17,16,15},
                                    {0,1,2,3,4,6,5,7,8,9,10,13,14,11,12,17,18,15,16}};
  static constexpr double w[19] = {1.0/3, 1.0/18, 1.0/18, 1.0/18, 1.0/18, 1.0/18, 1.0/18,
                                   1.0/36, 1.0/36, 1.0/36, 1.0/36, 1.0/36, 1.0/36,
                                   1.0/36, 1.0/36, 1.0/36, 1.0/36, 1.0/36, 1.0/36};
  static constexpr double cs2 = 1.0/3;
  static constexpr double flux_norm = 10.0;
};

// The reflection tables reverse exactly one component of each velocity.
template <int Q>
constexpr bool refl_consistent() {
  using L = Lat<Q>;
  for (int a = 0; a < 3; ++a)
    for (int i = 0; i < Q; ++i)
      for (int b = 0; b < 3; ++b)
        if (L::c[L::refl[a][i]][b] != (a == b ? -L::c[i][b] : L::c[i][b])) return false;
  return true;
}
static_assert(refl_consistent<5>() && refl_consistent<9>() && refl_consistent<7>() && refl_consistent<19>(),
              "reflection tables");

// Index of c_i with the components on the flagged axes reversed, from a
// table in constant memory (read on the edge tiles only; a select over
// constants would hold every candidate in scalar registers).
template <int Q>
struct ReflTab {
  signed char r[Q][8];
};
template <int Q>
constexpr ReflTab<Q> make_refl_tab() {
  ReflTab<Q> t{};
  for (int i = 0; i < Q; ++i)
    for (int m = 0; m < 8; ++m) {
      int j = i;
      for (int a = 0; a < 3; ++a)
        if ((m >> a) & 1) j = Lat<Q>::refl[a][j];
      t.r[i][m] = (signed char)j;
    }
  return t;
}
static __constant__ const ReflTab<5> kRefl5 = make_refl_tab<5>();
static __constant__ const ReflTab<9> kRefl9 = make_refl_tab<9>();
static __constant__ const ReflTab<7> kRefl7 = make_refl_tab<7>();
static __constant__ const ReflTab<19> kRefl19 = make_refl_tab<19>();
template <int Q> __device__ __forceinline__ const ReflTab<Q>& refl_tab();
template <> __device__ __forceinline__ const ReflTab<5>& refl_tab<5>() { return kRefl5; }
template <> __device__ __forceinline__ const ReflTab<9>& refl_tab<9>() { return kRefl9; }
template <> __device__ __forceinline__ const ReflTab<7>& refl_tab<7>() { return kRefl7; }
template <> __device__ __forceinline__ const ReflTab<19>& refl_tab<19>() { return kRefl19; }

template <int Q>
__device__ __forceinline__ int lat_reflected(int i, int fx, int fy, int fz) {
  const int m = fx | (fy << 1) | (fz << 2);
  return m ? (int)refl_tab<Q>().r[i][m] : i;
}

// ------------------------------------------------------------- parameters
// Constants of the step in the compute precision, reciprocals precomputed.
template <class CT>
struct KP {
  CT k1, inv_k1, U0, theta0, eps4, dn, d_psi, inv_tau0, D, lam, Mcinf, inv_Le, beta_inter;
  CT sharp, M_phi, Wphi2, k_s, rho_l, rho_g, drho, mu_l, mu_g, g, s_phi, s_th, aW0;
  CT C_ref;                     // bulk solute 1 + (1-k) U0 of the deviation storage
  // heat properties (liquid = solid = 1): gas ratios of rho, c_p, k_T, alpha / cs2
  CT th_rho_g, th_cp_g, th_k_g, alpha_cs;
  int varheat;                  // a gas ratio differs from 1
};

// Planes of a 2D step tape (compute type, N nodes each): grad phi (x, y),
// Laplacian of phi, grad psi (x, y), grad U (x, y), mass-flux force (x, y).
constexpr int TAPE_PLANES = 9;

// Everything a kernel needs, passed by value (well under the 4 KB limit).
struct DevParams {
  int nx, ny, nz, dim;
  int wall[3];                 // non-periodic axis: a wall or a symmetry plane
  int sym;                     // symmetry planes: bit a = low side of axis a, bit 3 + a = high side
  int far;                     // far-field Dirichlet sides, bits as sym
  long long N;                 // nodes
  // population plane offsets (-1 = set inactive)
  int o_ns, o_phi, o_psi, o_c, o_th;
  int q_ns, q_phi, q_sc;
  // history plane offsets (-1 = absent)
  int h_psi, h_S, h_phiv, h_B, h_Hv;
  int first;                   // backward differences are zero on this step
  int nseed, nbub;
  // derived constants (lattice units)
  double W0, tau0, d_psi, eps4, k, D, alpha, inv_Le, Mcinf, lam, U0, theta0;
  double rho_l, rho_g, drho, mu_l, mu_g, W_phi, sharp, k_s, M_phi, beta_inter, g;
  double delta_n2, s_phi, s_th, a_at;
  double th_rho_g, th_cp_g, th_k_g;   // gas ratios of the heat properties
  double phi_tanh, psi_tanh;   // tanh arguments per unit distance of the initial profiles
  // device pointers inside the aux buffer
  const uint8_t* grain;        // nearest-seed id per node
  const double* grain_cs;      // cos, sin of each seed's angle
  const double* seeds;         // x, y, z, r, angle per seed
  const double* bubbles;       // x, y, z, r per bubble
  int fast;                    // byte offsets of every buffer fit in 32 bits
  int plane32;                 // byte offsets within one plane fit in 32 bits
  int zc;                      // 3D: z planes per workgroup chunk
  int le1;                     // AAC form for Le = O(1): a_n = a_s^2 F(U), no F in D_psi and S_psi
  int vel;                     // velocity sides, bits as sym (also set in far: psi, C, theta see a far-field side)
  double vin[3];               // velocity of the velocity sides
  int pres;                    // pressure sides (p = 0), bits as sym (also set in far)
  const void* hist_src;        // history read from here (null: the written buffer)
  int sr;                      // stochastic rounding of 16-bit stores
  int nt;                      // step stores non-temporal (streamed past the last-level cache)
  uint32_t step_ctr;           // step counter, part of the rounding key
  void* tape;                  // 2D: stencil results written here when set (TAPE_PLANES planes)
  uint32_t mmask;              // macro mode: planes written (bit k = macro k), packed in bit order
  int mf32;                    // macro mode: FP32 output (else FP64)
  uint32_t given;              // init from macros: input planes given (bit 0 phi .. 3 theta, 4 v)
  KP<double> kd;
  KP<float> kf;
  // rest equilibria r_i of the deviation storage (per set, per direction)
  double ref_ns[19], ref_phi[19], ref_psi[7], ref_c[7], ref_th[7];
};

// Whether the low (lo) or high boundary of axis a is a symmetry plane.
__device__ __forceinline__ bool sym_side(const DevParams& P, int a, bool lo) {
  return (P.sym >> (lo ? a : 3 + a)) & 1;
}
// Whether the low (lo) or high boundary of axis a is a far-field side.
__device__ __forceinline__ bool far_side(const DevParams& P, int a, bool lo) {
  return (P.far >> (lo ? a : 3 + a)) & 1;
}

// Macro mode of the step kernels: the planes of m (phi, psi, C, theta, U, p,
// v_x, v_y, v_z) selected by P.mmask, packed in that order, as FP64 or FP32.
__device__ __forceinline__ void put_macros(const DevParams& P, double* mout, long long idx, const double (&m)[9]) {
  int o = 0;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    if ((P.mmask >> k) & 1u) {
      if (P.mf32) ((float*)mout)[(long long)o * P.N + idx] = (float)m[k];
      else mout[(long long)o * P.N + idx] = m[k];
      ++o;
    }
  }
}

// --------------------------------------------------------- storage types
// FP32, FP16 and BF16 storage hold deviations f_i - r_i from the rest
// equilibrium r_i of the bulk liquid (phi = 1, psi = -1, C = C_ref,
// theta = theta0, v = p = 0); FP64 storage holds full populations (r_i = 0).
// The step kernel works on the stored values directly; the init and export
// kernels add or remove r_i.
// PCG hash (Jarzynski and Olano, "Hash Functions for GPU Rendering", JCGT
// 2020): one LCG step of PCG followed by its RXS-M-XS output permutation.
// A counter-based source of 32 random bits for stochastic rounding.
__device__ __forceinline__ uint32_t pcg_hash(uint32_t v) {
  const uint32_t s = v * 747796405u + 2891336453u;
  const uint32_t w = ((s >> ((s >> 28u) + 4u)) ^ s) * 277803737u;
  return (w >> 22u) ^ w;
}

// Stochastic rounding of an FP32 value to a format keeping the top 32 - D
// bits of its encoding: add D random bits to the magnitude bits and cut them
// off; the result rounds up with probability equal to the discarded fraction.
// Infinities pass unchanged (their low D bits are zero, so nothing carries).
// A NaN stays a NaN unless its mantissa lies within 2^D of all ones, which
// neither the default NaN of arithmetic nor a NaN loaded from 16-bit storage
// (low D bits zero) does.  For FP16, values below its normal range lose more
// than D bits and the conversion rounds the rest to nearest.
template <int D>
__device__ __forceinline__ uint32_t sround_bits(float v, uint32_t r) {
  constexpr uint32_t m = (1u << D) - 1u;
  return (__float_as_uint(v) + (r & m)) & ~m;
}

struct half_dev { __half v; };
struct bf16_dev { __hip_bfloat16 v; };

template <class ST> struct Store;
// Storage forms: ld/st convert between the stored value and the compute type;
// enc / enc_sr give the stored bits (16-bit forms: round to nearest /
// stochastically with the random bits r), written by the step's stores.
template <> struct Store<double> {
  using raw = double;
  using bits = double;
  template <class CT> __device__ static CT ld(const raw* p) { return (CT)(*p); }
  template <class CT> __device__ static void st(raw* p, CT v) { *p = (double)v; }
  template <class CT> __device__ static bits enc(CT v) { return (double)v; }
};
template <> struct Store<float> {
  using raw = float;
  using bits = float;
  template <class CT> __device__ static CT ld(const raw* p) { return (CT)(*p); }
  template <class CT> __device__ static void st(raw* p, CT v) { *p = (float)v; }
  template <class CT> __device__ static bits enc(CT v) { return (float)v; }
};
template <> struct Store<half_dev> {
  using raw = __half;
  using bits = unsigned short;
  template <class CT> __device__ static CT ld(const raw* p) { return (CT)__half2float(*p); }
  template <class CT> __device__ static void st(raw* p, CT v) { *p = __float2half_rn((float)v); }
  template <class CT> __device__ static bits enc(CT v) { return __half_as_ushort(__float2half_rn((float)v)); }
  template <class CT> __device__ static bits enc_sr(CT v, uint32_t r) {
    return __half_as_ushort(__float2half_rn(__uint_as_float(sround_bits<13>((float)v, r))));
  }
};
template <> struct Store<bf16_dev> {
  using raw = __hip_bfloat16;
  using bits = unsigned short;
  template <class CT> __device__ static CT ld(const raw* p) { return (CT)__bfloat162float(*p); }
  template <class CT> __device__ static void st(raw* p, CT v) { *p = __float2bfloat16((float)v); }
  template <class CT> __device__ static bits enc(CT v) { return __bfloat16_as_ushort(__float2bfloat16((float)v)); }
  template <class CT> __device__ static bits enc_sr(CT v, uint32_t r) {
    // the low 16 bits are zero after rounding: the top half is the BF16 value
    return (unsigned short)(sround_bits<16>((float)v, r) >> 16);
  }
};

template <class CT> __device__ __forceinline__ const KP<CT>& kp(const DevParams& P);
template <> __device__ __forceinline__ const KP<double>& kp<double>(const DevParams& P) { return P.kd; }
template <> __device__ __forceinline__ const KP<float>& kp<float>(const DevParams& P) { return P.kf; }

}  // namespace pfl
