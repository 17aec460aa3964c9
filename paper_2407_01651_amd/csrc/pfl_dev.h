// Device-side definitions shared by the step, init, export and reduction
// kernels: lattice tables, the parameter block passed by value to every
// kernel, storage conversions.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <hip/hip_bf16.h>
#include <cstdint>

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
  static constexpr double w[5] = {1.0/3, 1.0/6, 1.0/6, 1.0/6, 1.0/6};
  static constexpr double cs2 = 1.0/3;
  static constexpr double flux_norm = 2.0;   // sum_i c_ia^2
};

template <> struct Lat<9> {
  static constexpr int Q = 9, D = 2;
  static constexpr int c[9][3] = {{0,0,0},{1,0,0},{0,1,0},{-1,0,0},{0,-1,0},
                                  {1,1,0},{-1,1,0},{-1,-1,0},{1,-1,0}};
  static constexpr int opp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
  static constexpr double w[9] = {4.0/9, 1.0/9, 1.0/9, 1.0/9, 1.0/9,
                                  1.0/36, 1.0/36, 1.0/36, 1.0/36};
  static constexpr double cs2 = 1.0/3;
  static constexpr double flux_norm = 6.0;
};

template <> struct Lat<7> {
  static constexpr int Q = 7, D = 3;
  static constexpr int c[7][3] = {{0,0,0},{1,0,0},{-1,0,0},{0,1,0},{0,-1,0},{0,0,1},{0,0,-1}};
  static constexpr int opp[7] = {0, 2, 1, 4, 3, 6, 5};
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
  static constexpr double w[19] = {1.0/3, 1.0/18, 1.0/18, 1.0/18, 1.0/18, 1.0/18, 1.0/18,
                                   1.0/36, 1.0/36, 1.0/36, 1.0/36, 1.0/36, 1.0/36,
                                   1.0/36, 1.0/36, 1.0/36, 1.0/36, 1.0/36, 1.0/36};
  static constexpr double cs2 = 1.0/3;
  static constexpr double flux_norm = 10.0;
};

// ------------------------------------------------------------- parameters
// Constants of the step in the compute precision, reciprocals precomputed.
template <class CT>
struct KP {
  CT k1, inv_k1, U0, theta0, eps4, dn, d_psi, inv_tau0, D, lam, Mcinf, inv_Le, beta_inter;
  CT sharp, M_phi, Wphi2, k_s, rho_l, rho_g, drho, mu_l, mu_g, g, s_phi, s_th, aW0;
};

// Everything a kernel needs, passed by value (well under the 4 KB limit).
struct DevParams {
  int nx, ny, nz, dim;
  int wall[3];
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
  double phi_tanh, psi_tanh;   // tanh arguments per unit distance of the initial profiles
  // device pointers inside the aux buffer
  const uint8_t* grain;        // nearest-seed id per node
  const double* grain_cs;      // cos, sin of each seed's angle
  const double* seeds;         // x, y, z, r, angle per seed
  const double* bubbles;       // x, y, z, r per bubble
  int fast;                    // byte offsets of every buffer fit in 32 bits
  KP<double> kd;
  KP<float> kf;
  // reference populations of the deviation storage (per set, per direction)
  float ref_ns[19], ref_phi[19], ref_psi[7], ref_c[7], ref_th[7];
};

// --------------------------------------------------------- storage types
// FP16/BF16 hold deviations from a per-direction reference value.
struct half_dev { __half v; };
struct bf16_dev { __hip_bfloat16 v; };

template <class ST> struct Store;
template <> struct Store<double> {
  using raw = double;
  template <class CT> __device__ static CT ld(const raw* p, float) { return (CT)(*p); }
  template <class CT> __device__ static void st(raw* p, CT v, float) { *p = (double)v; }
};
template <> struct Store<float> {
  using raw = float;
  template <class CT> __device__ static CT ld(const raw* p, float) { return (CT)(*p); }
  template <class CT> __device__ static void st(raw* p, CT v, float) { *p = (float)v; }
};
template <> struct Store<half_dev> {
  using raw = __half;
  template <class CT> __device__ static CT ld(const raw* p, float ref) {
    return (CT)(__half2float(*p) + ref);
  }
  template <class CT> __device__ static void st(raw* p, CT v, float ref) {
    *p = __float2half_rn((float)v - ref);
  }
};
template <> struct Store<bf16_dev> {
  using raw = __hip_bfloat16;
  template <class CT> __device__ static CT ld(const raw* p, float ref) {
    return (CT)(__bfloat162float(*p) + ref);
  }
  template <class CT> __device__ static void st(raw* p, CT v, float ref) {
    *p = __float2bfloat16((float)v - ref);
  }
};

template <class CT> __device__ __forceinline__ const KP<CT>& kp(const DevParams& P);
template <> __device__ __forceinline__ const KP<double>& kp<double>(const DevParams& P) { return P.kd; }
template <> __device__ __forceinline__ const KP<float>& kp<float>(const DevParams& P) { return P.kf; }

}  // namespace pfl
