// Discrete adjoint of the fused 2D step: FP64 instantiations, the initial-
// state adjoint, and the dispatch over storage types (the FP32-compute
// instantiations live in pfl_adj2d_lowp.hip).
#include "pfl_adj2d_impl.h"

namespace pfl {

namespace {

// ------------------------------------------------------------ initial state
// Gradient of lambda^0 . x^0 with respect to k, Omega and the bubble radii,
// through the initial profiles of init_fields: phi = 1/2 + 1/2 tanh(a d_b)
// with d_b the distance to the nearest bubble surface, C = phi (1 + (1-k) U0)
// (1 - (1-k) h), theta = theta0 (Omega enters as theta0 = -Omega with the heat
// equation, as U0 = -Omega without it).  Per node the contributions go to
// planes: [k1, Omega, radius of the nearest bubble] and the bubble id.
template <int QP, class AT>
__global__ __launch_bounds__(256) void adj_init_kernel(const DevParams P, int fields,
                                                       const AT* __restrict__ lam0,
                                                       double* __restrict__ S) {
  using LP = Lat<QP>;
  using LS = Lat<5>;
  const long long n = (long long)blockIdx.x * 256 + threadIdx.x;
  if (n >= P.N) return;
  const long long N = P.N;
  const int x = (int)(n % P.nx), y = (int)(n / P.nx);
  const double X[2] = {(double)x, (double)y};
  auto dist = [&](const double* c) {
    double d2 = 0.0;
    const int nn[2] = {P.nx, P.ny};
    for (int a = 0; a < 2; ++a) {
      double dd = fabs(X[a] - c[a]);
      if (!P.wall[a]) dd = fmin(dd, (double)nn[a] - dd);
      d2 += dd * dd;
    }
    return sqrt(d2);
  };
  double ds = 0.0;
  for (int s = 0; s < P.nseed; ++s) {
    const double d = dist(P.seeds + 5 * s) - P.seeds[5 * s + 3];
    ds = (s == 0) ? d : fmin(ds, d);
  }
  double phi = 1.0, dphi_dR = 0.0;
  int bid = -1;
  if ((fields & F_PHI) && P.nbub > 0) {
    double db = 0.0;
    for (int b = 0; b < P.nbub; ++b) {
      const double d = dist(P.bubbles + 4 * b) - P.bubbles[4 * b + 3];
      if (b == 0 || d < db) { db = d; bid = b; }
    }
    const double t = tanh(P.phi_tanh * db);
    phi = 0.5 + 0.5 * t;
    dphi_dR = -0.5 * P.phi_tanh * (1.0 - t * t);
  }
  const double psi = ((fields & F_PSI) && P.nseed > 0) ? tanh(P.psi_tanh * (-ds)) : -1.0;
  const double h = (psi + 1.0) * 0.5;
  const double k1 = P.kd.k1, U0 = P.U0;
  double lphi = 0.0, lC = 0.0, lth = 0.0;
  if (fields & F_PHI) {
#pragma unroll
    for (int i = 0; i < QP; ++i) lphi += (double)lam0[(long long)(P.o_phi + i) * N + n] * LP::w[i];
  }
  if (fields & F_C) {
#pragma unroll
    for (int i = 0; i < 5; ++i) lC += (double)lam0[(long long)(P.o_c + i) * N + n] * LS::w[i];
  }
  if (fields & F_TH) {
#pragma unroll
    for (int i = 0; i < 5; ++i) lth += (double)lam0[(long long)(P.o_th + i) * N + n] * LS::w[i];
  }
  const double cfac = (1.0 + k1 * U0) * (1.0 - k1 * h);
  double gR = (lphi + lC * cfac) * dphi_dR;
  double gk1 = lC * phi * (U0 * (1.0 - k1 * h) - h * (1.0 + k1 * U0));
  double gOm = (fields & F_TH) ? -lth : -lC * phi * k1 * (1.0 - k1 * h);
  if ((fields & F_TH) && P.kd.varheat) {
    // rest population rho (c_p theta0 - h) + (w_0 - 1) theta0, rho and c_p linear in phi
    const double l0 = (double)lam0[(long long)P.o_th * N + n];
    const double rh = P.th_rho_g + (1.0 - P.th_rho_g) * phi, cp = P.th_cp_g + (1.0 - P.th_cp_g) * phi;
    gOm -= l0 * (rh * cp - 1.0);
    gR += l0 * ((1.0 - P.th_rho_g) * (cp * P.theta0 - h) + rh * (1.0 - P.th_cp_g) * P.theta0) * dphi_dR;
  }
  S[0 * N + n] = gk1;
  S[1 * N + n] = gOm;
  S[2 * N + n] = gR;
  S[3 * N + n] = (double)bid;
}

__global__ __launch_bounds__(256) void adj_init_sum_kernel(long long N, const double* __restrict__ S,
                                                           int nbub, double* __restrict__ dparams) {
  // block 0: k (= -k1 gradient), block 1: Omega, block 2 + b: radius of bubble b
  const int b = blockIdx.x;
  double a = 0.0;
  for (long long n = threadIdx.x; n < N; n += 256) {
    if (b == 0) a += S[n];
    else if (b == 1) a += S[N + n];
    else if ((int)S[3 * N + n] == b - 2) a += S[2 * N + n];
  }
  __shared__ double s[256];
  s[threadIdx.x] = a;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (b == 0) dparams[1] -= s[0];
    else if (b == 1) dparams[2] += s[0];
    else dparams[3 + (b - 2)] += s[0];
  }
}

}  // namespace


size_t adj_scratch_bytes(int nx, int ny, int store) {
  const long long N = (long long)nx * ny;
  const size_t elem = store == 0 ? sizeof(double) : sizeof(float);
  // partial slots: one per 256 nodes, or one per tile of the fused flow pass
  const size_t nb = (size_t)((N + 255) / 256);
  const size_t tiles = (size_t)((nx + TX - 1) / TX) * (size_t)((ny + TY - 1) / TY);
  const size_t bytes = part_offset(N, elem) + 3 * (nb > tiles ? nb : tiles) * sizeof(double);
  // the initial-state adjoint uses four FP64 planes of the same buffer
  const size_t init = 4 * (size_t)N * sizeof(double);
  return bytes > init ? bytes : init;
}

bool adj2d_supported(int fields) {
  switch (fields) {
    case F_NS | F_PHI | F_PSI | F_C | F_TH:
    case F_PSI | F_C:
    case F_PSI | F_C | F_TH:
    case F_NS | F_PHI:
    case F_PHI | F_PSI | F_C | F_TH:
    case F_PHI:
    case F_NS | F_PSI | F_TH:
    case F_PSI | F_TH:
    case F_PSI:
      return true;
    default:
      return false;
  }
}

hipError_t launch_adj_step2d(const DevParams& P, int fields, int store, const void* fin, const void* hist,
                             const void* tape, const void* lam_in, void* lam_out, void* scratch,
                             double* dparams, hipStream_t s, bool& ok, const AdjOpts& o) {
  hipError_t e;
  switch (store) {
    case 0:
      e = adj_dispatch<double, double>(P, fields, fin, hist, tape, lam_in, lam_out, scratch, dparams, s, o, ok);
      break;
    case 1:
    case 2:
    case 3:
      return launch_adj_step2d_lowp(P, fields, store, fin, hist, tape, lam_in, lam_out, scratch, dparams, s, ok, o);
    default: ok = false; return hipSuccess;
  }
  return e;
}

hipError_t launch_adj_init2d(const DevParams& P, int fields, int store, const void* lam0, void* scratch,
                             double* dparams, hipStream_t s) {
  const unsigned nb = (unsigned)((P.N + 255) / 256);
  double* S = (double*)scratch;
  if (store == 0) {
    if (P.q_phi == 9)
      hipLaunchKernelGGL((adj_init_kernel<9, double>), dim3(nb), dim3(256), 0, s, P, fields, (const double*)lam0, S);
    else
      hipLaunchKernelGGL((adj_init_kernel<5, double>), dim3(nb), dim3(256), 0, s, P, fields, (const double*)lam0, S);
  } else {
    if (P.q_phi == 9)
      hipLaunchKernelGGL((adj_init_kernel<9, float>), dim3(nb), dim3(256), 0, s, P, fields, (const float*)lam0, S);
    else
      hipLaunchKernelGGL((adj_init_kernel<5, float>), dim3(nb), dim3(256), 0, s, P, fields, (const float*)lam0, S);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(adj_init_sum_kernel, dim3(2 + P.nbub), dim3(256), 0, s, P.N, S, P.nbub, dparams);
  return hipGetLastError();
}

}  // namespace pfl
