// Initialisation, node-form state export/import and FP64 reductions, for
// 2D and 3D lattices.  None of these is on the per-step path.
#include "pfl_kernels.h"

#include <mutex>

namespace pfl {

namespace {

constexpr int BT = 256;

// Node-form slot of population i at node (x, y, z) in pull storage: the
// value is held at its source node x - c_i; when that source lies beyond a
// wall, in the node's own opposite slot; beyond a symmetry plane, at the
// mirror of the source as the population with that component reversed.
template <int Q>
__device__ __forceinline__ long long slot(const DevParams& P, int x, int y, int z, int i) {
  using L = Lat<Q>;
  int s[3] = {x - L::c[i][0], y - L::c[i][1], z - L::c[i][2]};
  const int n[3] = {P.nx, P.ny, P.nz};
  bool bounce = false;
  int fl[3] = {0, 0, 0};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (s[a] < 0 || s[a] >= n[a]) {
      if (!P.wall[a]) s[a] = s[a] < 0 ? s[a] + n[a] : s[a] - n[a];
      else if (sym_side(P, a, s[a] < 0)) { s[a] = s[a] < 0 ? -1 - s[a] : 2 * n[a] - 1 - s[a]; fl[a] = 1; }
      else bounce = true;
    }
  }
  if (bounce) return (long long)L::opp[i] * P.N + ((long long)z * P.ny + y) * P.nx + x;
  const int j = lat_reflected<Q>(i, fl[0], fl[1], fl[2]);
  return (long long)j * P.N + ((long long)s[2] * P.ny + s[1]) * P.nx + s[0];
}

// plane index (within a set) of a slot
__device__ __forceinline__ int plane_of(long long sl, long long N) { return (int)(sl / N); }

template <int Q, class ST>
__device__ void scatter_set(const DevParams& P, typename Store<ST>::raw* base, const double* ref,
                            int x, int y, int z, const double f[Q]) {
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const long long sl = slot<Q>(P, x, y, z, i);
    // population i of this node lands in plane i, opp(i) across a wall or
    // its reflection across a symmetry plane: a population of direction
    // plane_of(sl) at its slot
    Store<ST>::st(base + sl, f[i] - ref[i]);
  }
}

template <int Q, class ST>
__device__ void gather_set(const DevParams& P, const typename Store<ST>::raw* base, const double* ref,
                           int x, int y, int z, double f[Q]) {
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const long long sl = slot<Q>(P, x, y, z, i);
    f[i] = Store<ST>::template ld<double>(base + sl) + ref[i];
  }
}

__device__ __forceinline__ double pdist2(const DevParams& P, const double* X, const double* c) {
  const int n[3] = {P.nx, P.ny, P.nz};
  double d2 = 0.0;
  for (int a = 0; a < P.dim; ++a) {
    double dd = fabs(X[a] - c[a]);
    if (!P.wall[a]) dd = fmin(dd, (double)n[a] - dd);
    d2 = d2 + dd * dd;
  }
  return d2;
}

template <int QN, int QP, int QS, class ST, class HT>
__global__ __launch_bounds__(BT) void init_kernel(const DevParams P, int fields, int mode,
                                                  const double* __restrict__ macros,
                                                  typename Store<ST>::raw* __restrict__ pops,
                                                  HT* __restrict__ hist, int hist_planes,
                                                  uint8_t* __restrict__ grain) {
  const long long n = (long long)blockIdx.x * BT + threadIdx.x;
  if (n >= P.N) return;
  const int x = (int)(n % P.nx);
  const int y = (int)((n / P.nx) % P.ny);
  const int z = (int)(n / ((long long)P.nx * P.ny));
  const double X[3] = {(double)x, (double)y, (double)z};
  // nearest seed (ties to the lowest index) and signed distance to seeds
  int gid = 0;
  double best = 0.0, ds = 0.0;
  for (int s = 0; s < P.nseed; ++s) {
    const double* S = P.seeds + 5 * s;
    const double d2 = pdist2(P, X, S);
    const double d = sqrt(d2) - S[3];
    if (s == 0 || d2 < best) { best = d2; gid = s; }
    ds = (s == 0) ? d : fmin(ds, d);
  }
  grain[n] = (uint8_t)gid;
  double phi, psi, C, theta, v[3] = {0.0, 0.0, 0.0};
  if (mode == 0) {
    phi = 1.0;
    if ((fields & F_PHI) && P.nbub > 0) {
      double db = 0.0;
      for (int b = 0; b < P.nbub; ++b) {
        const double* B = P.bubbles + 4 * b;
        const double d = sqrt(pdist2(P, X, B)) - B[3];
        db = (b == 0) ? d : fmin(db, d);
      }
      phi = 0.5 + 0.5 * tanh(P.phi_tanh * db);
    }
    psi = -1.0;
    if ((fields & F_PSI) && P.nseed > 0) psi = tanh(P.psi_tanh * (-ds));
    const double h = (psi + 1.0) * 0.5;
    C = phi * (1.0 + (1.0 - P.k) * P.U0) * (1.0 - (1.0 - P.k) * h);
    theta = P.theta0;
  } else {
    // planes not given: the bulk liquid at rest, with the partitioned
    // solute profile of the given phi and psi
    phi = (P.given & 1u) ? macros[0 * P.N + n] : 1.0;
    psi = (P.given & 2u) ? macros[1 * P.N + n] : -1.0;
    const double h0 = (psi + 1.0) * 0.5;
    C = (P.given & 4u) ? macros[2 * P.N + n] : phi * (1.0 + (1.0 - P.k) * P.U0) * (1.0 - (1.0 - P.k) * h0);
    theta = (P.given & 8u) ? macros[3 * P.N + n] : P.theta0;
    if (P.given & 16u)
      for (int a = 0; a < P.dim; ++a) v[a] = macros[(4 + a) * P.N + n];
  }
  const double h = (psi + 1.0) * 0.5;
  if (fields & F_NS) {
    using L = Lat<QN>;
    const double rho = P.rho_g + P.drho * phi;
    const double vv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    double f[QN];
    for (int i = 0; i < QN; ++i) {
      const double cv = L::c[i][0] * v[0] + L::c[i][1] * v[1] + L::c[i][2] * v[2];
      f[i] = L::w[i] * rho * (cv / L::cs2 + cv * cv / (2.0 * L::cs2 * L::cs2) - vv / (2.0 * L::cs2));
    }
    scatter_set<QN, ST>(P, pops + (long long)P.o_ns * P.N, P.ref_ns, x, y, z, f);
  }
  if (fields & F_PHI) {
    using L = Lat<QP>;
    double f[QP];
    for (int i = 0; i < QP; ++i) f[i] = L::w[i] * phi;
    scatter_set<QP, ST>(P, pops + (long long)P.o_phi * P.N, P.ref_phi, x, y, z, f);
  }
  using LS = Lat<QS>;
  if (fields & F_PSI) {
    double f[QS];
    for (int i = 0; i < QS; ++i) f[i] = LS::w[i] * psi;
    scatter_set<QS, ST>(P, pops + (long long)P.o_psi * P.N, P.ref_psi, x, y, z, f);
  }
  if (fields & F_C) {
    double f[QS];
    for (int i = 0; i < QS; ++i) f[i] = LS::w[i] * C;
    scatter_set<QS, ST>(P, pops + (long long)P.o_c * P.N, P.ref_c, x, y, z, f);
  }
  if (fields & F_TH) {
    double f[QS];
    for (int i = 0; i < QS; ++i) f[i] = LS::w[i] * theta;
    // rest population rho H + (w_0 - 1) theta, H = c_p theta - h (rho, c_p
    // linear in phi, liquid = solid = 1)
    const double rh = P.th_rho_g + (1.0 - P.th_rho_g) * phi;
    const double cp = P.th_cp_g + (1.0 - P.th_cp_g) * phi;
    f[0] = rh * (cp * theta - h) + (LS::w[0] - 1.0) * theta;
    scatter_set<QS, ST>(P, pops + (long long)P.o_th * P.N, P.ref_th, x, y, z, f);
  }
  for (int hp = 0; hp < hist_planes; ++hp) hist[(long long)hp * P.N + n] = (HT)0;
}

template <int QN, int QP, int QS, class ST, class HT>
__global__ __launch_bounds__(BT) void state_kernel(const DevParams P, int fields, int dir,
                                                   typename Store<ST>::raw* __restrict__ pops,
                                                   HT* __restrict__ hist, int hist_planes,
                                                   double* __restrict__ node) {
  const long long n = (long long)blockIdx.x * BT + threadIdx.x;
  if (n >= P.N) return;
  const int x = (int)(n % P.nx);
  const int y = (int)((n / P.nx) % P.ny);
  const int z = (int)(n / ((long long)P.nx * P.ny));
  long long plane = 0;
  auto set = [&](auto qtag, int off, const double* ref) {
    constexpr int Q = decltype(qtag)::value;
    double f[Q];
    if (dir == 0) {
      gather_set<Q, ST>(P, pops + (long long)off * P.N, ref, x, y, z, f);
      for (int i = 0; i < Q; ++i) node[(plane + i) * P.N + n] = f[i];
    } else {
      for (int i = 0; i < Q; ++i) f[i] = node[(plane + i) * P.N + n];
      scatter_set<Q, ST>(P, pops + (long long)off * P.N, ref, x, y, z, f);
    }
    plane += Q;
  };
  if (fields & F_NS) set(std::integral_constant<int, QN>{}, P.o_ns, P.ref_ns);
  if (fields & F_PHI) set(std::integral_constant<int, QP>{}, P.o_phi, P.ref_phi);
  if (fields & F_PSI) set(std::integral_constant<int, QS>{}, P.o_psi, P.ref_psi);
  if (fields & F_C) set(std::integral_constant<int, QS>{}, P.o_c, P.ref_c);
  if (fields & F_TH) set(std::integral_constant<int, QS>{}, P.o_th, P.ref_th);
  for (int hp = 0; hp < hist_planes; ++hp) {
    if (dir == 0) node[(plane + hp) * P.N + n] = (double)hist[(long long)hp * P.N + n];
    else hist[(long long)hp * P.N + n] = (HT)node[(plane + hp) * P.N + n];
  }
}

template <int QN, int QP, int QS, class ST, class HT>
__global__ __launch_bounds__(BT) void reduce_kernel(const DevParams P, int fields,
                                                    const typename Store<ST>::raw* __restrict__ pops,
                                                    const HT* __restrict__ hist, int hist_planes,
                                                    double* __restrict__ red) {
  double acc[RED_VALS] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (long long n = (long long)blockIdx.x * BT + threadIdx.x; n < P.N; n += (long long)gridDim.x * BT) {
    const int x = (int)(n % P.nx);
    const int y = (int)((n / P.nx) % P.ny);
    const int z = (int)(n / ((long long)P.nx * P.ny));
    bool bad = false;
    double phi = 1.0, psi = -1.0, C = 0.0;
    auto zeroth = [&](auto qtag, int off, const double* ref) {
      constexpr int Q = decltype(qtag)::value;
      double f[Q];
      gather_set<Q, ST>(P, pops + (long long)off * P.N, ref, x, y, z, f);
      double s = 0.0;
      for (int i = 0; i < Q; ++i) { s += f[i]; bad = bad || !isfinite(f[i]); }
      return s;
    };
    if (fields & F_NS) zeroth(std::integral_constant<int, QN>{}, P.o_ns, P.ref_ns);
    if (fields & F_PHI) phi = zeroth(std::integral_constant<int, QP>{}, P.o_phi, P.ref_phi);
    if (fields & F_PSI) psi = zeroth(std::integral_constant<int, QS>{}, P.o_psi, P.ref_psi);
    if (fields & F_C) C = zeroth(std::integral_constant<int, QS>{}, P.o_c, P.ref_c);
    if (fields & F_TH) zeroth(std::integral_constant<int, QS>{}, P.o_th, P.ref_th);
    for (int hp = 0; hp < hist_planes; ++hp) bad = bad || !isfinite((double)hist[(long long)hp * P.N + n]);
    const double gas = 1.0 - phi;
    acc[0] += phi;
    acc[1] += gas;
    acc[2] += C;
    acc[3] += (psi + 1.0) * 0.5;
    acc[4] += gas * x;
    acc[5] += gas * y;
    acc[6] += gas * z;
    acc[7] += bad ? 1.0 : 0.0;
  }
  // wave64 shuffle, then across the block's waves in LDS (fixed order)
  __shared__ double s_acc[BT / 64][RED_VALS];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int v = 0; v < RED_VALS; ++v) {
    double a = acc[v];
    for (int off = 32; off > 0; off >>= 1) a += __shfl_down(a, off, 64);
    if (lane == 0) s_acc[wave][v] = a;
  }
  __syncthreads();
  if (threadIdx.x < RED_VALS) {
    double a = 0.0;
    for (int w = 0; w < BT / 64; ++w) a += s_acc[w][threadIdx.x];
    red[(long long)blockIdx.x * RED_VALS + threadIdx.x] = a;
  }
}

__global__ void reduce_final(double* red) {
  // one wave; lane v < RED_VALS sums the per-block partials in block order
  const int v = threadIdx.x;
  if (v >= RED_VALS) return;
  double a = 0.0;
  for (int b = 0; b < RED_BLOCKS; ++b) a += red[(long long)b * RED_VALS + v];
  red[(long long)RED_BLOCKS * RED_VALS + v] = a;
}

// In-step checks of pfl_step: the check area after the reduction's final
// values holds the first failing step (INT64_MAX if none), the step of the
// last check and that check's final values.
__global__ void check_reset(double* red) {
  long long* ck = (long long*)(red + (size_t)(RED_BLOCKS + 1) * RED_VALS);
  if (threadIdx.x == 0) {
    ck[0] = 0x7fffffffffffffffLL;
    ck[1] = -1;
  }
}

__global__ void check_record(double* red, long long step) {
  const int v = threadIdx.x;
  const double* fin = red + (size_t)RED_BLOCKS * RED_VALS;
  long long* ck = (long long*)(red + (size_t)(RED_BLOCKS + 1) * RED_VALS);
  double* diag = (double*)(ck + 2);
  if (v < RED_VALS) diag[v] = fin[v];
  if (v == 0) {
    ck[1] = step;
    const bool bad = fin[7] != 0.0 || !isfinite(fin[0]) || !isfinite(fin[2]);
    if (bad && ck[0] > step) ck[0] = step;
  }
}

// Adjoint of the zeroth moments: every population of a set whose sum is
// seeded takes dL/d(sum); other entries zero.
template <class AT>
__global__ __launch_bounds__(BT) void seed_kernel(const DevParams P, int fields, const double* __restrict__ dL,
                                                  uint32_t mask, AT* __restrict__ out, int planes) {
  const long long n = (long long)blockIdx.x * BT + threadIdx.x;
  if (n >= P.N) return;
  int plane = 0;
  auto set = [&](int q, bool on, int bit) {
    AT v = AT(0);
    if (on && ((mask >> bit) & 1u)) v = (AT)dL[(long long)__popc(mask & ((1u << bit) - 1u)) * P.N + n];
    for (int i = 0; i < q; ++i) out[(long long)(plane + i) * P.N + n] = v;
    plane += q;
  };
  if (fields & F_NS) set(P.q_ns, false, 0);
  if (fields & F_PHI) set(P.q_phi, true, 0);
  if (fields & F_PSI) set(P.q_sc, true, 1);
  if (fields & F_C) set(P.q_sc, true, 2);
  if (fields & F_TH) set(P.q_sc, false, 0);
  for (; plane < planes; ++plane) out[(long long)plane * P.N + n] = AT(0);
}

template <class ST, class HT>
struct Disp {
  template <int QN, int QP, int QS>
  static hipError_t init(const DevParams& P, int fields, int mode, const double* m, void* pops,
                         void* hist, int hp, uint8_t* grain, hipStream_t s) {
    const unsigned nb = (unsigned)((P.N + BT - 1) / BT);
    hipLaunchKernelGGL((init_kernel<QN, QP, QS, ST, HT>), dim3(nb), dim3(BT), 0, s, P, fields, mode, m,
                       (typename Store<ST>::raw*)pops, (HT*)hist, hp, grain);
    return hipGetLastError();
  }
  template <int QN, int QP, int QS>
  static hipError_t state(const DevParams& P, int fields, int dir, void* pops, void* hist, int hp,
                          double* node, hipStream_t s) {
    const unsigned nb = (unsigned)((P.N + BT - 1) / BT);
    hipLaunchKernelGGL((state_kernel<QN, QP, QS, ST, HT>), dim3(nb), dim3(BT), 0, s, P, fields, dir,
                       (typename Store<ST>::raw*)pops, (HT*)hist, hp, node);
    return hipGetLastError();
  }
  template <int QN, int QP, int QS>
  static hipError_t reduce(const DevParams& P, int fields, const void* pops, const void* hist, int hp,
                           double* red, hipStream_t s) {
    hipLaunchKernelGGL((reduce_kernel<QN, QP, QS, ST, HT>), dim3(RED_BLOCKS), dim3(BT), 0, s, P, fields,
                       (const typename Store<ST>::raw*)pops, (const HT*)hist, hp, red);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(reduce_final, dim3(1), dim3(64), 0, s, red);
    return hipGetLastError();
  }
};

int hist_planes_of(const DevParams& P, int fields) {
  int h = 0;
  if (fields & F_PSI) h += 2;
  if (fields & F_PHI) h += P.dim;
  if (fields & F_C) h += P.dim;
  if (fields & F_TH) h += P.dim;
  return h;
}

// Calls fn.template run<QN,QP,QS>() on the lattice combination of P.
template <class ST, class HT, class Fn>
hipError_t by_lattice(const DevParams& P, Fn&& fn) {
  if (P.dim == 2) {
    if (P.q_phi == 9) return fn.template operator()<ST, HT, 9, 9, 5>();
    return fn.template operator()<ST, HT, 9, 5, 5>();
  }
  return fn.template operator()<ST, HT, 19, 7, 7>();
}

template <class Fn>
hipError_t by_store(int store, const DevParams& P, Fn&& fn) {
  switch (store) {
    case 0: return by_lattice<double, double>(P, fn);
    case 1: return by_lattice<float, float>(P, fn);
    case 2: return by_lattice<half_dev, float>(P, fn);
    case 3: return by_lattice<bf16_dev, float>(P, fn);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_init(const DevParams& P, int fields, int store, int mode, const double* macros,
                       void* pops, void* hist, uint8_t* grain, hipStream_t s) {
  const int hp = hist_planes_of(P, fields);
  return by_store(store, P, [&]<class ST, class HT, int QN, int QP, int QS>() {
    return Disp<ST, HT>::template init<QN, QP, QS>(P, fields, mode, macros, pops, hist, hp, grain, s);
  });
}

hipError_t launch_get_state(const DevParams& P, int fields, int store, const void* pops,
                            const void* hist, double* out, hipStream_t s) {
  const int hp = hist_planes_of(P, fields);
  return by_store(store, P, [&]<class ST, class HT, int QN, int QP, int QS>() {
    return Disp<ST, HT>::template state<QN, QP, QS>(P, fields, 0, const_cast<void*>(pops),
                                                   const_cast<void*>(hist), hp, out, s);
  });
}

hipError_t launch_set_state(const DevParams& P, int fields, int store, const double* in, void* pops,
                            void* hist, hipStream_t s) {
  const int hp = hist_planes_of(P, fields);
  return by_store(store, P, [&]<class ST, class HT, int QN, int QP, int QS>() {
    return Disp<ST, HT>::template state<QN, QP, QS>(P, fields, 1, pops, hist, hp,
                                                   const_cast<double*>(in), s);
  });
}

hipError_t launch_check_reset(double* red, hipStream_t s) {
  hipLaunchKernelGGL(check_reset, dim3(1), dim3(64), 0, s, red);
  return hipGetLastError();
}

hipError_t launch_check_record(double* red, long long step, hipStream_t s) {
  hipLaunchKernelGGL(check_record, dim3(1), dim3(64), 0, s, red, step);
  return hipGetLastError();
}

hipError_t launch_adjoint_seed(const DevParams& P, int fields, int store, const double* dL, uint32_t mask,
                               void* out, int planes, hipStream_t s) {
  const unsigned nb = (unsigned)((P.N + BT - 1) / BT);
  if (store == 0)
    hipLaunchKernelGGL((seed_kernel<double>), dim3(nb), dim3(BT), 0, s, P, fields, dL, mask, (double*)out, planes);
  else
    hipLaunchKernelGGL((seed_kernel<float>), dim3(nb), dim3(BT), 0, s, P, fields, dL, mask, (float*)out, planes);
  return hipGetLastError();
}

// Partials and final values of the allocation-free reduction
// (pfl_reduce_noalloc): one array per GPU, held until the process ends.
// Every call on a GPU shares it, so calls that overlap on one GPU race.
static __device__ __align__(256) double scratch[REDUCE_SCRATCH_DOUBLES];

namespace {
std::mutex g_scratch_mu;
double* g_scratch_ptr[MAX_DEVICES] = {};
}  // namespace

hipError_t resolve_reduce_scratch(int device) {
  if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  // the array's name is a host-side stand-in; its device address on the
  // current device comes from the runtime
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[device] = (double*)ptr;
  return hipSuccess;
}

double* reduce_scratch(int device) {
  if (device < 0 || device >= MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_ptr[device];
}

hipError_t launch_reduce(const DevParams& P, int fields, int store, const void* pops,
                         const void* hist, int hist_planes, double* red, hipStream_t s) {
  return by_store(store, P, [&]<class ST, class HT, int QN, int QP, int QS>() {
    return Disp<ST, HT>::template reduce<QN, QP, QS>(P, fields, pops, hist, hist_planes, red, s);
  });
}

}  // namespace pfl
