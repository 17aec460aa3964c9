// Device helpers shared by the 2D and 3D step kernels: reciprocals, clamps,
// wall/periodic coordinate mapping, byte addressing, XCD-aware tile order.
#pragma once
#include "pfl_dev.h"

namespace pfl {

template <class CT>
__device__ __forceinline__ CT clamp01(CT v) { return v < CT(0) ? CT(0) : (v > CT(1) ? CT(1) : v); }

// Reciprocal and inverse square root: correctly rounded in FP64 (the parity
// path), the hardware approximations (1 ulp) in FP32.
__device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rsq(double x) { return 1.0 / sqrt(x); }
__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }

// XCD-aware tile order.  Workgroups are dispatched round-robin over the 8
// XCDs (workgroup b runs on XCD b mod 8), and each XCD has its own L2.  Give
// XCD k a contiguous range of logical tiles in row-major order (x fastest),
// i.e. a band of the grid, so tiles that share halo rows run on the same XCD
// at about the same time.  Returns the logical tile index of workgroup b out
// of T tiles.
constexpr int NXCD = 8;
__device__ __forceinline__ int logical_tile(int b, int T) {
  const int q = T / NXCD, r = T % NXCD;
  const int k = b % NXCD, j = b / NXCD;
  return k * q + (k < r ? k : r) + j;
}

// Map a (possibly out-of-domain) coordinate to the node whose value it
// holds: periodic wrap, or mirror across a half-way wall (clamped so that
// positions no valid node needs stay in range).
__device__ __forceinline__ int map_coord(int g, int n, int wall) {
  if (g >= 0 && g < n) return g;
  if (!wall) { g %= n; if (g < 0) g += n; return g; }
  g = g < 0 ? -1 - g : 2 * n - 1 - g;
  return g < 0 ? 0 : (g >= n ? n - 1 : g);
}

template <class ST>
__device__ __forceinline__ const typename Store<ST>::raw* at_byte(const typename Store<ST>::raw* base, uint32_t b) {
  return (const typename Store<ST>::raw*)((const char*)base + b);
}
template <class ST>
__device__ __forceinline__ typename Store<ST>::raw* at_byte(typename Store<ST>::raw* base, uint32_t b) {
  return (typename Store<ST>::raw*)((char*)base + b);
}

// Store of one post-collision value: 16-bit storage rounds stochastically
// when P.sr is set, keyed on (node, step, plane).
template <class ST, class CT>
__device__ __forceinline__ void store_pop(const DevParams& P, typename Store<ST>::raw* p, CT v,
                                          uint32_t hnode, int plane) {
  if constexpr (sizeof(typename Store<ST>::raw) == 2) {
    if (P.sr) { Store<ST>::st_sr(p, v, pcg_hash(hnode + (uint32_t)plane)); return; }
  }
  Store<ST>::st(p, v);
}

}  // namespace pfl
