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

// Two values read from 16-bit storage, kept as their stored bits in one
// register (exact: each is a value of the storage type), and one of them back.
template <class ST>
__device__ __forceinline__ uint32_t keep16(float a, float b) {
  return (uint32_t)Store<ST>::enc(a) | ((uint32_t)Store<ST>::enc(b) << 16);
}
template <class ST>
__device__ __forceinline__ float unkeep16(uint32_t w, int hi) {
  using raw = typename Store<ST>::raw;
  const raw r = __builtin_bit_cast(raw, (unsigned short)(hi ? w >> 16 : w & 0xffffu));
  return Store<ST>::template ld<float>(&r);
}

// Random bits for the stochastic rounding of one node's stores.  The seed is
// the PCG hash of (node, step); population i of a set takes the 16-bit half
// i mod 2 of the PCG hash of the Weyl sequence entry seed + (i/2 + 1) * g
// (g the 32-bit golden ratio), so runs are reproducible.  All sets of the node
// take the bits of their population index: every population of a set has
// bits of its own, and no conserved sum mixes sets.  (A xorshift32 stream
// from the same seed was cheaper but its correlated outputs gave about 1.6
// times the spread of the conserved-mass random walk.)
template <int NH>
struct RoundBits {
  uint32_t h[NH];
  __device__ RoundBits(uint32_t seed, bool on) {
    if (on) {
#pragma unroll
      for (int j = 0; j < NH; ++j) h[j] = pcg_hash(seed + (uint32_t)(j + 1) * 0x9E3779B9u);
    } else {
#pragma unroll
      for (int j = 0; j < NH; ++j) h[j] = 0u;
    }
  }
  // 16 bits for population i of a set (i a compile-time index)
  __device__ __forceinline__ uint32_t bits(int i) const {
    return (i & 1) ? (h[i >> 1] >> 16) : (h[i >> 1] & 0xFFFFu);
  }
};

__device__ __forceinline__ uint32_t round_seed(const DevParams& P, uint32_t node) {
  return pcg_hash(node ^ pcg_hash(P.step_ctr));
}

// Write of one value, non-temporal when NT is set.  A step whose state is
// larger than the last-level cache writes non-temporally: the value is read
// again only in the next step, after the rest of the state has passed through
// the cache, so caching it only evicts what the step is about to read.
// A state that fits is written normally and the next step's pulls hit it.
// (A compile-time choice: the two forms of a store differ only in metadata,
// and a runtime branch between them is merged into one plain store.)
template <bool NT, class B>
__device__ __forceinline__ void put(B* p, B v) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}

// Store of one post-collision value: 16-bit storage rounds stochastically
// with the random bits r when P.sr is set.
template <class ST, class CT, bool NT>
__device__ __forceinline__ void store_pop(const DevParams& P, typename Store<ST>::raw* p, CT v,
                                          uint32_t r) {
  using B = typename Store<ST>::bits;
  B b;
  if constexpr (sizeof(B) == 2) b = P.sr ? Store<ST>::enc_sr(v, r) : Store<ST>::enc(v);
  else b = Store<ST>::enc(v);
  put<NT, B>((B*)p, b);
}

// Source offsets along one axis for a node at coordinate x: entry c + 1
// holds the element offset of x - c (periodic wrap) and whether x - c lies
// beyond a wall (then the population bounces back into the node's own
// opposite slot).  Beyond a symmetry plane (sym_lo / sym_hi: the low / high
// boundary is one) the source is the mirror node, x itself on this axis
// (offset 0, no bounce); which population it is comes from sym_touch.
struct AxisSrc {
  int off[3];
  bool wall[3];
};
__device__ __forceinline__ void axis_src(int x, int n, int wall, int sym_lo, int sym_hi, int stride, AxisSrc& a) {
  const bool hi = x + 1 >= n, lo = x - 1 < 0;
  a.off[1] = 0;
  a.wall[1] = false;
  a.wall[0] = wall && !sym_hi && hi;
  a.off[0] = hi ? (wall ? 0 : (1 - n) * stride) : stride;
  a.wall[2] = wall && !sym_lo && lo;
  a.off[2] = lo ? (wall ? 0 : (n - 1) * stride) : -stride;
}

// Symmetry planes next to node (x, y, z), one bit each: 0 low x, 1 high x,
// 2 low y, 3 high y, 4 low z, 5 high z (zero without symmetry planes).
__device__ __forceinline__ int sym_touch(const DevParams& P, int x, int y, int z) {
  if (!P.sym) return 0;
  const int c[3] = {x, y, z}, n[3] = {P.nx, P.ny, P.nz};
  int m = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (c[a] == 0 && sym_side(P, a, true)) m |= 1 << (2 * a);
    if (c[a] == n[a] - 1 && sym_side(P, a, false)) m |= 2 << (2 * a);
  }
  return m;
}

// The population read in place of population i at a node with sym_touch m:
// the components whose source lies beyond a symmetry plane are reversed.
template <int Q>
__device__ __forceinline__ int pulled_population(int i, int m) {
  using L = Lat<Q>;
  int f = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    // c_a > 0 reads across the low plane, c_a < 0 across the high one
    if (L::c[i][a] > 0) f |= ((m >> (2 * a)) & 1) << a;
    if (L::c[i][a] < 0) f |= ((m >> (2 * a + 1)) & 1) << a;
  }
  return f ? lat_reflected<Q>(i, f & 1, (f >> 1) & 1, (f >> 2) & 1) : i;
}

}  // namespace pfl
