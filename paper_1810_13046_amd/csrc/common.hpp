// Shared host/device helpers for the ibvt HIP library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ibvt {

constexpr int kWave = 64;

// Device-side status bits (OR-ed into a flag word by kernels).
constexpr unsigned kFlagOutOfGrid = 1u;
constexpr unsigned kFlagCapacity = 2u;
constexpr unsigned kFlagNonFinite = 4u;
constexpr unsigned kFlagValence = 8u;
constexpr unsigned kFlagTetSpan = 16u;  // a tet spans more than kMaxTetCells cells
constexpr int kMaxTetCells = 65535;     // cells of one lattice a tet may span
constexpr int kMaxChunks = 8;           // pair chunks of the clip and integration

// Counter slots (unsigned long long) written by the assembly kernels.
enum Counter : int {
  kCntPieces = 0,
  kCntDropped = 1,
  kCntZeroTets = 2,
  kCntSubtets = 3,
  kCntUnused4 = 4,
  kCntUnused5 = 5,  // 5, 6, 7: unused
  kCntDist = 8,   // signed distances evaluated by the clip
  kCntCutPts = 9, // cut points made by the clip
  kCntRowOverflow = 10,  // rows too wide for the LDS row gather (unstructured)
  kCntPlanes = 11,  // (pair, cell plane) clips run by the clip
  kCntChunkPool = 12,  // 12..19: piece-store records asked for by each pair chunk
  kCntSlots = 20,
};

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Orders the LDS accesses of one wave around this point (the wave's LDS
// operations execute in issue order; this keeps the compiler from moving
// them across).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

__device__ __forceinline__ int wave_min(int v) {
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, kWave));
  return v;
}

__device__ __forceinline__ int wave_max(int v) {
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, kWave));
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
  return v;
}

__device__ __forceinline__ uint64_t ballot64(bool p) { return __ballot(p); }

__device__ __forceinline__ int popc64(uint64_t m) { return __popcll(m); }

// Lanes below this one in a wave64 mask.
__device__ __forceinline__ int rank_below(uint64_t m) {
  return __popcll(m & ((1ull << __lane_id()) - 1ull));
}

__host__ __device__ __forceinline__ int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Per-tet cell range for one velocity component: first cell index and
// cell count along each axis (packed 6 x int32).
struct CellRange {
  int32_t lo[3];
  int32_t n[3];
};

// Copies n values (n a multiple of 16 bytes' worth) between a 16-byte
// aligned row in memory and registers with 16-byte accesses.
template <int N, typename T>
__device__ __forceinline__ void load_row(const T* __restrict__ src, T (&dst)[N]) {
  static_assert((N * sizeof(T)) % 16 == 0, "row of whole 16-byte words");
  constexpr int W = 16 / sizeof(T);
  typedef T V __attribute__((ext_vector_type(W)));
  const V* s = reinterpret_cast<const V*>(src);
#pragma unroll
  for (int k = 0; k < N / W; ++k) {
    const V v = s[k];
#pragma unroll
    for (int e = 0; e < W; ++e) dst[k * W + e] = v[e];
  }
}

template <int N, typename T>
__device__ __forceinline__ void store_row(T* __restrict__ dst, const T (&src)[N]) {
  static_assert((N * sizeof(T)) % 16 == 0, "row of whole 16-byte words");
  constexpr int W = 16 / sizeof(T);
  typedef T V __attribute__((ext_vector_type(W)));
  V* d = reinterpret_cast<V*>(dst);
#pragma unroll
  for (int k = 0; k < N / W; ++k) {
    V v;
#pragma unroll
    for (int e = 0; e < W; ++e) v[e] = src[k * W + e];
    d[k] = v;
  }
}

}  // namespace ibvt
