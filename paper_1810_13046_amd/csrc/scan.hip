// Exclusive prefix sums (int64 totals) for counts, offsets and index maps.
// Three passes: per-block totals, one block scanning the totals, per-block
// scan plus offset.  Deterministic (integer) and independent of timing.
#include "internal.hpp"

namespace ibvt {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;
constexpr int kSumsThreads = 1024;  // the one block that scans the block totals

template <typename Tin>
__global__ __launch_bounds__(kScanThreads) void k_block_sums(const Tin* __restrict__ in, int64_t n,
                                                            int64_t* __restrict__ bsum) {
  __shared__ int64_t red[kScanThreads / kWave];
  const int64_t base = int64_t(blockIdx.x) * kScanTile;
  int64_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + int64_t(k) * kScanThreads + threadIdx.x;
    if (i < n) s += int64_t(in[i]);
  }
  s = wave_sum(s);
  if (lane_id() == 0) red[threadIdx.x / kWave] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t t = 0;
    for (int w = 0; w < kScanThreads / kWave; ++w) t += red[w];
    bsum[blockIdx.x] = t;
  }
}

// Inclusive scan of one value per thread across the block; returns the
// exclusive prefix and writes the block total to *total.  sh holds one
// entry per wave.
__device__ int64_t block_exclusive(int64_t v, int64_t* sh, int64_t* total) {
  // wave-level inclusive scan
  int64_t x = v;
  const int l = lane_id();
  for (int o = 1; o < kWave; o <<= 1) {
    const int64_t y = __shfl_up(x, o, kWave);
    if (l >= o) x += y;
  }
  const int w = threadIdx.x / kWave;
  if (l == kWave - 1) sh[w] = x;
  __syncthreads();
  int64_t pre = 0, tot = 0;
  for (int k = 0; k < int(blockDim.x) / kWave; ++k) {
    if (k < w) pre += sh[k];
    tot += sh[k];
  }
  __syncthreads();
  *total = tot;
  return pre + x - v;
}

// Exclusive scan of the nb block totals in place by one block: each thread
// takes a run of consecutive totals.
__global__ __launch_bounds__(kSumsThreads) void k_scan_sums(int64_t* __restrict__ bsum, int64_t nb,
                                                           int64_t* __restrict__ total_out) {
  __shared__ int64_t sh[kSumsThreads / kWave];
  const int64_t per = ceil_div(nb > 0 ? nb : 1, kSumsThreads);
  const int64_t b0 = int64_t(threadIdx.x) * per;
  const int64_t b1 = min<int64_t>(nb, b0 + per);
  int64_t s = 0;
  for (int64_t b = b0; b < b1; ++b) s += bsum[b];
  int64_t tot;
  int64_t pre = block_exclusive(s, sh, &tot);
  for (int64_t b = b0; b < b1; ++b) {
    const int64_t v = bsum[b];
    bsum[b] = pre;
    pre += v;
  }
  if (threadIdx.x == 0) *total_out = tot;
}

// Per tile: the items are read with consecutive threads on consecutive
// items into LDS, each thread scans its run of kScanItems there (rows
// padded by one entry against bank conflicts), and the results leave the
// same coalesced way.
__device__ __forceinline__ int scan_slot(int i) { return (i / kScanItems) * (kScanItems + 1) + i % kScanItems; }

template <typename Tin>
__global__ __launch_bounds__(kScanThreads) void k_scan_tiles(const Tin* __restrict__ in, int64_t n,
                                                            const int64_t* __restrict__ bsum,
                                                            int64_t* __restrict__ out) {
  __shared__ int64_t buf[kScanThreads * (kScanItems + 1)];
  __shared__ int64_t sh[kScanThreads / kWave];
  const int64_t base = int64_t(blockIdx.x) * kScanTile;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int i = k * kScanThreads + int(threadIdx.x);
    buf[scan_slot(i)] = (base + i < n) ? int64_t(in[base + i]) : 0;
  }
  __syncthreads();
  int64_t* row = buf + threadIdx.x * (kScanItems + 1);
  int64_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) s += row[k];
  int64_t tot;
  int64_t pre = block_exclusive(s, sh, &tot) + bsum[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t v = row[k];
    row[k] = pre;
    pre += v;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int i = k * kScanThreads + int(threadIdx.x);
    if (base + i < n) out[base + i] = buf[scan_slot(i)];
  }
}

template <typename Tin>
int scan_impl(ibvt_coupling* c, const Tin* in, int64_t* out, int64_t n, hipStream_t s) {
  const int64_t nb = ceil_div(n > 0 ? n : 1, kScanTile);
  int st = ensure(c, c->scan_tmp, size_t(nb) * sizeof(int64_t));
  if (st) return st;
  int64_t* bsum = c->scan_tmp.as<int64_t>();
  if (n > 0) k_block_sums<Tin><<<dim3(unsigned(nb)), kScanThreads, 0, s>>>(in, n, bsum);
  else {
    st = hip_check(hipMemsetAsync(bsum, 0, sizeof(int64_t), s), "memset");
    if (st) return st;
  }
  k_scan_sums<<<1, kSumsThreads, 0, s>>>(bsum, n > 0 ? nb : 0, out + n);
  if (n > 0) k_scan_tiles<Tin><<<dim3(unsigned(nb)), kScanThreads, 0, s>>>(in, n, bsum, out);
  return hip_check(hipGetLastError(), "scan launch");
}

}  // namespace

int scan_i64(ibvt_coupling* c, const int64_t* in, int64_t* out, int64_t n, hipStream_t s) {
  return scan_impl<int64_t>(c, in, out, n, s);
}

int scan_i32_to_i64(ibvt_coupling* c, const int32_t* in, int64_t* out, int64_t n, hipStream_t s) {
  return scan_impl<int32_t>(c, in, out, n, s);
}

}  // namespace ibvt
