// Stable sorts by small integer keys, written for wave64: the pair order of
// the clip (8-bit keys) and the radix passes of the transpose (keys of up to
// 2 x kMaxDigitBits bits).
//
// One pass orders the items by one digit of the key, keeping the input
// order among equal digits (LSD radix pass):
//   k_digit_count    each wave takes a tile of kSortTile consecutive items
//                    and counts its digits in LDS; the tile's histogram is
//                    written digit-major (hist[digit][tile]).
//   scan             exclusive prefix over the histogram: the first output
//                    position of each (digit, tile).
//   k_digit_scatter  each wave walks its tile again in rounds of 64 items in
//                    input order; within a round the lanes with the same digit
//                    find each other by one ballot per digit bit, take
//                    consecutive positions in lane order and advance the
//                    tile's running position of that digit (LDS).
// Positions follow from the input order alone: the result does not depend
// on timing, and no value is combined.
#include "internal.hpp"

#include <type_traits>

namespace ibvt {

namespace {

constexpr int kSortWaves = 4;                 // waves (tiles) per block
constexpr int kSortRounds = 128;              // rounds of 64 items per tile
constexpr int kSortTile = kWave * kSortRounds;

template <typename K>
__device__ __forceinline__ uint32_t digit_of(K key, int shift, uint32_t mask) {
  return (uint32_t(key) >> shift) & mask;
}

template <typename K, int BITS>
__global__ __launch_bounds__(kWave * kSortWaves) void k_digit_count(
    int64_t n, const K* __restrict__ keys, int shift, int64_t ntiles,
    int32_t* __restrict__ hist) {
  constexpr int kBins = 1 << BITS;
  __shared__ int32_t h[kSortWaves][kBins];
  const int w = threadIdx.x / kWave, lane = lane_id();
  const int64_t tile = int64_t(blockIdx.x) * kSortWaves + w;
  for (int b = lane; b < kBins; b += kWave) h[w][b] = 0;
  wave_lds_sync();
  if (tile < ntiles) {
    const int64_t base = tile * kSortTile;
    for (int r = 0; r < kSortRounds; ++r) {
      const int64_t i = base + int64_t(r) * kWave + lane;
      if (i < n) atomicAdd(&h[w][digit_of(keys[i], shift, kBins - 1)], 1);
    }
  }
  wave_lds_sync();
  if (tile < ntiles)
    for (int b = lane; b < kBins; b += kWave) hist[int64_t(b) * ntiles + tile] = h[w][b];
}

// vals_in == nullptr: the value carried is the item's index.
template <typename K, typename V, int BITS>
__global__ __launch_bounds__(kWave * kSortWaves) void k_digit_scatter(
    int64_t n, const K* __restrict__ keys_in, const V* __restrict__ vals_in, int shift,
    int64_t ntiles, const int64_t* __restrict__ off, K* __restrict__ keys_out,
    V* __restrict__ vals_out) {
  constexpr int kBins = 1 << BITS;
  __shared__ int32_t run[kSortWaves][kBins];  // n < 2^31
  const int w = threadIdx.x / kWave, lane = lane_id();
  const int64_t tile = int64_t(blockIdx.x) * kSortWaves + w;
  if (tile >= ntiles) return;  // the whole wave
  for (int b = lane; b < kBins; b += kWave) run[w][b] = int32_t(off[int64_t(b) * ntiles + tile]);
  wave_lds_sync();
  const uint64_t below = (uint64_t(1) << lane) - 1;
  const int64_t base = tile * kSortTile;
  for (int r = 0; r < kSortRounds; ++r) {
    const int64_t i = base + int64_t(r) * kWave + lane;
    const bool act = i < n;
    K key = K(0);
    if (act) key = keys_in[i];
    const uint32_t dg = digit_of(key, shift, kBins - 1);
    uint64_t peers = ballot64(act);
#pragma unroll
    for (int b = 0; b < BITS; ++b) {
      const uint64_t m = ballot64((dg >> b) & 1u);
      peers &= ((dg >> b) & 1u) ? m : ~m;
    }
    const int rank = popc64(peers & below);
    const int cnt = popc64(peers);
    int32_t pos = 0;
    if (act) pos = run[w][dg] + rank;
    wave_lds_sync();  // every lane has read its digit's position
    if (act && rank == cnt - 1) run[w][dg] = pos + 1;
    wave_lds_sync();
    if (act) {
      if (keys_out) keys_out[pos] = key;
      if constexpr (std::is_integral<V>::value)
        vals_out[pos] = vals_in ? vals_in[i] : V(i);
      else
        vals_out[pos] = vals_in[i];
    }
  }
}

inline unsigned blocks_for_tiles(int64_t ntiles) {
  return unsigned(ceil_div(ntiles > 0 ? ntiles : 1, kSortWaves));
}

}  // namespace

int64_t sort_tiles(int64_t n) { return ceil_div(n > 0 ? n : 1, kSortTile); }

namespace {
size_t hist_bytes(int64_t m) { return (size_t(m + 1) * sizeof(int32_t) + 255) & ~size_t(255); }
}  // namespace

// Scratch bytes of one pass with 2^bits digits (histogram and offsets).
size_t sort_pass_bytes(int64_t n, int bits) {
  const int64_t m = (int64_t(1) << bits) * sort_tiles(n);
  return hist_bytes(m) + size_t(m + 1) * sizeof(int64_t) + 256;
}

const int64_t* sort_digit_starts(const void* scratch, int64_t n, int bits) {
  const int64_t m = (int64_t(1) << bits) * sort_tiles(n);
  return reinterpret_cast<const int64_t*>(static_cast<const char*>(scratch) + hist_bytes(m));
}

template <typename K, typename V, int BITS>
int digit_pass(ibvt_coupling* c, int64_t n, const K* keys_in, const V* vals_in, int shift,
               K* keys_out, V* vals_out, void* scratch, hipStream_t s) {
  const int64_t ntiles = sort_tiles(n);
  const int64_t m = (int64_t(1) << BITS) * ntiles;
  int32_t* hist = static_cast<int32_t*>(scratch);
  int64_t* off = reinterpret_cast<int64_t*>(static_cast<char*>(scratch) + hist_bytes(m));
  k_digit_count<K, BITS><<<blocks_for_tiles(ntiles), kWave * kSortWaves, 0, s>>>(
      n, keys_in, shift, ntiles, hist);
  int st = hip_check(hipGetLastError(), "digit count launch");
  if (st) return st;
  if ((st = scan_i32_to_i64(c, hist, off, m, s))) return st;
  k_digit_scatter<K, V, BITS><<<blocks_for_tiles(ntiles), kWave * kSortWaves, 0, s>>>(
      n, keys_in, vals_in, shift, ntiles, off, keys_out, vals_out);
  return hip_check(hipGetLastError(), "digit scatter launch");
}

int order_by_byte_key(ibvt_coupling* c, int64_t n, const uint8_t* keys, int32_t* order,
                      void* scratch, hipStream_t s) {
  if (n <= 0) return IBVT_OK;
  return digit_pass<uint8_t, int32_t, 8>(c, n, keys, nullptr, 0, nullptr, order, scratch, s);
}

template <typename V>
int sort_pairs_i32(ibvt_coupling* c, int64_t n, int end_bit, int32_t* keys, V* vals,
                   int32_t* keys_tmp, V* vals_tmp, void* scratch, hipStream_t s) {
  if (n <= 0) return IBVT_OK;
  if (end_bit > 2 * kMaxDigitBits)
    return set_error(IBVT_E_CAPACITY, "sort key wider than two digit passes");
  // two passes of equal width: the result lands back in keys / vals
  const int lo_bits = (end_bit + 1) / 2;
  int st;
  switch (lo_bits) {
#define IBVT_PASS(B)                                                                         \
  case B:                                                                                    \
    if ((st = digit_pass<int32_t, V, B>(c, n, keys, vals, 0, keys_tmp, vals_tmp, scratch, s))) \
      return st;                                                                             \
    return digit_pass<int32_t, V, B>(c, n, keys_tmp, vals_tmp, B, keys, vals, scratch, s);
    IBVT_PASS(1)
    IBVT_PASS(2)
    IBVT_PASS(3)
    IBVT_PASS(4)
    IBVT_PASS(5)
    IBVT_PASS(6)
    IBVT_PASS(7)
    IBVT_PASS(8)
    IBVT_PASS(9)
    IBVT_PASS(10)
    IBVT_PASS(11)
#undef IBVT_PASS
    default:
      return set_error(IBVT_E_CAPACITY, "sort digit width");
  }
}

template int sort_pairs_i32<SortVal32>(ibvt_coupling*, int64_t, int, int32_t*, SortVal32*,
                                       int32_t*, SortVal32*, void*, hipStream_t);
template int sort_pairs_i32<SortVal64>(ibvt_coupling*, int64_t, int, int32_t*, SortVal64*,
                                       int32_t*, SortVal64*, void*, hipStream_t);

}  // namespace ibvt
