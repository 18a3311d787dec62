// Stable sorts by small integer keys, written for wave64: the orders of the
// pairs and of the (component, tet) items by 8-bit keys.
//
// One pass orders the items by one digit of the key, keeping the input
// order among equal digits (LSD radix pass):
//   k_digit_count    each wave takes a tile of consecutive items (32 rounds
//                    of 64, 16 for 16-byte values), loads them all, counts
//                    their digits in LDS and writes the tile's histogram
//                    digit-major (hist[digit][tile]).
//   scan             exclusive prefix over the histogram: the first output
//                    position of each (digit, tile).
//   k_digit_scatter  each wave loads its tile again (keys and values in
//                    registers), ranks the items round by round in input
//                    order by digit (one ballot per digit bit), stages the
//                    tile in LDS in digit order and writes it out in runs of
//                    consecutive addresses per digit.
// Positions follow from the input order alone: the result does not depend
// on timing, and no value is combined.
#include "internal.hpp"

#include <algorithm>
#include <type_traits>

namespace ibvt {

namespace {

constexpr int kSortWaves = 4;  // waves (tiles) per block of the count kernel

// Rounds of 64 items per tile: every item of a tile is held in registers
// while it is ranked (values of 16 bytes take half the rounds).
template <typename V>
constexpr int sort_rounds() {
  return sizeof(V) > 8 ? 16 : 32;
}

template <typename K>
__device__ __forceinline__ uint32_t digit_of(K key, int shift, uint32_t mask) {
  return (uint32_t(key) >> shift) & mask;
}

template <typename K, int BITS, int R>
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
    const int64_t base = tile * int64_t(R * kWave);
    // every load of the tile in flight before the first count
    K kv[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t i = base + int64_t(r) * kWave + lane;
      kv[r] = i < n ? keys[i] : K(0);
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t i = base + int64_t(r) * kWave + lane;
      if (i < n) atomicAdd(&h[w][digit_of(kv[r], shift, kBins - 1)], 1);
    }
  }
  wave_lds_sync();
  if (tile < ntiles)
    for (int b = lane; b < kBins; b += kWave) hist[int64_t(b) * ntiles + tile] = h[w][b];
}

// One wave per tile.  The tile's items are first ranked in input order
// (the lanes with the same digit find each other by one ballot per digit
// bit and take consecutive places in lane order) and put in LDS in digit
// order; the wave then writes the staged tile out, so the items of one
// digit leave as a run of consecutive addresses.  The value carried with
// item i is src.load<W>(i, active) (an input array's entry).
// Values travel as raw words of their size (no per-field work on them),
// held as native vectors so that they stay in registers.
typedef uint32_t RawWord2 __attribute__((ext_vector_type(2)));
typedef uint32_t RawWord4 __attribute__((ext_vector_type(4)));
template <typename V>
using RawWord = std::conditional_t<
    sizeof(V) == 16, RawWord4,
    std::conditional_t<sizeof(V) == 8, RawWord2, std::conditional_t<sizeof(V) == 4, uint32_t, V>>>;

// the item's own index as the value (an order of the items)
struct IndexVals {
  template <typename W>
  __device__ __forceinline__ W load(int64_t i, bool) const {
    return W(uint32_t(i));
  }
};

// Where a pass's items go: keys and values to two arrays (the keys may be
// left out).
template <typename K, typename V>
struct PlainOut {
  K* keys_out;
  V* vals_out;
  template <typename W>
  __device__ __forceinline__ void put(int64_t pos, K key, const W& w) const {
    if (keys_out) keys_out[pos] = key;
    reinterpret_cast<W*>(vals_out)[pos] = w;
  }
};

template <typename K, typename V, int BITS, int R, typename Src, typename Dst>
__global__ __launch_bounds__(kWave) void k_digit_scatter(
    int64_t n, const K* __restrict__ keys_in, Src src, int shift, int64_t ntiles,
    const int32_t* __restrict__ hist, const int64_t* __restrict__ off, Dst dst) {
  constexpr int kBins = 1 << BITS;
  constexpr int kPer = (kBins + kWave - 1) / kWave;  // bins per lane in the local scan
  constexpr int kTile = R * kWave;
  using W = RawWord<V>;
  static_assert(sizeof(W) == sizeof(V), "value word size");
  __shared__ K sk[kTile];
  __shared__ W sv[kTile];
  __shared__ int32_t lstart[kBins], run[kBins];
  __shared__ int64_t gstart[kBins];
  const int lane = lane_id();
  const int64_t tile = blockIdx.x;
  const int64_t base = tile * int64_t(kTile);
  // the tile's first place of each digit, locally (exclusive scan of the
  // tile's counts) and in the output
  int32_t cnt[kPer];
  int32_t sum = 0;
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int b = lane * kPer + k;
    cnt[k] = b < kBins ? hist[int64_t(b) * ntiles + tile] : 0;
    if (b < kBins) gstart[b] = off[int64_t(b) * ntiles + tile];
    sum += cnt[k];
  }
  int32_t incl = sum;
  for (int o = 1; o < kWave; o <<= 1) {
    const int32_t y = __shfl_up(incl, o, kWave);
    if (lane >= o) incl += y;
  }
  int32_t acc = incl - sum;
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int b = lane * kPer + k;
    if (b < kBins) {
      lstart[b] = acc;
      run[b] = acc;
    }
    acc += cnt[k];
  }
  wave_lds_sync();
  const uint64_t below = (uint64_t(1) << lane) - 1;
  // every load of the tile in flight before the ranking starts
  K kv[R];
  W vv[R];
#pragma clang loop unroll(full)
  for (int r = 0; r < R; ++r) {
    const int64_t i = base + int64_t(r) * kWave + lane;
    const bool act = i < n;
    kv[r] = act ? keys_in[i] : K(0);
    vv[r] = src.template load<W>(i, act);
  }
#pragma clang loop unroll(full)
  for (int r = 0; r < R; ++r) {
    const int64_t i = base + int64_t(r) * kWave + lane;
    const bool act = i < n;
    const K key = kv[r];
    const uint32_t dg = digit_of(key, shift, kBins - 1);
    uint64_t peers = ballot64(act);
#pragma unroll
    for (int b = 0; b < BITS; ++b) {
      const uint64_t m = ballot64((dg >> b) & 1u);
      peers &= ((dg >> b) & 1u) ? m : ~m;
    }
    const int rank = popc64(peers & below);
    const int cnt_d = popc64(peers);
    int32_t pos = 0;
    if (act) pos = run[dg] + rank;
    wave_lds_sync();  // every lane has read its digit's place
    if (act && rank == cnt_d - 1) run[dg] = pos + 1;
    if (act) {
      sk[pos] = key;
      sv[pos] = vv[r];
    }
    wave_lds_sync();
  }
  const int m = int(min<int64_t>(kTile, n - base));
  for (int j = lane; j < m; j += kWave) {
    const K key = sk[j];
    const uint32_t dg = digit_of(key, shift, kBins - 1);
    dst.put(gstart[dg] + (j - lstart[dg]), key, sv[j]);
  }
}

inline unsigned blocks_for_tiles(int64_t ntiles) {
  return unsigned(ceil_div(ntiles > 0 ? ntiles : 1, kSortWaves));
}

}  // namespace

namespace {
int64_t tiles_for(int64_t n, int rounds) { return ceil_div(n > 0 ? n : 1, int64_t(rounds) * kWave); }
size_t hist_bytes(int64_t m) { return (size_t(m + 1) * sizeof(int32_t) + 255) & ~size_t(255); }
}  // namespace

int64_t sort_tiles(int64_t n, int value_bytes) {
  return tiles_for(n, value_bytes > 8 ? sort_rounds<PairDesc>() : sort_rounds<int32_t>());
}

// Scratch bytes of one pass with 2^bits digits (histogram and offsets), for
// the smallest tiles any value type takes.
size_t sort_pass_bytes(int64_t n, int bits) {
  const int64_t m = (int64_t(1) << bits) * tiles_for(n, sort_rounds<SortVal64>());
  return hist_bytes(m) + size_t(m + 1) * sizeof(int64_t) + 256;
}

const int64_t* sort_digit_starts(const void* scratch, int64_t n, int bits, int value_bytes) {
  const int64_t m = (int64_t(1) << bits) * sort_tiles(n, value_bytes);
  return reinterpret_cast<const int64_t*>(static_cast<const char*>(scratch) + hist_bytes(m));
}

template <typename K, typename V, int BITS, typename Src, typename Dst>
int digit_pass(ibvt_coupling* c, int64_t n, const K* keys_in, Src src, int shift, Dst dst,
               void* scratch, hipStream_t s) {
  constexpr int R = sort_rounds<V>();
  const int64_t ntiles = tiles_for(n, R);
  const int64_t m = (int64_t(1) << BITS) * ntiles;
  int32_t* hist = static_cast<int32_t*>(scratch);
  int64_t* off = reinterpret_cast<int64_t*>(static_cast<char*>(scratch) + hist_bytes(m));
  k_digit_count<K, BITS, R><<<blocks_for_tiles(ntiles), kWave * kSortWaves, 0, s>>>(
      n, keys_in, shift, ntiles, hist);
  int st = hip_check(hipGetLastError(), "digit count launch");
  if (st) return st;
  if ((st = scan_i32_to_i64(c, hist, off, m, s))) return st;
  k_digit_scatter<K, V, BITS, R, Src, Dst><<<unsigned(ntiles), kWave, 0, s>>>(
      n, keys_in, src, shift, ntiles, hist, off, dst);
  return hip_check(hipGetLastError(), "digit scatter launch");
}

int order_by_byte_key(ibvt_coupling* c, int64_t n, const uint8_t* keys, int32_t* order,
                      void* scratch, hipStream_t s) {
  if (n <= 0) return IBVT_OK;
  return digit_pass<uint8_t, int32_t, 8>(c, n, keys, IndexVals{}, 0,
                                         PlainOut<uint8_t, int32_t>{nullptr, order}, scratch, s);
}

}  // namespace ibvt
