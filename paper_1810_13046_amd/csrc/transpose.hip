// B^dT over the touched fluid nodes (the force transfer's operator).
//
// Rows of B^dT are the fluid nodes that occur as columns of B^d, in
// ascending node order, each listing its vertices in ascending order.  Large
// operators go through buckets of kBucketNodes consecutive lattice nodes:
//   k_bucket_count    blocks of kBucketRows rows of B^d take their nonzeros
//                     in rounds of kRound; within a wave the nonzeros of one
//                     bucket come in runs (a row's columns ascend), and each
//                     run's head adds its count into an LDS hash table, so
//                     one global atomic per (round, bucket) sums them; every
//                     nonzero marks its node (a byte per lattice node).
//   scans             bucket offsets in B^dT (from the counts), row offsets
//                     (from the marked nodes per bucket) and the list of
//                     nonempty buckets; one read-back gives the touched-node
//                     and nonempty-bucket counts.
//   k_bucket_scatter  the same rounds reserve a range per (round, bucket);
//                     run heads take their runs' places in it and every
//                     nonzero writes its (value, vertex, node) record.
//   k_bucket_sort     one block per nonempty bucket: a counting sort of its
//                     records by node in LDS, then each record's place in its
//                     node's row is the number of that row's vertices below
//                     its own (a row's vertices are distinct); the block
//                     writes the bucket's columns, values, row pointers and
//                     row map.
// Small operators take a counting sort over the whole lattice instead
// (column marks and their prefix sum, column counts, a scatter into slots,
// then each row of B^dT put in vertex order by ranking).  Atomics only
// reserve space; every position follows from the (node, vertex) order, so
// the result is deterministic either way.
#include <climits>
#include <cstdlib>
#include <type_traits>

#include "internal.hpp"

namespace ibvt {

namespace {

__global__ void k_mark(int64_t nnz, const int32_t* __restrict__ col, int32_t* __restrict__ mark) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k < nnz) mark[col[k]] = 1;
}

__global__ void k_compact(int64_t n, const int32_t* __restrict__ mark,
                          const int64_t* __restrict__ cidx, int32_t* __restrict__ rowmap) {
  const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j < n && mark[j]) rowmap[cidx[j]] = int32_t(j);
}

// A nonzero carried through the counting sort: its value and its row.
template <typename T>
using ValRow = std::conditional_t<std::is_same<T, float>::value, SortVal32, SortVal64>;

constexpr int kKeyLanes = 16;  // lanes per row of B^d in the counting sort's scatter

// Counting sort for small operators, where the bucket path's fixed launches
// dominate.  tcnt[c] = nonzeros of B^d in compacted column c (integer
// atomics).
__global__ void k_tcount(int64_t nnz, const int32_t* __restrict__ col,
                         const int64_t* __restrict__ cidx, int32_t* __restrict__ tcnt) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k < nnz) atomicAdd(&tcnt[cidx[col[k]]], 1);
}

// Every nonzero (i, j) of B^d takes a slot of row cidx[j] of B^dT by counting
// that row's tcnt down (the slot order depends on timing; k_trow_order puts
// each row in vertex order afterwards).
template <typename T>
__global__ __launch_bounds__(256) void k_tscatter(int64_t n_rows, const int64_t* __restrict__ rowptr,
                                                  const int32_t* __restrict__ col,
                                                  const T* __restrict__ val,
                                                  const int64_t* __restrict__ cidx,
                                                  const int64_t* __restrict__ trowptr,
                                                  int32_t* __restrict__ tcnt,
                                                  ValRow<T>* __restrict__ vr) {
  const int64_t i = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / kKeyLanes;
  const int lane = threadIdx.x % kKeyLanes;
  if (i >= n_rows) return;
  for (int64_t k = rowptr[i] + lane; k < rowptr[i + 1]; k += kKeyLanes) {
    const int64_t cc = cidx[col[k]];
    const int slot = atomicSub(&tcnt[cc], 1) - 1;
    ValRow<T> x;
    x.v = val[k];
    x.r = int32_t(i);
    vr[trowptr[cc] + slot] = x;
  }
}

// One wave per row of B^dT: the row's vertices are distinct, so an entry's
// place in ascending vertex order is the number of the row's entries with a
// smaller vertex.  The row is read in tiles of kWave entries whose vertices
// are broadcast lane by lane.  Positions do not depend on the slot order
// k_tscatter left, so the result is deterministic.
template <typename T>
__global__ __launch_bounds__(256) void k_trow_order(int64_t n_rows,
                                                    const int64_t* __restrict__ trowptr,
                                                    const ValRow<T>* __restrict__ vr,
                                                    int32_t* __restrict__ tcol,
                                                    T* __restrict__ tval) {
  const int64_t r = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / kWave;
  const int lane = lane_id();
  if (r >= n_rows) return;  // the whole wave
  const int64_t b = trowptr[r];
  const int L = __builtin_amdgcn_readfirstlane(int(trowptr[r + 1] - b));
  for (int c0 = 0; c0 < L; c0 += kWave) {
    const bool mine = c0 + lane < L;
    ValRow<T> x;
    x.v = T(0);
    x.r = INT_MAX;
    if (mine) x = vr[b + c0 + lane];
    int rank = 0;
    for (int m0 = 0; m0 < L; m0 += kWave) {
      const int y = (m0 + lane < L) ? vr[b + m0 + lane].r : INT_MAX;
      const int nm = L - m0 < kWave ? L - m0 : kWave;
      for (int m = 0; m < nm; ++m) rank += __builtin_amdgcn_readlane(y, m) < x.r ? 1 : 0;
    }
    if (mine) {
      tcol[b + rank] = x.r;
      tval[b + rank] = x.v;
    }
  }
}

// ---- bucket transpose (large operators) ----

constexpr int kBucketBits = 5;
constexpr int kBucketNodes = 1 << kBucketBits;  // consecutive lattice nodes per bucket
constexpr int kBucketRows = 64;                 // rows of B^d per block (count, scatter)
constexpr int kBucketThreads = 256;
constexpr int kRound = 2048;                    // nonzeros per round (8 per thread)
constexpr int kTableBits = 12;
constexpr int kTable = 1 << kTableBits;         // hash slots per round (>= 2 x kRound)
constexpr int kSortCap = 4096;                  // records a bucket sorts in LDS
static_assert(kRound % kBucketThreads == 0 && 2 * kRound <= kTable, "round and table sizes");

// A nonzero of B^d on its way into B^dT: value, and vertex (its row of B^d)
// with the node within the bucket in one word (vertices below 2^27).
template <typename T>
struct BucketRec {
  T v;
  uint32_t rn;  // vertex << kBucketBits | node
  __device__ __forceinline__ int32_t r() const { return int32_t(rn >> kBucketBits); }
  __device__ __forceinline__ int nl() const { return int(rn & (kBucketNodes - 1)); }
};
constexpr int64_t kBucketMaxVert = int64_t(1) << (32 - kBucketBits);

// A nonempty bucket as the sort takes it: its first record (= its first
// place in B^dT), its first row of B^dT, the bucket and its record count.
struct BucketSpan {
  int64_t a, t;
  int32_t b, n;
};

// Slot of bucket b in a round's table (open addressing; a round has at most
// kRound distinct buckets, so a free slot always exists).
__device__ __forceinline__ int table_slot(int32_t* key, int32_t b) {
  int h = int((uint32_t(b) * 2654435761u) >> (32 - kTableBits));
  for (;;) {
    const int32_t prev = atomicCAS(&key[h], -1, b);
    if (prev == -1 || prev == b) return h;
    h = (h + 1) & (kTable - 1);
  }
}

// Row block of this workgroup.  Workgroups are dispatched to the 8 XCDs in
// turn; handing each XCD a contiguous run of row blocks keeps the bucket
// ranges one XCD writes away from the others' (whole cache lines per L2).
// The grid has 8 * per blocks.
__device__ __forceinline__ int64_t xcd_row_block(int64_t per) {
  return int64_t(blockIdx.x % 8) * per + int64_t(blockIdx.x / 8);
}

// Runs of one bucket among a wave's consecutive nonzeros (a row's columns
// ascend, so its buckets come in runs): a run starts where the bucket
// differs from the previous lane's, or at lane 0.  The valid lanes are a
// prefix of the wave.  Gives the lane's run start and run end (one past).
struct WaveRun {
  int head, end;
  bool is_head;
};
__device__ __forceinline__ WaveRun wave_run(int32_t bucket, bool valid) {
  const int l = lane_id();
  const int32_t prev = __shfl_up(bucket, 1, kWave);
  WaveRun w;
  w.is_head = valid && (l == 0 || prev != bucket);
  const uint64_t heads = ballot64(w.is_head);
  const uint64_t n_valid = uint64_t(popc64(ballot64(valid)));
  const uint64_t upto = (2ull << l) - 1ull;  // lanes 0..l (all lanes when l = 63)
  const uint64_t below = heads & upto, above = heads & ~upto;
  w.head = below ? 63 - __builtin_clzll(below) : 0;
  w.end = above ? __builtin_ctzll(above) : int(n_valid);
  return w;
}

// Per bucket: nonzero count (only run heads touch the round's table), and
// a byte per node that occurs (plain stores: every writer stores 1).
__global__ __launch_bounds__(kBucketThreads) void k_bucket_count(
    int64_t n_rows, int64_t per, const int64_t* __restrict__ rowptr,
    const int32_t* __restrict__ col, int32_t* __restrict__ bcount, uint8_t* __restrict__ mark) {
  __shared__ int32_t key[kTable];
  __shared__ int32_t cnt[kTable];
  const int64_t r0 = xcd_row_block(per) * kBucketRows;
  if (r0 >= n_rows) return;
  const int64_t r1 = min<int64_t>(n_rows, r0 + kBucketRows);
  const int64_t k0 = rowptr[r0], k1 = rowptr[r1];
  const int l = lane_id();
  for (int64_t kb = k0; kb < k1; kb += kRound) {
    for (int h = threadIdx.x; h < kTable; h += kBucketThreads) {
      key[h] = -1;
      cnt[h] = 0;
    }
    __syncthreads();
    constexpr int J = kRound / kBucketThreads;
    int32_t nodes[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {  // all loads first
      const int64_t k = kb + j * kBucketThreads + threadIdx.x;
      nodes[j] = k < k1 ? col[k] : 0;
    }
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const bool valid = kb + j * kBucketThreads + threadIdx.x < k1;
      const int32_t node = nodes[j];
      const WaveRun w = wave_run(node >> kBucketBits, valid);
      if (valid) mark[node] = 1;
      if (w.is_head) atomicAdd(&cnt[table_slot(key, node >> kBucketBits)], w.end - l);
    }
    __syncthreads();
    for (int h = threadIdx.x; h < kTable; h += kBucketThreads) {
      const int32_t b = key[h];
      if (b >= 0) atomicAdd(&bcount[b], cnt[h]);
    }
    __syncthreads();
  }
}

// Touched nodes per bucket (its marked nodes) and its nonempty flag.
__global__ void k_bucket_rows(int64_t nb, const uint32_t* __restrict__ mark,
                              int32_t* __restrict__ tb, int32_t* __restrict__ nonempty) {
  const int64_t b = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (b < nb) {
    int m = 0;
#pragma unroll
    for (int w = 0; w < kBucketNodes / 4; ++w) m += __popc(mark[b * (kBucketNodes / 4) + w]);
    tb[b] = m;
    nonempty[b] = m != 0;
  }
}

// The nonempty buckets in ascending order.
__global__ void k_bucket_list(int64_t nb, const int32_t* __restrict__ nonempty,
                              const int64_t* __restrict__ pos, const int64_t* __restrict__ boff,
                              const int64_t* __restrict__ toff, BucketSpan* __restrict__ list) {
  const int64_t b = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (b < nb && nonempty[b]) {
    BucketSpan e;
    e.a = boff[b];
    e.t = toff[b];
    e.b = int32_t(b);
    e.n = int32_t(boff[b + 1] - boff[b]);
    list[pos[b]] = e;
  }
}

// The same rounds as k_bucket_count: each (round, bucket) reserves a range
// of the bucket, run heads take their runs' places in it, and every
// nonzero writes its record there.
template <typename T>
__global__ __launch_bounds__(kBucketThreads) void k_bucket_scatter(
    int64_t n_rows, int64_t per, const int64_t* __restrict__ rowptr,
    const int32_t* __restrict__ col, const T* __restrict__ val, const int64_t* __restrict__ boff,
    int32_t* __restrict__ bfill, BucketRec<T>* __restrict__ rec) {
  __shared__ int32_t key[kTable];
  __shared__ int32_t cnt[kTable];  // then the slot's first position in the records
  __shared__ int64_t srp[kBucketRows + 1];
  const int64_t r0 = xcd_row_block(per) * kBucketRows;
  if (r0 >= n_rows) return;
  const int nr = int(min<int64_t>(n_rows - r0, kBucketRows));
  for (int i = threadIdx.x; i <= nr; i += kBucketThreads) srp[i] = rowptr[r0 + i];
  __syncthreads();
  const int64_t k0 = srp[0], k1 = srp[nr];
  const int l = lane_id();
  constexpr int J = kRound / kBucketThreads;
  for (int64_t kb = k0; kb < k1; kb += kRound) {
    for (int h = threadIdx.x; h < kTable; h += kBucketThreads) {
      key[h] = -1;
      cnt[h] = 0;
    }
    __syncthreads();
    int slot[J], rank[J];
    int32_t node[J];
    T v[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {  // all loads first
      const int64_t k = kb + j * kBucketThreads + threadIdx.x;
      node[j] = k < k1 ? col[k] : 0;
      v[j] = k < k1 ? val[k] : T(0);
    }
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const bool valid = kb + j * kBucketThreads + threadIdx.x < k1;
      const WaveRun w = wave_run(node[j] >> kBucketBits, valid);
      int h = 0, r = 0;
      if (w.is_head) {
        h = table_slot(key, node[j] >> kBucketBits);
        r = atomicAdd(&cnt[h], w.end - l);
      }
      slot[j] = valid ? __shfl(h, w.head, kWave) : -1;
      rank[j] = __shfl(r, w.head, kWave) + (l - w.head);
    }
    __syncthreads();
    for (int h = threadIdx.x; h < kTable; h += kBucketThreads) {
      const int32_t b = key[h];
      if (b >= 0) cnt[h] = int32_t(boff[b]) + atomicAdd(&bfill[b], cnt[h]);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < J; ++j) {
      if (slot[j] < 0) continue;
      const int64_t k = kb + j * kBucketThreads + threadIdx.x;
      // row of nonzero k: srp[lo] <= k < srp[lo + 1] (empty rows skipped)
      int lo = 0, hi = nr;
      while (hi - lo > 1) {
        const int m = (lo + hi) >> 1;
        if (srp[m] <= k) lo = m;
        else hi = m;
      }
      BucketRec<T> x;
      x.v = v[j];
      x.rn = (uint32_t(r0 + lo) << kBucketBits) | uint32_t(node[j] & (kBucketNodes - 1));
      rec[cnt[slot[j]] + rank[j]] = x;
    }
    __syncthreads();
  }
}

// One block per nonempty bucket (each bucket owns its ranges of B^dT): row
// pointers and row map of its nodes, then its records in (node, vertex)
// order.  A bucket that fits the LDS is read once into registers; counting
// a record's node also gives it a slot among that node's records, the LDS
// holds the vertices grouped by node, and each record is ranked from its
// registers.
template <typename T>
__global__ __launch_bounds__(kBucketThreads) void k_bucket_sort(
    const BucketSpan* __restrict__ list, BucketRec<T>* __restrict__ rec,
    int32_t* __restrict__ tcol, T* __restrict__ tval, int64_t* __restrict__ trowptr,
    int32_t* __restrict__ rowmap, int64_t touched, int64_t nnz) {
  constexpr int R = kSortCap / kBucketThreads;
  __shared__ int32_t ncnt[kBucketNodes], noff[kBucketNodes], nfill[kBucketNodes];
  __shared__ int32_t sr[kSortCap];
  const BucketSpan e = list[blockIdx.x];
  const int64_t a = e.a;
  const int n = e.n;
  const int t = threadIdx.x;
  const bool fits = n <= kSortCap;
  if (t < kBucketNodes) {
    ncnt[t] = 0;
    nfill[t] = 0;
  }
  if (blockIdx.x == 0 && t == 0) trowptr[touched] = nnz;
  BucketRec<T> x[R];
  int slot[R];
  if (fits) {
#pragma unroll
    for (int i = 0; i < R; ++i)
      if (t + i * kBucketThreads < n) x[i] = rec[a + t + i * kBucketThreads];
  }
  __syncthreads();
  if (fits) {
#pragma unroll
    for (int i = 0; i < R; ++i)
      if (t + i * kBucketThreads < n) slot[i] = atomicAdd(&ncnt[x[i].nl()], 1);
  } else {
    for (int j = t; j < n; j += kBucketThreads) atomicAdd(&ncnt[rec[a + j].nl()], 1);
  }
  __syncthreads();
  if (t < kWave) {  // the first wave: node offsets, and the touched nodes' rows
    const int cn = t < kBucketNodes ? ncnt[t] : 0;
    int y = cn;
    for (int o = 1; o < kBucketNodes; o <<= 1) {
      const int z = __shfl_up(y, o, kWave);
      if (t >= o) y += z;
    }
    const uint64_t m = ballot64(cn > 0);
    if (t < kBucketNodes) noff[t] = y - cn;
    if (cn > 0) {
      const int64_t row = e.t + rank_below(m);
      trowptr[row] = a + (y - cn);
      rowmap[row] = (e.b << kBucketBits) | t;
    }
  }
  __syncthreads();
  if (fits) {
#pragma unroll
    for (int i = 0; i < R; ++i)
      if (t + i * kBucketThreads < n) sr[noff[x[i].nl()] + slot[i]] = x[i].r();
    __syncthreads();
    // a record's place in its row: the row's vertices below its own
#pragma unroll
    for (int i = 0; i < R; ++i) {
      if (t + i * kBucketThreads >= n) continue;
      const int nl = x[i].nl();
      const int s0 = noff[nl], s1 = s0 + ncnt[nl];
      const int32_t r = x[i].r();
      int rank = 0, u = s0;
      for (; u + 8 <= s1; u += 8) {  // eight reads in flight
        int32_t y[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) y[k] = sr[u + k];
#pragma unroll
        for (int k = 0; k < 8; ++k) rank += y[k] < r ? 1 : 0;
      }
      for (; u < s1; ++u) rank += sr[u] < r ? 1 : 0;
      tcol[a + s0 + rank] = r;
      tval[a + s0 + rank] = x[i].v;
    }
  } else {
    // more records than the LDS holds: group them by node in B^dT's arrays,
    // copy the grouped records back over the bucket's (consumed) ones, then
    // rank each node's records against its row, kSortCap of the row's
    // vertices at a time through LDS
    for (int j = t; j < n; j += kBucketThreads) {
      const BucketRec<T> g = rec[a + j];
      const int64_t q = a + noff[g.nl()] + atomicAdd(&nfill[g.nl()], 1);
      tcol[q] = g.r();
      tval[q] = g.v;
    }
    __syncthreads();
    for (int j = t; j < n; j += kBucketThreads) {
      BucketRec<T> g;
      g.v = tval[a + j];
      g.rn = uint32_t(tcol[a + j]) << kBucketBits;
      rec[a + j] = g;
    }
    for (int nl = 0; nl < kBucketNodes; ++nl) {
      const int L = ncnt[nl];
      const int64_t s0 = a + noff[nl];
      for (int q0 = 0; q0 < L; q0 += kBucketThreads) {
        const int q = q0 + t;
        BucketRec<T> g;
        g.v = T(0);
        g.rn = 0;
        int rank = 0;
        for (int c0 = 0; c0 < L; c0 += kSortCap) {
          const int m = min(kSortCap, L - c0);
          __syncthreads();  // the grouped records are written; sr is free
          if (c0 == 0 && q < L) g = rec[s0 + q];
          for (int u = t; u < m; u += kBucketThreads) sr[u] = rec[s0 + c0 + u].r();
          __syncthreads();
          if (q < L)
            for (int u = 0; u < m; ++u) rank += sr[u] < g.r() ? 1 : 0;
        }
        if (q < L) {
          tcol[s0 + rank] = g.r();
          tval[s0 + rank] = g.v;
        }
      }
    }
  }
}

// Nonzeros from which the bucket transpose is taken: 2^22, or
// IBVT_BUCKET_NNZ from the environment (a positive integer; small values put
// small operators through the bucket path, as the tests do).  Both paths
// give the same B^dT.
int64_t bucket_nnz() {
  if (const char* e = std::getenv("IBVT_BUCKET_NNZ")) {
    char* end = nullptr;
    const long long v = std::strtoll(e, &end, 10);
    if (end != e && *end == '\0' && v > 0) return int64_t(v);
  }
  return int64_t(4) << 20;
}

inline unsigned blocks_for(int64_t n, int threads) {
  return unsigned(ceil_div(n > 0 ? n : 1, threads));
}

// Counting sort over the whole lattice (small operators; nnz == 0 too).
template <typename T>
int transpose_counting(ibvt_coupling* c, int d, hipStream_t s) {
  const int64_t nf = c->n_fluid[d];
  const Csr& B = c->B[d];
  Csr& Bt = c->Bt[d];
  int st;
  if ((st = ensure(c, c->mark, size_t(nf + 1) * sizeof(int32_t)))) return st;
  if ((st = ensure(c, c->cidx, size_t(nf + 1) * sizeof(int64_t)))) return st;
  if ((st = hip_check(hipMemsetAsync(c->mark.p, 0, size_t(nf) * sizeof(int32_t), s), "memset")))
    return st;
  if (B.nnz)
    k_mark<<<blocks_for(B.nnz, 256), 256, 0, s>>>(B.nnz, B.col.as<int32_t>(), c->mark.as<int32_t>());
  if ((st = scan_i32_to_i64(c, c->mark.as<int32_t>(), c->cidx.as<int64_t>(), nf, s))) return st;
  int64_t touched = 0;
  {
    const int64_t* src[1] = {c->cidx.as<int64_t>() + nf};
    if ((st = read_counts(c, src, 1, &touched, s))) return st;
  }
  Bt.nrows = touched;
  Bt.nnz = B.nnz;
  if ((st = ensure(c, Bt.rowptr, size_t(touched + 1) * sizeof(int64_t)))) return st;
  if ((st = ensure(c, Bt.rowmap, size_t(touched + 1) * sizeof(int32_t)))) return st;
  if ((st = ensure(c, Bt.col, size_t(B.nnz + 1) * sizeof(int32_t)))) return st;
  if ((st = ensure(c, Bt.val, size_t(B.nnz + 1) * sizeof(T)))) return st;
  k_compact<<<blocks_for(nf, 256), 256, 0, s>>>(nf, c->mark.as<int32_t>(), c->cidx.as<int64_t>(),
                                                Bt.rowmap.as<int32_t>());
  if (B.nnz == 0) {
    int64_t z = 0;
    return hip_check(hipMemcpyAsync(Bt.rowptr.p, &z, sizeof(z), hipMemcpyHostToDevice, s),
                     "rowptr");
  }
  // row pointers of B^dT from the per-column counts, then the scatter into
  // slots and the per-row ordering
  int32_t* tcnt = c->mark.as<int32_t>();  // the marks are no longer needed
  if ((st = hip_check(hipMemsetAsync(tcnt, 0, size_t(touched) * sizeof(int32_t), s), "memset")))
    return st;
  k_tcount<<<blocks_for(B.nnz, 256), 256, 0, s>>>(B.nnz, B.col.as<int32_t>(),
                                                  c->cidx.as<int64_t>(), tcnt);
  if ((st = scan_i32_to_i64(c, tcnt, Bt.rowptr.as<int64_t>(), touched, s))) return st;
  if ((st = ensure(c, c->tbuf, size_t(B.nnz) * sizeof(ValRow<T>)))) return st;
  ValRow<T>* vr = c->tbuf.as<ValRow<T>>();
  k_tscatter<T><<<blocks_for(c->n_vert * kKeyLanes, 256), 256, 0, s>>>(
      c->n_vert, B.rowptr.as<int64_t>(), B.col.as<int32_t>(), B.val.as<T>(),
      c->cidx.as<int64_t>(), Bt.rowptr.as<int64_t>(), tcnt, vr);
  k_trow_order<T><<<blocks_for(touched * kWave, 256), 256, 0, s>>>(
      touched, Bt.rowptr.as<int64_t>(), vr, Bt.col.as<int32_t>(), Bt.val.as<T>());
  return hip_check(hipGetLastError(), "transpose launch");
}

// Bucket transpose (large operators).
template <typename T>
int transpose_buckets(ibvt_coupling* c, int d, hipStream_t s) {
  const int64_t nf = c->n_fluid[d];
  const Csr& B = c->B[d];
  Csr& Bt = c->Bt[d];
  int st;
  const int64_t nb = ceil_div(nf, kBucketNodes);
  auto al = [](size_t n) { return (n + 255) & ~size_t(255); };
  const size_t rec_b = al(size_t(B.nnz) * sizeof(BucketRec<T>));
  const size_t i32_b = al(size_t(nb) * sizeof(int32_t));
  const size_t i64_b = al(size_t(nb + 1) * sizeof(int64_t));
  const size_t mark_b = al(size_t(nb) * kBucketNodes);  // a byte per lattice node
  const size_t zero_b = 2 * i32_b + mark_b;             // counts, fill levels, marks
  const size_t list_b = al(size_t(nb) * sizeof(BucketSpan));
  if ((st = ensure(c, c->tbuf, rec_b + zero_b + 2 * i32_b + 3 * i64_b + list_b))) return st;
  char* p = c->tbuf.as<char>();
  BucketRec<T>* rec = reinterpret_cast<BucketRec<T>*>(p);
  p += rec_b;
  int32_t* bcount = reinterpret_cast<int32_t*>(p);
  int32_t* bfill = reinterpret_cast<int32_t*>(p + i32_b);
  uint8_t* mark = reinterpret_cast<uint8_t*>(p + 2 * i32_b);
  if ((st = hip_check(hipMemsetAsync(p, 0, zero_b, s), "memset"))) return st;
  p += zero_b;
  int32_t* tb = reinterpret_cast<int32_t*>(p);
  int32_t* nonempty = reinterpret_cast<int32_t*>(p + i32_b);
  p += 2 * i32_b;
  int64_t* boff = reinterpret_cast<int64_t*>(p);
  int64_t* toff = reinterpret_cast<int64_t*>(p + i64_b);
  int64_t* lpos = reinterpret_cast<int64_t*>(p + 2 * i64_b);
  BucketSpan* list = reinterpret_cast<BucketSpan*>(p + 3 * i64_b);

  const int64_t n_rows = c->n_vert;
  const int64_t per = ceil_div(ceil_div(n_rows, kBucketRows), 8);
  const unsigned grid = unsigned(8 * per);
  k_bucket_count<<<grid, kBucketThreads, 0, s>>>(n_rows, per, B.rowptr.as<int64_t>(),
                                                 B.col.as<int32_t>(), bcount, mark);
  k_bucket_rows<<<blocks_for(nb, 256), 256, 0, s>>>(nb, reinterpret_cast<const uint32_t*>(mark),
                                                    tb, nonempty);
  if ((st = hip_check(hipGetLastError(), "transpose count launch"))) return st;
  if ((st = scan_i32_to_i64(c, bcount, boff, nb, s))) return st;
  if ((st = scan_i32_to_i64(c, tb, toff, nb, s))) return st;
  if ((st = scan_i32_to_i64(c, nonempty, lpos, nb, s))) return st;
  k_bucket_list<<<blocks_for(nb, 256), 256, 0, s>>>(nb, nonempty, lpos, boff, toff, list);
  int64_t got[2] = {0, 0};
  {
    const int64_t* src[2] = {toff + nb, lpos + nb};
    if ((st = read_counts(c, src, 2, got, s))) return st;
  }
  const int64_t touched = got[0], n_nonempty = got[1];
  Bt.nrows = touched;
  Bt.nnz = B.nnz;
  if ((st = ensure(c, Bt.rowptr, size_t(touched + 1) * sizeof(int64_t)))) return st;
  if ((st = ensure(c, Bt.rowmap, size_t(touched + 1) * sizeof(int32_t)))) return st;
  if ((st = ensure(c, Bt.col, size_t(B.nnz + 1) * sizeof(int32_t)))) return st;
  if ((st = ensure(c, Bt.val, size_t(B.nnz + 1) * sizeof(T)))) return st;
  k_bucket_scatter<T><<<grid, kBucketThreads, 0, s>>>(n_rows, per, B.rowptr.as<int64_t>(),
                                                      B.col.as<int32_t>(), B.val.as<T>(), boff,
                                                      bfill, rec);
  k_bucket_sort<T><<<unsigned(n_nonempty), kBucketThreads, 0, s>>>(
      list, rec, Bt.col.as<int32_t>(), Bt.val.as<T>(), Bt.rowptr.as<int64_t>(),
      Bt.rowmap.as<int32_t>(), touched, B.nnz);
  return hip_check(hipGetLastError(), "transpose launch");
}

}  // namespace

template <typename T>
int transpose_one(ibvt_coupling* c, int d, hipStream_t s) {
  return c->B[d].nnz >= bucket_nnz() && c->n_vert < kBucketMaxVert
             ? transpose_buckets<T>(c, d, s)
             : transpose_counting<T>(c, d, s);
}

template int transpose_one<float>(ibvt_coupling*, int, hipStream_t);
template int transpose_one<double>(ibvt_coupling*, int, hipStream_t);

}  // namespace ibvt
