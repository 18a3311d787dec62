// B^dT over the touched fluid nodes (the force transfer's operator).
//
// The touched fluid nodes are compacted with a prefix sum over the lattice;
// the nonzeros of B^d, taken in their CSR order (row i ascending, then
// column), are sorted by compacted column with a stable LSD radix sort
// (digit passes of at most 8 bits, sort.hip) that carries each nonzero's
// (value, row) along, so each row of B^dT lists its vertices in ascending
// order; the last pass writes B^dT's columns, values and row pointers
// directly (no gather by permutation follows).  Small
// operators take a counting sort instead (column counts, their prefix sum,
// a scatter into slots, then each row of B^dT put in vertex order by
// ranking).  No value is reduced and no position depends on timing: the
// result is deterministic either way.
#include <climits>
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

// A nonzero carried through the sort: its value and its row.
template <typename T>
using ValRow = std::conditional_t<std::is_same<T, float>::value, SortVal32, SortVal64>;

// keys[k] = compacted column of nonzero k, vr[k] = (value, row).
// kKeyLanes lanes per row (coalesced reads and writes).
constexpr int kKeyLanes = 16;
template <typename T>
__global__ __launch_bounds__(256) void k_keys(int64_t n_rows, const int64_t* __restrict__ rowptr,
                                              const int32_t* __restrict__ col,
                                              const T* __restrict__ val,
                                              const int64_t* __restrict__ cidx,
                                              int32_t* __restrict__ keys,
                                              ValRow<T>* __restrict__ vr) {
  const int64_t i = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / kKeyLanes;
  const int lane = threadIdx.x % kKeyLanes;
  if (i >= n_rows) return;
  for (int64_t k = rowptr[i] + lane; k < rowptr[i + 1]; k += kKeyLanes) {
    keys[k] = int32_t(cidx[col[k]]);
    ValRow<T> x;
    x.v = val[k];
    x.r = int32_t(i);
    vr[k] = x;
  }
}

// Counting sort for small operators (below kCountingNnz nonzeros), where
// the radix sort's fixed passes and launches dominate.  tcnt[c] = nonzeros
// of B^d in compacted column c (integer atomics).
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

// Below this many nonzeros the counting sort is faster; at 34M its two
// passes of device-scope atomics make it slower than the radix sort.
constexpr int64_t kCountingNnz = int64_t(4) << 20;

inline unsigned blocks_for(int64_t n, int threads) {
  return unsigned(ceil_div(n > 0 ? n : 1, threads));
}

int end_bit_for(int64_t n) {
  int b = 1;
  while ((int64_t(1) << b) < n + 1) ++b;
  return b;
}

}  // namespace

template <typename T>
int transpose_one(ibvt_coupling* c, int d, hipStream_t s) {
  const int64_t nf = c->n_fluid[d];
  const Csr& B = c->B[d];
  Csr& Bt = c->Bt[d];
  int st;
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
  if (B.nnz < kCountingNnz) {
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
  // sort scratch: keys and (value, row) pairs, their copies for the
  // alternating digit passes, and the passes' histogram
  const int end_bit = end_bit_for(touched);
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  const size_t n4 = al(size_t(B.nnz) * sizeof(int32_t));
  const size_t nv = al(size_t(B.nnz) * sizeof(ValRow<T>));
  const size_t sb = sort_pass_bytes(B.nnz, 8);
  if ((st = ensure(c, c->tbuf, 2 * n4 + 2 * nv + sb + 256))) return st;
  char* base = c->tbuf.as<char>();
  int32_t* keys = reinterpret_cast<int32_t*>(base);
  int32_t* keys_tmp = reinterpret_cast<int32_t*>(base + n4);
  ValRow<T>* vr = reinterpret_cast<ValRow<T>*>(base + 2 * n4);
  ValRow<T>* vr_tmp = reinterpret_cast<ValRow<T>*>(base + 2 * n4 + nv);
  void* scratch = base + 2 * n4 + 2 * nv;
  k_keys<T><<<blocks_for(c->n_vert * kKeyLanes, 256), 256, 0, s>>>(
      c->n_vert, B.rowptr.as<int64_t>(), B.col.as<int32_t>(), B.val.as<T>(),
      c->cidx.as<int64_t>(), keys, vr);
  if ((st = hip_check(hipGetLastError(), "transpose keys launch"))) return st;
  return sort_to_csr<ValRow<T>>(c, B.nnz, end_bit, keys, vr, keys_tmp, vr_tmp, scratch, s,
                                Bt.col.as<int32_t>(), Bt.val.as<T>(), Bt.rowptr.as<int64_t>(),
                                touched);
}

template int transpose_one<float>(ibvt_coupling*, int, hipStream_t);
template int transpose_one<double>(ibvt_coupling*, int, hipStream_t);

}  // namespace ibvt
