// Assembly of the mortar matrices B^d (Section 2.3, steps (I)-(IV)).
//
//  k_tet_prep      per tet: bounding box -> cell index range on each
//                  component's lattice (replaces the tree search: on a
//                  rectilinear grid the overlap candidates of a tet are an
//                  index box), volume, geometry record, validity checks.
//  scan            candidate (tet, component, cell) pair offsets.
//  k_order_count / k_order_scatter
//                  per chunk: the pairs' 16-byte descriptors in clip
//                  order (key: the cell planes the tet straddles, in
//                  classes by cut count: vertex slots 10, 12, 16), counted
//                  and placed per (tet, key) group from the cell ranges.
//  k_clip<T,MAXV>  one lane per pair: clip the tet by the straddled cell
//                  planes in double (vertex graph in LDS), fan the piece
//                  into sub-tetrahedra and store them as records.
//  k_integrate<T>  one lane per record: its 32 cell-local moments, summed
//                  per pair; then one lane per pair turns them into the 32
//                  values ∫ λ_i N_j.
//  k_row_box / k_rows<T> / k_rows_compact<T>
//                  each (solid vertex, component) row gathered in an LDS
//                  node box after each chunk's integration (rows whose
//                  pairs span chunks keep double partial sums between
//                  chunks), pairs added in a fixed order (deterministic,
//                  no value atomics outside LDS), written column-sorted,
//                  then compacted into CSR.
//  transpose       B^dT over the touched fluid nodes (transpose.hip).
//  masses          lumped m_i = Σ_{T∋i} |T|/4 and the consistent P1 mass
//                  matrix |T|(1+δ_il)/20 (Section 2.1), per vertex in
//                  incident-tet order.

#include "geometry.hpp"
#include "internal.hpp"

#include <climits>
#include <cstdlib>

namespace ibvt {

namespace {

constexpr int kRowNodes = 80;   // LDS box nodes per row per pass in k_rows

__device__ __forceinline__ int upper_bound_d(const double* L, int n, double x) {
  int lo = 0, hi = n;  // first index with L[idx] > x
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (L[mid] <= x) lo = mid + 1; else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ int lower_bound_d(const double* L, int n, double x) {
  int lo = 0, hi = n;  // first index with L[idx] >= x
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (L[mid] < x) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// ---------------------------------------------------------------------------
// topology: vertex -> incident tets
// ---------------------------------------------------------------------------

// K vertices per element: 4 (tetrahedra) or 3 (triangles, the planar case).
template <int K>
__global__ void k_vt_count(int64_t n_t, int64_t n_v, const int32_t* __restrict__ tets,
                           unsigned long long* __restrict__ deg, unsigned* flags) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= n_t) return;
  int v[K];
  bool bad = false;
  for (int k = 0; k < K; ++k) {
    v[k] = tets[K * t + k];
    bad |= (v[k] < 0) || (int64_t(v[k]) >= n_v);
  }
  for (int a = 0; a < K; ++a)
    for (int b = a + 1; b < K; ++b) bad |= (v[a] == v[b]);
  if (bad) {
    atomicOr(flags, kFlagValence);
    return;
  }
  for (int k = 0; k < K; ++k) atomicAdd(&deg[v[k]], 1ull);
}

template <int K>
__global__ void k_vt_fill(int64_t n_t, const int32_t* __restrict__ tets,
                          const int64_t* __restrict__ vt_ptr, unsigned long long* __restrict__ cur,
                          int32_t* __restrict__ vt_tet) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= n_t) return;
  for (int k = 0; k < K; ++k) {
    const int v = tets[K * t + k];
    const int64_t pos = vt_ptr[v] + int64_t(atomicAdd(&cur[v], 1ull));
    vt_tet[pos] = int32_t(t);
  }
}

__global__ void k_sort_segments_i32(int64_t n, const int64_t* __restrict__ ptr,
                                    int32_t* __restrict__ key) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t b = ptr[i], e = ptr[i + 1];
  for (int64_t k = b + 1; k < e; ++k) {
    const int32_t x = key[k];
    int64_t j = k - 1;
    while (j >= b && key[j] > x) {
      key[j + 1] = key[j];
      --j;
    }
    key[j + 1] = x;
  }
}

// Consistent-mass pattern: distinct vertices of the incident elements.
template <int K, bool FILL>
__global__ void k_mass_pattern(int64_t n_v, const int64_t* __restrict__ vt_ptr,
                               const int32_t* __restrict__ vt_tet, const int32_t* __restrict__ tets,
                               int64_t* __restrict__ rowcnt, const int64_t* __restrict__ rowptr,
                               int32_t* __restrict__ col) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n_v) return;
  const int64_t b = vt_ptr[i], e = vt_ptr[i + 1];
  int cur = -1;
  int64_t cnt = 0;
  int64_t pos = FILL ? rowptr[i] : 0;
  for (;;) {
    int nxt = INT_MAX;
    for (int64_t k = b; k < e; ++k) {
      const int64_t t = vt_tet[k];
      for (int q = 0; q < K; ++q) {
        const int v = tets[K * t + q];
        if (v > cur && v < nxt) nxt = v;
      }
    }
    if (nxt == INT_MAX) break;
    if (FILL) col[pos++] = nxt;
    ++cnt;
    cur = nxt;
  }
  if (!FILL) rowcnt[i] = cnt;
}

// ---------------------------------------------------------------------------
// per-tet preparation
// ---------------------------------------------------------------------------

__global__ void k_tet_prep(int64_t n_t, const double* __restrict__ X,
                           const int32_t* __restrict__ tets, const double* __restrict__ lat,
                           LatDesc ld, double* __restrict__ tetvol, CellRange* __restrict__ rng,
                           int64_t* __restrict__ cnt, double* __restrict__ tetrec,
                           double* __restrict__ tetgrad, unsigned* flags,
                           unsigned long long* counters) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  bool zero = false;
  if (t < n_t) {
    double P[4][3];
    bool finite = true;
    for (int k = 0; k < 4; ++k) {
      const int64_t v = tets[4 * t + k];
      for (int e = 0; e < 3; ++e) {
        P[k][e] = X[3 * v + e];
        finite &= isfinite(P[k][e]);
      }
    }
    double mn[3], mx[3];
    for (int e = 0; e < 3; ++e) {
      mn[e] = fmin(fmin(P[0][e], P[1][e]), fmin(P[2][e], P[3][e]));
      mx[e] = fmax(fmax(P[0][e], P[1][e]), fmax(P[2][e], P[3][e]));
    }
    double a[3], b[3], c[3];
    for (int e = 0; e < 3; ++e) {
      a[e] = P[1][e] - P[0][e];
      b[e] = P[2][e] - P[0][e];
      c[e] = P[3][e] - P[0][e];
    }
    const double det = a[0] * (b[1] * c[2] - b[2] * c[1]) - a[1] * (b[0] * c[2] - b[2] * c[0]) +
                       a[2] * (b[0] * c[1] - b[1] * c[0]);
    const double vol = fabs(det) / 6.0;
    tetvol[t] = finite ? vol : 0.0;
    {
      TetGeom G;
      for (int k = 0; k < 4; ++k)
        for (int e = 0; e < 3; ++e) G.V[k][e] = P[k][e];
      tet_geom(G);
      double r[kTetRec];
      store_tet_rec(G, r);
      store_row<kTetRec>(tetrec + t * kTetRec, r);
      double g[12];
      for (int k = 0; k < 4; ++k)
        for (int e = 0; e < 3; ++e) g[3 * k + e] = G.g[k][e];
      store_row<12>(tetgrad + t * 12, g);
    }
    zero = finite && (vol == 0.0);
    if (!finite) atomicOr(flags, kFlagNonFinite);
    for (int d = 0; d < 3; ++d) {
      CellRange r;
      bool ok = finite && !zero;
      for (int e = 0; e < 3; ++e) {
        const double* L = lat + ld.off[3 * d + e];
        const int n = ld.n[3 * d + e];
        if (!(mn[e] >= L[0] && mx[e] <= L[n - 1])) {
          if (finite) atomicOr(flags, kFlagOutOfGrid);
          ok = false;
          r.lo[e] = 0;
          r.n[e] = 0;
          continue;
        }
        int lo = upper_bound_d(L, n, mn[e]) - 1;
        lo = min(max(lo, 0), n - 2);
        int hi = lower_bound_d(L, n, mx[e]) - 1;
        hi = min(max(hi, lo), n - 2);
        r.lo[e] = lo;
        r.n[e] = hi - lo + 1;
      }
      if (!ok) r.n[0] = r.n[1] = r.n[2] = 0;
      rng[d * n_t + t] = r;
      cnt[d * n_t + t] = int64_t(r.n[0]) * r.n[1] * r.n[2];
      if (int64_t(r.n[0]) * r.n[1] * r.n[2] > kMaxTetCells) atomicOr(flags, kFlagTetSpan);
    }
  }
  const uint64_t zm = ballot64(zero);
  if (lane_id() == 0 && zm) atomicAdd(&counters[kCntZeroTets], (unsigned long long)popc64(zm));
}

// ---------------------------------------------------------------------------
// clip + integrate, one lane per (tet, component, cell) pair
// ---------------------------------------------------------------------------

// The clip order of a chunk, from the cell ranges alone.  Which of the six
// cell planes a pair's tet straddles follows from indices: the low plane of
// cell ci cuts the tet iff ci > the first cell of the tet's range along that
// axis, the high plane iff ci < the last.  Sort key = class · 64 + pattern
// (the straddled planes, two bits per axis), class 0: <= 3 cuts, 1: 4,
// 2: >= 5 (classes need 10, 12, 16 vertex slots); ordering the pairs by
// key gives every wave the same sequence of clips.  Along an axis with n
// cells the pairs fall into at most three runs (first cell, inner cells,
// last cell), so a (component, tet) item's pairs form at most 27 groups of
// one key each, counted and placed per group:
//   k_order_count    per block of kOrderItems items: pairs per key (LDS
//                    integer atomics) → hist[key][block];
//   scan             → the first place of each (key, block), key-major, so
//                    entry 64·k·blocks is where class k starts;
//   k_order_scatter  each item takes chunk-local places for its groups
//                    from its block's running offsets (LDS atomics: the
//                    order within a key depends on timing, which changes no
//                    result: a pair's clip and its records depend on the
//                    pair alone) and writes the groups' descriptors
//                    (pair_desc's fields), and the owner (the item's index)
//                    of each of its pairs.
constexpr int kOrderItems = 256;

struct AxisRuns {
  int n;          // runs along the axis (1, 2 or 3)
  int start[3];   // first cell of each run (range-relative)
  int count[3];   // cells in each run
  int bits[3];    // straddled planes of the run's cells: 1 low, 2 high
};

__device__ __forceinline__ AxisRuns axis_runs(int n) {
  AxisRuns a;
  if (n <= 1) {
    a.n = 1;
    a.start[0] = 0; a.count[0] = n; a.bits[0] = 0;
  } else {
    a.n = n > 2 ? 3 : 2;
    a.start[0] = 0; a.count[0] = 1; a.bits[0] = 2;
    a.start[1] = n - 1; a.count[1] = 1; a.bits[1] = 1;
    a.start[2] = 1; a.count[2] = n - 2; a.bits[2] = 3;
  }
  return a;
}

__device__ __forceinline__ int order_key(int pattern) {
  const int cuts = __popc(pattern);
  return (cuts <= 3 ? 0 : (cuts == 4 ? 1 : 2)) * 64 + pattern;
}

__global__ __launch_bounds__(kOrderItems) void k_order_count(int64_t tc0, int64_t n_items,
                                                             const CellRange* __restrict__ rng,
                                                             int32_t* __restrict__ hist) {
  __shared__ int32_t h[256];
  const int64_t nb = gridDim.x;
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t w = int64_t(blockIdx.x) * kOrderItems + threadIdx.x;
  if (w < n_items) {
    const CellRange r = rng[tc0 + w];
    if (int64_t(r.n[0]) * r.n[1] * r.n[2] > 0) {
      const AxisRuns ax = axis_runs(r.n[0]), ay = axis_runs(r.n[1]), az = axis_runs(r.n[2]);
      for (int c = 0; c < az.n; ++c)
        for (int b = 0; b < ay.n; ++b)
          for (int a = 0; a < ax.n; ++a) {
            const int cnt = ax.count[a] * ay.count[b] * az.count[c];
            if (cnt > 0)
              atomicAdd(&h[order_key(ax.bits[a] | (ay.bits[b] << 2) | (az.bits[c] << 4))], cnt);
          }
    }
  }
  __syncthreads();
  hist[int64_t(threadIdx.x) * nb + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(kOrderItems) void k_order_scatter(
    int64_t tc0, int64_t n_items, int64_t n_t, const CellRange* __restrict__ rng,
    const int64_t* __restrict__ pair_off, const int64_t* __restrict__ first,
    PairDesc* __restrict__ order, int32_t* __restrict__ owner) {
  __shared__ unsigned long long cur[256];
  const int64_t nb = gridDim.x;
  cur[threadIdx.x] = (unsigned long long)first[int64_t(threadIdx.x) * nb + blockIdx.x];
  __syncthreads();
  const int64_t w = int64_t(blockIdx.x) * kOrderItems + threadIdx.x;
  if (w >= n_items) return;
  const int64_t tc = tc0 + w;
  const CellRange r = rng[tc];
  if (int64_t(r.n[0]) * r.n[1] * r.n[2] == 0) return;
  const int d = (tc >= n_t) + (tc >= 2 * n_t);
  const uint32_t td = uint32_t(tc - int64_t(d) * n_t) | (uint32_t(d) << 30);
  const int64_t pb = pair_off[tc];
  const int64_t cnt_all = int64_t(r.n[0]) * r.n[1] * r.n[2];
  for (int64_t q = 0; q < cnt_all; ++q) owner[pb + q] = int32_t(tc);
  const AxisRuns ax = axis_runs(r.n[0]), ay = axis_runs(r.n[1]), az = axis_runs(r.n[2]);
  for (int c = 0; c < az.n; ++c)
    for (int b = 0; b < ay.n; ++b)
      for (int a = 0; a < ax.n; ++a) {
        const int cnt = ax.count[a] * ay.count[b] * az.count[c];
        if (cnt == 0) continue;
        const int key = order_key(ax.bits[a] | (ay.bits[b] << 2) | (az.bits[c] << 4));
        int64_t pos = int64_t(atomicAdd(&cur[key], (unsigned long long)cnt));
        for (int z = az.start[c]; z < az.start[c] + az.count[c]; ++z)
          for (int y = ay.start[b]; y < ay.start[b] + ay.count[b]; ++y)
            for (int x = ax.start[a]; x < ax.start[a] + ax.count[a]; ++x) {
              PairDesc o;
              o.p = int32_t(pb + x + int64_t(r.n[0]) * (y + int64_t(r.n[1]) * z));
              o.td = td;
              o.cell = uint64_t(uint32_t(r.lo[0] + x)) |
                       (uint64_t(uint32_t(r.lo[1] + y)) << kCellBits) |
                       (uint64_t(uint32_t(r.lo[2] + z)) << (2 * kCellBits));
              order[pos++] = o;  // chunk-local place
            }
      }
}

// Clip every (tet, component, cell) pair in double, one lane per pair, and
// store the fan sub-tetrahedra of the piece.  The pairs come as descriptors
// in clip order (pattern-sorted).  The grid is sized to the resident waves
// and each wave loops over batches of 64 pairs.  A wave takes store space in
// chunks of `chunk` records (one atomic per chunk, not per batch:
// same-address atomics serialise device-wide) and hands each batch a
// contiguous block of its chunk, so every pair's records are contiguous and
// in fan order; the unused tail of a chunk is left empty.  The counters are
// summed per wave and added once at the end.
template <typename T, int MAXV>
__global__ __launch_bounds__(kWave) void k_clip(
    const int64_t* __restrict__ cls_first, const int64_t* __restrict__ cls_end,
    const PairDesc* __restrict__ desc_all, const double* __restrict__ tetrec,
    const double* __restrict__ lat, LatDesc ld, double drop_rel, T* __restrict__ pool,
    int64_t pool_cap, uint64_t* __restrict__ pinfo, unsigned long long* pool_used,
    unsigned* flags, unsigned long long* counters) {
  __shared__ double sx[MAXV * kWave], sy[MAXV * kWave], sz[MAXV * kWave];
  __shared__ uint32_t snb[MAXV * kWave];
  const int lane = threadIdx.x;
  // this class's stretch of the pair order (read here, so the host needs
  // no class sizes); chunk ~ 1/8 of a wave's expected records (about 3 per
  // pair), so the unused chunk tails stay a few percent of the store
  const int64_t first = *cls_first;
  const int64_t n_list = *cls_end - first;
  const PairDesc* __restrict__ desc = desc_all + first;
  const int chunk = int(min<int64_t>(
      2048, max<int64_t>(1, (3 * n_list) / (8 * int64_t(gridDim.x)))));
  const PolyView P{sx + lane, sy + lane, sz + lane, snb + lane, kWave, (1u << MAXV) - 1u};
  unsigned long long nk = 0, nd = 0, ns = 0;
  ClipCount cc;
  unsigned long long cbase = 0;  // next free record of the wave's chunk
  int cleft = 0;                 // records left in it
  bool fail = false;
  for (int64_t p0 = int64_t(blockIdx.x) * kWave; p0 < n_list; p0 += int64_t(gridDim.x) * kWave) {
    const bool active = p0 + lane < n_list;
    TetGeom G;
    double lo[3], hi[3];
    int64_t p = 0;
    uint32_t live = 0;
    uint64_t seen = 0;
    int want = 0;
    bool ok = true;
    if (active) {
      int d, ci[3];
      int64_t t;
      desc_cell(desc[p0 + lane], lat, ld, p, d, t, ci, lo, hi);
      double r[kTetRec];
      load_row<kTetRec>(tetrec + t * kTetRec, r);
      load_tet_box(G, r);
      live = poly_init_tet(P, G.V, G.det < 0.0);
      ok = poly_clip_box<MAXV>(P, live, lo, hi, G.mn, G.mx, &cc);
      if (ok) {
        want = poly_fan_prepare(P, live, seen);
        if (want < 0) {
          ok = false;
          want = 0;
        }
      }
    }
    int incl = want;
    for (int o = 1; o < kWave; o <<= 1) {
      const int y = __shfl_up(incl, o, kWave);
      if (lane >= o) incl += y;
    }
    const int wave_total = __shfl(incl, kWave - 1, kWave);
    if (wave_total > cleft) {
      const int take = wave_total > chunk ? wave_total : chunk;
      unsigned long long b = 0;
      if (lane == 0) b = atomicAdd(pool_used, (unsigned long long)take);
      cbase = __shfl(b, 0, kWave);
      cleft = take;
    }
    const unsigned long long wbase = cbase;
    cbase += unsigned(wave_total);
    cleft -= wave_total;
    if (active) {
      const int64_t my = int64_t(wbase) + (incl - want);
      const bool fits = my + want <= pool_cap;
      double vol6 = 0.0;
      int nsub = 0;
      if (ok && want > 0) {
        T* rec = pool + my * kRecord;
        ok = emit_subtets<T>(
            P, live, seen, lo, hi,
            [&](int k, const T(&r)[kRecord]) {
              if (fits && k < want) store_row<kRecord>(rec + int64_t(k) * kRecord, r);
            },
            vol6, nsub);
      }
      if (ok && nsub != want) ok = false;
      ns += unsigned(nsub);
      if (!ok) {
        fail = true;
        pinfo[p] = 0;
      } else {
        const double cv = (hi[0] - lo[0]) * (hi[1] - lo[1]) * (hi[2] - lo[2]);
        const double vol = vol6 * cv / 6.0;
        const bool kp = vol > drop_rel * (fabs(G.det) / 6.0);
        // records past the store's end were not written: the pair reads as
        // empty, and the host sees the overflow and runs the clip again
        pinfo[p] = (kp && fits) ? ((uint64_t(my) << 8) | uint64_t(nsub)) : 0;
        if (kp) ++nk;
        else if (vol > 0.0) ++nd;
      }
    }
  }
  nk = wave_sum(nk);
  nd = wave_sum(nd);
  ns = wave_sum(ns);
  const unsigned long long ndist = wave_sum((unsigned long long)cc.dist);
  const unsigned long long ncut = wave_sum((unsigned long long)cc.cuts);
  const unsigned long long npl = wave_sum((unsigned long long)cc.planes);
  const uint64_t fm = ballot64(fail);
  if (lane == 0) {
    if (npl) atomicAdd(&counters[kCntPlanes], npl);
    if (nk) atomicAdd(&counters[kCntPieces], nk);
    if (nd) atomicAdd(&counters[kCntDropped], nd);
    if (ns) atomicAdd(&counters[kCntSubtets], ns);
    if (ndist) atomicAdd(&counters[kCntDist], ndist);
    if (ncut) atomicAdd(&counters[kCntCutPts], ncut);
    if (fm) atomicOr(flags, kFlagCapacity);
  }
}

// One wave per group of 64 consecutive pairs, whose records are contiguous:
// records are taken one per lane (balanced whatever the count per pair) and
// summed per pair in record order through LDS (deterministic).  Returns,
// for the group's dense record index s, the owning lane (largest j with
// excl_j <= s, excl = exclusive prefix of the per-pair counts).
__device__ __forceinline__ int owner_lane(int excl, int s) {
  int lo = 0, hi = kWave - 1;
#pragma unroll
  for (int it = 0; it < 6; ++it) {
    const int mid = (lo + hi + 1) >> 1;
    const int e = __shfl(excl, mid, kWave);
    if (e <= s) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// (III) integrate every stored sub-tetrahedron: its 32 moments (cell-local,
// centred) with the 11-point degree-4 rule, summed per pair in record order through
// LDS (deterministic) into pmom[pair][m] (rows of kMomPad).  Then each lane
// turns its pair's moments into the 4 x 8 values ∫ λ_i N_j, written to
// pval[i][pair - p_begin][j] (the chunk's pairs only; local-vertex major:
// each vertex row of a pair is 8 contiguous values, planes of plane_pairs
// pairs).
template <typename T>
__global__ __launch_bounds__(kWave) void k_integrate(
    int64_t plane_pairs, int64_t p_begin, int64_t p_end, int64_t n_t,
    const uint64_t* __restrict__ pinfo, const T* __restrict__ pool,
    const int32_t* __restrict__ owner, const int64_t* __restrict__ pair_off,
    const CellRange* __restrict__ rng, const double* __restrict__ tetrec,
    const double* __restrict__ lat, LatDesc ld, uint8_t* __restrict__ keep,
    T* __restrict__ pval, T* __restrict__ pmom, int dual) {
  __shared__ __align__(16) T red[kWave][kMomLds];  // a record's moments per row, padded
  const int lane = threadIdx.x;
  const int64_t g0 = p_begin + int64_t(blockIdx.x) * kWave;
  const int64_t pj = g0 + lane;
  int cnt = 0;
  int64_t beg = 0;
  if (pj < p_end) {
    const uint64_t pi = pinfo[pj];
    cnt = int(pi & 0xff);
    beg = int64_t(pi >> 8);
    keep[pj] = cnt > 0 ? 1 : 0;
  }
  int incl = cnt;
  for (int o = 1; o < kWave; o <<= 1) {
    const int y = __shfl_up(incl, o, kWave);
    if (lane >= o) incl += y;
  }
  const int excl = incl - cnt;
  const int total = __shfl(incl, kWave - 1, kWave);
  T run = T(0);
  for (int s0 = 0; s0 < total; s0 += kWave) {
    const int s = s0 + lane;
    const int j = owner_lane(excl, s);
    const int ex_j = __shfl(excl, j, kWave);
    const int in_j = __shfl(incl, j, kWave);
    const long long bj = __shfl((long long)beg, j, kWave);
    T M[kMom];
#pragma unroll
    for (int k = 0; k < kMom; ++k) M[k] = T(0);
    if (s < total) {
      T r[kRecord];
      load_row<kRecord>(pool + (int64_t(bj) + (s - ex_j)) * kRecord, r);
      T y[4][3];
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int e = 0; e < 3; ++e) y[v][e] = r[v * 3 + e];
      subtet_moments<T>(y, subtet_det<T>(y[0], y[1], y[2], y[3]), M);
    }
    {
      T Mp[kMomLds];
#pragma unroll
      for (int k = 0; k < kMom; ++k) Mp[k] = M[k];
#pragma unroll
      for (int k = kMom; k < kMomLds; ++k) Mp[k] = T(0);
      store_row<kMomLds>(&red[lane][0], Mp);  // 16-byte LDS writes
    }
    // the record that ends each pair, and each record's pair, are uniform
    // across the wave: a ballot and lane reads (no LDS)
    const uint64_t last = ballot64((s < total) && (s + 1 == in_j));
    __syncthreads();
    if (lane < kMom) {
      const int rows = min(kWave, total - s0);
      for (int r = 0; r < rows; ++r) {
        run += red[r][lane];
        if ((last >> r) & 1ull) {
          pmom[(g0 + __builtin_amdgcn_readlane(j, r)) * kMomPad + lane] = run;
          run = T(0);
        }
      }
    }
    __syncthreads();
  }
  // the block barrier above orders these reads after the other lanes' writes
  if (cnt > 0) {
    T M[kMomPad];
    load_row<kMomPad>(pmom + pj * kMomPad, M);
    int d, ci[3];
    int64_t t;
    double lo[3], hi[3];
    pair_cell(pj, n_t, owner, pair_off, rng, lat, ld, d, t, ci, lo, hi);
    double rec[kTetRec];
    load_row<kTetRec>(tetrec + t * kTetRec, rec);
    T LA[4], LG[4][3];
    rec_cell_lambda<T>(rec, lo, hi, LA, LG);
    const T sc = T(-(hi[0] - lo[0]) * (hi[1] - lo[1]) * (hi[2] - lo[2]) / 6.0);
    const int64_t plane = plane_pairs * 8;
    T b[4][8];
    mom_to_b<T>(M, LA, LG, [&](int i, int jj, T v) { b[i][jj] = sc * v; });
    if (dual) {
      // dual multipliers ψ_i = 5λ_i − Σ_k λ_k: ∫ ψ_i N_j = 5 b_ij − Σ_k b_kj
#pragma unroll
      for (int jj = 0; jj < 8; ++jj) {
        const T sum = b[0][jj] + b[1][jj] + b[2][jj] + b[3][jj];
#pragma unroll
        for (int i = 0; i < 4; ++i) b[i][jj] = T(5) * b[i][jj] - sum;
      }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) store_row<8>(pval + i * plane + (pj - p_begin) * 8, b[i]);
  }
}

// ---------------------------------------------------------------------------
// row gather: one wavefront per (vertex, component)
// ---------------------------------------------------------------------------

// Node box of row (vertex i, component d): the union of the cell ranges of
// the incident tets, as lo[3] and extent[3] (nodes); its size bounds the row.
// chunks = first | last << 8: the pair chunks holding the row's pairs (0xff:
// the row has none).
struct RowBox {
  int32_t lo[3];
  int32_t n[3];
  int32_t chunks;
};

// The (component, tet) ranges of the pair chunks: chunk k holds the items
// [at[k], at[k + 1]).
struct ChunkBounds {
  int64_t at[kMaxChunks + 1];
  int n;
};

__device__ __forceinline__ int chunk_of(const ChunkBounds& cb, int64_t tc) {
  int k = 0;
  for (int j = 1; j < cb.n; ++j) k += tc >= cb.at[j] ? 1 : 0;
  return k;
}

// kBoxG lanes per row: each takes every kBoxG-th incident tet, then the
// group reduces its bounds with lane shuffles.  Also the row's first and
// last pair chunk; a row without pairs gets rownnz = 0 here (no chunk
// gathers it).
constexpr int kBoxG = 16;

__global__ __launch_bounds__(256) void k_row_box(int64_t n_v, int64_t n_t, ChunkBounds cb,
                                                 const int64_t* __restrict__ vt_ptr,
                                                 const int32_t* __restrict__ vt_tet,
                                                 const CellRange* __restrict__ rng,
                                                 RowBox* __restrict__ box,
                                                 int64_t* __restrict__ cap,
                                                 int64_t* __restrict__ rownnz) {
  const int64_t w = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / kBoxG;
  const int g = threadIdx.x % kBoxG;
  const bool active = w < 3 * n_v;
  int bmin[3] = {INT_MAX, INT_MAX, INT_MAX}, bmax[3] = {INT_MIN, INT_MIN, INT_MIN};
  int cmin = INT_MAX, cmax = INT_MIN;
  if (active) {
    const int d = int(w / n_v);
    const int64_t i = w - int64_t(d) * n_v;
    for (int64_t k = vt_ptr[i] + g; k < vt_ptr[i + 1]; k += kBoxG) {
      const int64_t tc = int64_t(d) * n_t + vt_tet[k];
      const CellRange r = rng[tc];
      if (int64_t(r.n[0]) * r.n[1] * r.n[2] == 0) continue;
      for (int e = 0; e < 3; ++e) {
        bmin[e] = min(bmin[e], r.lo[e]);
        bmax[e] = max(bmax[e], r.lo[e] + r.n[e]);
      }
      const int ch = chunk_of(cb, tc);
      cmin = min(cmin, ch);
      cmax = max(cmax, ch);
    }
  }
#pragma unroll
  for (int o = kBoxG / 2; o > 0; o >>= 1) {
    for (int e = 0; e < 3; ++e) {
      bmin[e] = min(bmin[e], __shfl_xor(bmin[e], o, kWave));
      bmax[e] = max(bmax[e], __shfl_xor(bmax[e], o, kWave));
    }
    cmin = min(cmin, __shfl_xor(cmin, o, kWave));
    cmax = max(cmax, __shfl_xor(cmax, o, kWave));
  }
  if (!active || g != 0) return;
  RowBox b;
  int64_t sz = 1;
  for (int e = 0; e < 3; ++e) {
    b.lo[e] = bmin[e] <= bmax[e] ? bmin[e] : 0;
    b.n[e] = bmin[e] <= bmax[e] ? bmax[e] - bmin[e] + 1 : 0;
    sz *= b.n[e];
  }
  b.chunks = cmin <= cmax ? (cmin | (cmax << 8)) : (0xff | (0xff << 8));
  box[w] = b;
  cap[w] = sz;
  if (cmin > cmax) rownnz[w] = 0;
}

// Spill capacity of each row: its box size if its pairs lie in more than one
// chunk (the partial sums wait between the chunks), else 0 (in place).
__global__ void k_row_spill_cap(int64_t n_rows, const RowBox* __restrict__ box,
                                int64_t* __restrict__ cap) {
  const int64_t w = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (w >= n_rows) return;
  const int ch = box[w].chunks;
  if ((ch & 0xff) == 0xff || (ch & 0xff) == (ch >> 8)) cap[w] = 0;
}

// Exact floor(q / n) for q < 2^16 and 1 <= n < 2^16 as a multiply-high by
// m = ceil(2^32 / n): with m n = 2^32 + e, 0 <= e < n, the error term q e / 2^32
// stays below 1.  n = 1 (m = 2^32) is coded as m = 0.
__device__ __forceinline__ uint32_t magic_div(uint32_t n) {
  return n <= 1u ? 0u : 0xFFFFFFFFu / n + 1u;
}
__device__ __forceinline__ uint32_t div_magic(uint32_t q, uint32_t m) {
  return m ? __umulhi(q, m) : q;
}

constexpr int kRowsPerWave = 8;  // rows served by one wavefront in k_rows

// Maximum of x over the kRowsPerWave row groups of a wavefront (lanes
// hl, hl + H, ...), for loop bounds common to all of them.
__device__ __forceinline__ int64_t rows_max(int64_t x) {
  for (int o = kWave / kRowsPerWave; o < kWave; o <<= 1) x = max(x, __shfl_xor(x, o, kWave));
  return x;
}

// Gather the pieces of the incident tets into the row's node box, kept in
// LDS kRowNodes nodes at a time.  Each wavefront serves kRowsPerWave rows,
// H = 64 / kRowsPerWave lanes each, so the memory latency of one row's steps
// overlaps the others'.  The row's incident tets are taken in ascending
// order; for each, the lanes take its pairs (cells), H at a time, each lane
// loading its pair's 8 values of this vertex at once, and the values are
// added corner by corner: for one corner the cells of one tet are distinct,
// so are the nodes they add to, and every node sums its contributions in
// the order (tet, corner) whatever the timing (deterministic, no value
// atomics outside LDS).  Per batch of H incident tets, each tet's offsets
// are set up once in LDS.  Touched nodes are written column-sorted at
// tmp_off[w].
//
// One launch per pair chunk ch (items [tc_lo, tc_hi), pairs from p_base,
// values in pval planes of plane_pairs pairs), over the rows w_begin ..
// w_begin + n_rows - 1: a row takes the incident tets of the chunk.  A row
// whose pairs lie in several chunks starts from zero in its first chunk,
// keeps its node sums (double) and touched flags in its spill space between
// the chunks, and is written in its last; the chunks come in tet order, so
// every node still sums in (tet, corner) order.
template <typename T>
__global__ __launch_bounds__(256) void k_rows(
    int64_t n_v, int64_t n_t, int ch, int64_t tc_lo, int64_t tc_hi, int64_t p_base,
    int64_t plane_pairs, int64_t w_begin, int64_t n_rows, const int64_t* __restrict__ vt_ptr,
    const int32_t* __restrict__ vt_tet, const int32_t* __restrict__ tets,
    const CellRange* __restrict__ rng, const int64_t* __restrict__ pair_off,
    const uint8_t* __restrict__ keep, const T* __restrict__ pval, LatDesc ld,
    const RowBox* __restrict__ box, const int64_t* __restrict__ tmp_off,
    int32_t* __restrict__ tmp_col, T* __restrict__ tmp_val, int64_t* __restrict__ rownnz,
    const int64_t* __restrict__ spill_off, double* __restrict__ spill_acc,
    uint8_t* __restrict__ spill_flg) {
  constexpr int H = kWave / kRowsPerWave;  // lanes per row
  constexpr int RB = 4 * kRowsPerWave;     // rows per block
  __shared__ double s_acc[RB][kRowNodes];  // summed in double in both precisions
  __shared__ uint8_t s_flag[RB][kRowNodes];
  __shared__ int4 s_m0[RB][H], s_m1[RB][H];
  const int lane = lane_id();
  const int h = lane / H, hl = lane % H;
  const int slot = kRowsPerWave * (threadIdx.x / kWave) + h;  // this row's LDS slot
  const int64_t wl =
      kRowsPerWave * ((int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / kWave) + h;
  const int64_t w = w_begin + wl;
  double* acc = s_acc[slot];
  uint8_t* flg = s_flag[slot];
  int4* M0 = s_m0[slot];
  int4* M1 = s_m1[slot];
  RowBox b{};
  if (wl < n_rows) b = box[w];
  // rows of this chunk: first <= ch <= last
  const int cf = b.chunks & 0xff, cl = (b.chunks >> 8) & 0xff;
  const bool live = wl < n_rows && cf != 0xff && cf <= ch && ch <= cl;
  const bool first = cf == ch, last = cl == ch;
  const int64_t so = (live && !(first && last)) ? spill_off[w] : 0;
  const int d = live ? int(w / n_v) : 0;
  const int64_t i = live ? w - int64_t(d) * n_v : 0;
  const int bn0 = b.n[0], bn1 = b.n[1];
  const int64_t total = live ? int64_t(bn0) * bn1 * b.n[2] : 0;
  int64_t outpos = live ? tmp_off[w] : 0;
  const int64_t start = outpos;
  const int64_t NX = ld.n[3 * d + 0], NY = ld.n[3 * d + 1];
  const int64_t beg = live ? vt_ptr[i] : 0, end = live ? vt_ptr[i + 1] : 0;
  // box-linear offsets of the 8 corners of a cell
  int coff[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) coff[j] = (j & 1) + bn0 * (((j >> 1) & 1) + bn1 * (j >> 2));
  const int64_t vplane = plane_pairs * 8;
  // loop bounds common to the row groups of the wave (each masks its own work)
  const int64_t total_max = rows_max(total);
  const int64_t ntet = end - beg;
  const int64_t ntet_max = rows_max(ntet);
  for (int64_t c0 = 0; c0 < total_max; c0 += kRowNodes) {
    const int span = int(max<int64_t>(0, min<int64_t>(kRowNodes, total - c0)));
    for (int k = hl; k < span; k += H) {
      acc[k] = first ? 0.0 : spill_acc[so + c0 + k];
      flg[k] = first ? 0 : spill_flg[so + c0 + k];
    }
    for (int64_t kb0 = 0; kb0 < ntet_max; kb0 += H) {
      const int nk = int(max<int64_t>(0, min<int64_t>(H, ntet - kb0)));
      wave_lds_sync();
      if (hl < nk) {
        const int64_t t = vt_tet[beg + kb0 + hl];
        const int64_t tc = int64_t(d) * n_t + t;
        const CellRange r = rng[tc];
        const int4 tv = *reinterpret_cast<const int4*>(tets + 4 * t);
        const int li =
            (tv.y == int32_t(i)) ? 1 : (tv.z == int32_t(i)) ? 2 : (tv.w == int32_t(i)) ? 3 : 0;
        const int64_t kbase = pair_off[tc];  // pair of cell 0
        // box-linear offset of the tet's first cell in this pass
        const int off0 = int(int64_t(r.lo[0] - b.lo[0]) +
                             int64_t(bn0) * ((r.lo[1] - b.lo[1]) +
                                             int64_t(bn1) * (r.lo[2] - b.lo[2])) -
                             c0);
        // tets of other chunks add nothing here
        const int cnt = (tc >= tc_lo && tc < tc_hi) ? r.n[0] * r.n[1] * r.n[2] : 0;
        M0[hl] = make_int4(int(kbase & 0xffffffffll), int(kbase >> 32), li, cnt);
        M1[hl] = make_int4(r.n[0] | (r.n[1] << 16), off0,
                           int(magic_div(uint32_t(max(r.n[0], 1)))),
                           int(magic_div(uint32_t(max(r.n[1], 1)))));
      }
      wave_lds_sync();
      const int nk_max = int(rows_max(int64_t(nk)));
      for (int kk = 0; kk < nk_max; ++kk) {
        int4 m0 = make_int4(0, 0, 0, 0), m1 = make_int4(0, 0, 0, 0);
        if (kk < nk) {
          m0 = M0[kk];
          m1 = M1[kk];
        }
        const int cnt = m0.w;
        const int cnt_max = int(rows_max(int64_t(cnt)));
        const int64_t kbase = int64_t((unsigned long long)(unsigned)m0.x |
                                      ((unsigned long long)(unsigned)m0.y << 32));
        const uint32_t n0 = uint32_t(m1.x) & 0xffffu, n1 = uint32_t(m1.x) >> 16;
        for (int q0 = 0; q0 < cnt_max; q0 += H) {
          const int q = q0 + hl;
          bool add = false;
          int base = 0;
          T v[8];
          if (q < cnt) {
            const uint32_t qy = div_magic(uint32_t(q), uint32_t(m1.z));
            const int ix = int(uint32_t(q) - qy * n0);
            const uint32_t iz = div_magic(qy, uint32_t(m1.w));
            const int iy = int(qy - iz * n1);
            base = m1.y + ix + bn0 * (iy + bn1 * int(iz));
            const int64_t ko = kbase + q;
            add = keep[ko] != 0;
            load_row<8>(pval + int64_t(m0.z) * vplane + (ko - p_base) * 8, v);
          }
          // corner by corner: the cells of one tet are distinct, so one
          // corner's adds go to distinct nodes
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            const int lin = base + coff[j];
            if (add && lin >= 0 && lin < span) {
              __hip_atomic_fetch_add(&acc[lin], double(v[j]), __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_WAVEFRONT);
              flg[lin] = 1;
            }
          }
        }
      }
    }
    wave_lds_sync();
    if (!last)
      for (int k = hl; k < span; k += H) {
        spill_acc[so + c0 + k] = acc[k];
        spill_flg[so + c0 + k] = flg[k];
      }
    const int span_max = int(rows_max(int64_t(span)));
    for (int k0 = 0; k0 < span_max; k0 += H) {
      const int k = k0 + hl;
      const bool tch = last && k < span && flg[k] != 0;
      const uint32_t m = uint32_t(ballot64(tch) >> (H * h)) & uint32_t((uint64_t(1) << H) - 1);
      if (tch) {
        // the box lies inside the lattice, whose node count fits int32
        const uint32_t lin = uint32_t(c0 + k);
        const uint32_t r = lin / uint32_t(bn0);
        const uint32_t zq = r / uint32_t(bn1);
        const int64_t gx = b.lo[0] + int64_t(lin - r * uint32_t(bn0));
        const int64_t gy = b.lo[1] + int64_t(r - zq * uint32_t(bn1));
        const int64_t gz = b.lo[2] + int64_t(zq);
        const int64_t pos = outpos + __popc(m & ((1u << hl) - 1u));
        tmp_col[pos] = int32_t(gx + NX * (gy + NY * gz));
        tmp_val[pos] = T(acc[k]);
      }
      outpos += __popc(m);
    }
    wave_lds_sync();
  }
  if (live && last && hl == 0) rownnz[w] = outpos - start;
}

// Copy each row from the box-capacity scratch into the CSR arrays.
constexpr int kCompactLanes = 16;
template <typename T>
__global__ __launch_bounds__(256) void k_rows_compact(
    int64_t n_v, const int64_t* __restrict__ tmp_off, const int32_t* __restrict__ tmp_col,
    const T* __restrict__ tmp_val, const int64_t* __restrict__ rp0,
    const int64_t* __restrict__ rp1, const int64_t* __restrict__ rp2, int32_t* __restrict__ c0,
    int32_t* __restrict__ c1, int32_t* __restrict__ c2, T* __restrict__ v0, T* __restrict__ v1,
    T* __restrict__ v2) {
  // kCompactLanes lanes per row
  const int64_t w = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / kCompactLanes;
  const int lane = threadIdx.x % kCompactLanes;
  if (w >= 3 * n_v) return;
  const int d = int(w / n_v);
  const int64_t i = w - int64_t(d) * n_v;
  const int64_t* rp = d == 0 ? rp0 : (d == 1 ? rp1 : rp2);
  int32_t* col = d == 0 ? c0 : (d == 1 ? c1 : c2);
  T* val = d == 0 ? v0 : (d == 1 ? v1 : v2);
  const int64_t src = tmp_off[w], dst = rp[i], n = rp[i + 1] - rp[i];
  for (int64_t k = lane; k < n; k += kCompactLanes) {
    col[dst + k] = tmp_col[src + k];
    val[dst + k] = tmp_val[src + k];
  }
}

// ---------------------------------------------------------------------------
// masses
// ---------------------------------------------------------------------------

template <typename T>
__global__ void k_lumped(int64_t n_v, const int64_t* __restrict__ vt_ptr,
                         const int32_t* __restrict__ vt_tet, const double* __restrict__ tetvol,
                         double* __restrict__ m, T* __restrict__ minv) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n_v) return;
  double s = 0.0;
  for (int64_t k = vt_ptr[i]; k < vt_ptr[i + 1]; ++k) s += tetvol[vt_tet[k]];
  s *= 0.25;
  m[i] = s;
  minv[i] = (s > 0.0) ? T(1.0 / s) : T(0);
}

// Consistent mass rows M_il = Σ_{T ∋ i, l} |T|(1 + δ_il)/20, kMassLanes
// lanes per vertex (rows hold ~15 columns): lane k holds column k of the
// row, and the incident tets are broadcast one at a time within the lane
// group (sum order = incident-tet order).
constexpr int kMassLanes = 16;
__global__ __launch_bounds__(256) void k_mass_values(
    int64_t n_v, const int64_t* __restrict__ vt_ptr, const int32_t* __restrict__ vt_tet,
    const int32_t* __restrict__ tets, const double* __restrict__ tetvol,
    const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col,
    double* __restrict__ val, float* __restrict__ val32, double* __restrict__ dinv) {
  constexpr int H = kMassLanes;
  const int64_t i = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / H;
  const int hl = threadIdx.x % H;
  if (i >= n_v) return;  // whole lane groups leave together
  const int64_t rb = rowptr[i], re = rowptr[i + 1];
  const int64_t tb = vt_ptr[i], te = vt_ptr[i + 1];
  double diag = 0.0;
  for (int64_t c0 = rb; c0 < re; c0 += H) {
    const bool has = c0 + hl < re;
    const int l = has ? col[c0 + hl] : -1;
    double a = 0.0;
    for (int64_t k0 = tb; k0 < te; k0 += H) {
      const int nk = int(min<int64_t>(H, te - k0));
      int4 tv = make_int4(-1, -1, -1, -1);
      double w = 0.0;
      if (hl < nk) {
        const int64_t t = vt_tet[k0 + hl];
        tv = *reinterpret_cast<const int4*>(tets + 4 * t);
        w = tetvol[t] / 20.0;
      }
      for (int k = 0; k < nk; ++k) {
        const int v0 = __shfl(tv.x, k, H), v1 = __shfl(tv.y, k, H), v2 = __shfl(tv.z, k, H),
                  v3 = __shfl(tv.w, k, H);
        const double wk = __shfl(w, k, H);
        if (l == v0 || l == v1 || l == v2 || l == v3) a += (int64_t(l) == i) ? 2.0 * wk : wk;
      }
    }
    if (has) {
      val[c0 + hl] = a;
      if (val32) val32[c0 + hl] = float(a);
      if (int64_t(l) == i) diag = a;
    }
  }
  for (int o = H / 2; o > 0; o >>= 1) diag += __shfl_xor(diag, o, H);
  if (hl == 0) dinv[i] = (diag > 0.0) ? 1.0 / diag : 0.0;
}

inline unsigned blocks_for(int64_t n, int threads) {
  return unsigned(ceil_div(n > 0 ? n : 1, threads));
}

// Blocks of one wave each that the device keeps resident for kernel f
// (grid of a persistent launch).
template <typename F>
int resident_blocks(F f) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, kWave, 0) != hipSuccess ||
      cus <= 0 || per_cu <= 0) {
    (void)hipGetLastError();  // a failed query must not read as a launch error
    return 1 << 16;
  }
  return cus * per_cu;
}

}  // namespace

int read_back(ibvt_coupling* c, void* host, const void* dev, size_t bytes, hipStream_t s) {
  (void)c;
  int st = hip_check(hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, s), "read back");
  if (st) return st;
  return hip_check(hipStreamSynchronize(s), "stream sync");
}

int flags_status(unsigned f) {
  if (f & kFlagNonFinite) return set_error(IBVT_E_INVALID, "non-finite vertex coordinate");
  if (f & kFlagValence) return set_error(IBVT_E_INVALID, "tet vertex index out of range or repeated");
  if (f & kFlagOutOfGrid)
    return set_error(IBVT_E_OUT_OF_GRID, "a tet's bounding box leaves a velocity lattice's node hull");
  if (f & kFlagCapacity)
    return set_error(IBVT_E_CAPACITY, "clipped piece exceeded the 16-vertex capacity");
  if (f & kFlagTetSpan)
    return set_error(IBVT_E_CAPACITY, "an element spans more than 65535 cells of one lattice");
  return IBVT_OK;
}

int check_flags(ibvt_coupling* c, hipStream_t s) {
  unsigned f = 0;
  int st = read_back(c, &f, c->flags_dev.p, sizeof(unsigned), s);
  if (st) return st;
  return flags_status(f);
}

namespace {
constexpr int kMaxCounts = 24;
struct CountSrc {
  const int64_t* p[kMaxCounts];
};
__global__ void k_gather_counts(CountSrc src, int n, const unsigned* __restrict__ flags,
                                int64_t* __restrict__ out) {
  const int k = threadIdx.x;
  if (k < n) out[k] = *src.p[k];
  if (k == 0) out[kMaxCounts] = int64_t(*flags);
}
}  // namespace

int read_counts(ibvt_coupling* c, const int64_t* const* srcs, int n, int64_t* out, hipStream_t s) {
  if (n < 0 || n > kMaxCounts) return set_error(IBVT_E_INVALID, "read_counts: too many values");
  int st = ensure(c, c->rb, (kMaxCounts + 1) * sizeof(int64_t));
  if (st) return st;
  if (!c->host_rb) {
    void* h = nullptr;
    if ((st = hip_check(hipHostMalloc(&h, (kMaxCounts + 1) * sizeof(int64_t), hipHostMallocDefault),
                        "hipHostMalloc")))
      return st;
    c->host_rb = static_cast<int64_t*>(h);
  }
  CountSrc src{};
  for (int k = 0; k < n; ++k) src.p[k] = srcs[k];
  k_gather_counts<<<1, 64, 0, s>>>(src, n, c->flags_dev.as<unsigned>(), c->rb.as<int64_t>());
  if ((st = hip_check(hipGetLastError(), "count gather launch"))) return st;
  if ((st = hip_check(hipMemcpyAsync(c->host_rb, c->rb.p, (kMaxCounts + 1) * sizeof(int64_t),
                                     hipMemcpyDeviceToHost, s),
                      "read back")))
    return st;
  if ((st = hip_check(hipStreamSynchronize(s), "stream sync"))) return st;
  for (int k = 0; k < n; ++k) out[k] = c->host_rb[k];
  c->host_flags = unsigned(c->host_rb[kMaxCounts]);
  return IBVT_OK;
}

namespace {

// (Component, tet) items per pair chunk: 3 · 2^19 (about 10M pairs at the
// three-body workload's density), or IBVT_CHUNK_ITEMS from the environment
// (a positive integer; small values put small meshes through the chunked
// path, as the tests do).  At most kMaxChunks chunks either way.
int64_t chunk_items() {
  if (const char* e = std::getenv("IBVT_CHUNK_ITEMS")) {
    char* end = nullptr;
    const long long v = std::strtoll(e, &end, 10);
    if (end != e && *end == '\0' && v > 0) return int64_t(v);
  }
  return int64_t(3) << 19;
}

// The assembly's second stream and its events, made on first use (default
// priority, no timing) and destroyed with the handle.
int side_stream(ibvt_coupling* c) {
  int st;
  if (!c->side &&
      (st = hip_check(hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking), "stream")))
    return st;
  for (hipEvent_t* e : {&c->ev_fork, &c->ev_join, &c->ev_sorted})
    if (!*e && (st = hip_check(hipEventCreateWithFlags(e, hipEventDisableTiming), "event")))
      return st;
  return IBVT_OK;
}

// Without stored matrices (IBVT_NO_STORE_B): after the overlap candidates,
// only the solid masses and the per-(component, tet) buffer of the
// matrix-free products (3 n_t x 4 values) are built.
template <typename T>
int finish_matfree(ibvt_coupling* c, hipStream_t s) {
  int st;
  if ((st = ensure(c, c->pval, size_t(3 * c->n_tet + 1) * 4 * sizeof(T)))) return st;
  for (int d = 0; d < 3; ++d) {
    c->B[d].nnz = 0;
    c->Bt[d].nrows = 0;
    c->Bt[d].nnz = 0;
  }
  if ((st = solid_masses(c, s))) return st;
  if ((st = matfree_order(c, s))) return st;
  int64_t zero = 0;
  {
    const int64_t* src[1] = {
        reinterpret_cast<const int64_t*>(c->counters.as<unsigned long long>() + kCntZeroTets)};
    if ((st = read_counts(c, src, 1, &zero, s))) return st;
  }
  if ((st = flags_status(c->host_flags))) return st;
  const int64_t done = c->stats.assemblies + 1;
  c->stats = AsmStats{};
  c->stats.pairs = c->n_pairs;
  c->stats.zero_tets = zero;
  c->stats.assemblies = done;
  c->mom_valid = false;
  return IBVT_OK;
}

template <typename T>
int assemble_typed(ibvt_coupling* c, hipStream_t s) {
  const int64_t n_t = c->n_tet, n_v = c->n_vert;
  int st;
  unsigned* flags = c->flags_dev.as<unsigned>();
  auto* counters = c->counters.as<unsigned long long>();
  if ((st = hip_check(hipMemsetAsync(flags, 0, sizeof(unsigned), s), "memset"))) return st;
  if ((st = hip_check(hipMemsetAsync(counters, 0, kCntSlots * sizeof(unsigned long long), s),
                      "memset")))
    return st;
  // (I) overlap candidates
  {
    ProfScope ps("tet_prep", s);
  k_tet_prep<<<blocks_for(n_t, 256), 256, 0, s>>>(
      n_t, c->X.as<double>(), c->tets.as<int32_t>(), c->lat.as<double>(), c->ld,
      c->tetvol.as<double>(), c->rng.as<CellRange>(), c->cnt.as<int64_t>(), c->tetrec.as<double>(),
      c->tetgrad.as<double>(),
      flags, counters);
  }
  if ((st = hip_check(hipGetLastError(), "prep launch"))) return st;
  if ((st = scan_i64(c, c->cnt.as<int64_t>(), c->pair_off.as<int64_t>(), 3 * n_t, s))) return st;
  // The pairs are clipped and integrated in chunks of consecutive (component,
  // tet) ranges: the piece store holds one chunk's sub-tetrahedra, and a
  // chunk's tet records stay in the caches while its pairs are clipped.
  const int64_t n_tc = 3 * n_t;
  const int nchunk =
      int(std::min<int64_t>(kMaxChunks, std::max<int64_t>(1, n_tc / chunk_items())));
  ChunkBounds cb{};
  cb.n = nchunk;
  for (int k = 0; k <= nchunk; ++k) cb.at[k] = n_tc * k / nchunk;
  const int64_t* tc_at = cb.at;
  // (IV, set-up) each row's node box and its first and last chunk: from the
  // cell ranges alone.  Rows gather their pairs after each chunk's
  // integration, so the per-pair values are held for one chunk only; a row
  // whose pairs lie in several chunks keeps its partial sums in spill space
  // of its box size.
  if (!c->matrix_free) {
    if ((st = ensure(c, c->rowbox, size_t(3 * n_v + 1) * sizeof(RowBox)))) return st;
    if ((st = ensure(c, c->rowcap, size_t(3 * n_v + 1) * sizeof(int64_t)))) return st;
    if ((st = ensure(c, c->rowtmpoff, size_t(3 * n_v + 1) * sizeof(int64_t)))) return st;
    if ((st = ensure(c, c->rowspilloff, size_t(3 * n_v + 1) * sizeof(int64_t)))) return st;
    if ((st = ensure(c, c->rownnz, size_t(3 * n_v + 1) * sizeof(int64_t)))) return st;
    {
      ProfScope ps("rows_box", s);
      k_row_box<<<blocks_for(3 * n_v * kBoxG, 256), 256, 0, s>>>(
          n_v, n_t, cb, c->vt_ptr.as<int64_t>(), c->vt_tet.as<int32_t>(), c->rng.as<CellRange>(),
          c->rowbox.as<RowBox>(), c->rowcap.as<int64_t>(), c->rownnz.as<int64_t>());
    }
    if ((st = hip_check(hipGetLastError(), "row box launch"))) return st;
    if ((st = scan_i64(c, c->rowcap.as<int64_t>(), c->rowtmpoff.as<int64_t>(), 3 * n_v, s)))
      return st;
    k_row_spill_cap<<<blocks_for(3 * n_v, 256), 256, 0, s>>>(3 * n_v, c->rowbox.as<RowBox>(),
                                                            c->rowcap.as<int64_t>());
    if ((st = hip_check(hipGetLastError(), "row spill launch"))) return st;
    if ((st = scan_i64(c, c->rowcap.as<int64_t>(), c->rowspilloff.as<int64_t>(), 3 * n_v, s)))
      return st;
  }
  // read-back 1: the chunks' first pairs (the last entry is the pair count),
  // the row scratch and spill sizes, and status flags
  int64_t pat[kMaxChunks + 3];
  {
    const int64_t* src[kMaxChunks + 3];
    for (int k = 0; k <= nchunk; ++k) src[k] = c->pair_off.as<int64_t>() + tc_at[k];
    int nsrc = nchunk + 1;
    if (!c->matrix_free) {
      src[nsrc++] = c->rowtmpoff.as<int64_t>() + 3 * n_v;
      src[nsrc++] = c->rowspilloff.as<int64_t>() + 3 * n_v;
    }
    if ((st = read_counts(c, src, nsrc, pat, s))) return st;
  }
  if ((st = flags_status(c->host_flags))) return st;
  const int64_t n_pairs = pat[nchunk];
  if (n_pairs >= (int64_t(1) << 31) - 1)
    return set_error(IBVT_E_CAPACITY, "2^31 or more (tet, cell) pairs");
  c->n_pairs = n_pairs;
  if (c->matrix_free) return finish_matfree<T>(c, s);
  const int64_t tmp_total = pat[nchunk + 1], spill_total = pat[nchunk + 2];
  int64_t chunk_max = 0;
  for (int k = 0; k < nchunk; ++k) chunk_max = std::max(chunk_max, pat[k + 1] - pat[k]);
  if ((st = ensure(c, c->owner, size_t(n_pairs + 1) * sizeof(int32_t)))) return st;
  if ((st = ensure(c, c->keep, size_t(n_pairs + 1)))) return st;
  // one chunk's values: 4 planes (local vertex) of chunk_max pairs x 8
  if ((st = ensure(c, c->pval, size_t(chunk_max + 1) * 32 * sizeof(T)))) return st;
  if ((st = ensure(c, c->rowtmpcol, size_t(tmp_total + 1) * sizeof(int32_t)))) return st;
  if ((st = ensure(c, c->rowtmpval, size_t(tmp_total + 1) * sizeof(T)))) return st;
  const size_t spill_acc_bytes = (size_t(spill_total + 1) * sizeof(double) + 255) & ~size_t(255);
  if ((st = ensure(c, c->rowspill, spill_acc_bytes + size_t(spill_total + 1)))) return st;
  double* spill_acc = c->rowspill.as<double>();
  uint8_t* spill_flg = c->rowspill.as<uint8_t>() + spill_acc_bytes;
  if ((st = ensure(c, c->pmom, size_t(n_pairs + 1) * kMomPad * sizeof(T)))) return st;
  if ((st = ensure(c, c->pinfo, size_t(n_pairs + 1) * sizeof(uint64_t)))) return st;
  // the clip order of one chunk at a time, as pair descriptors
  if ((st = ensure(c, c->order, size_t(chunk_max + 1) * sizeof(PairDesc)))) return st;
  // per chunk: the pair descriptors in clip order (k_order_count, scan,
  // k_order_scatter); the scanned key counts give the clip launches their
  // class stretches on the device
  int64_t items_max = 1;
  for (int k = 0; k < nchunk; ++k) items_max = std::max(items_max, tc_at[k + 1] - tc_at[k]);
  const int64_t ob_max = ceil_div(items_max, kOrderItems);
  const size_t hb = (size_t(256 * ob_max) * sizeof(int32_t) + 255) & ~size_t(255);
  if ((st = ensure(c, c->pscan, hb + size_t(256 * ob_max + 1) * sizeof(int64_t)))) return st;
  int32_t* ohist = c->pscan.as<int32_t>();
  int64_t* ofirst = reinterpret_cast<int64_t*>(c->pscan.as<char>() + hb);
  if ((st = side_stream(c))) return st;
  bool masses_done = false;
  for (int attempt = 0; attempt < 2; ++attempt) {
    const int64_t want = std::max<int64_t>(int64_t(3.25 * double(chunk_max)) + 1024,
                                           c->pool_needed + c->pool_needed / 32 + 1024);
    if (int64_t(c->pool.cap / (kRecord * sizeof(T))) < want &&
        (st = ensure(c, c->pool, size_t(want) * kRecord * sizeof(T))))
      return st;
    c->pool_cap = int64_t(c->pool.cap / (kRecord * sizeof(T)));
    // clear the clip's counters (the zero-tet count of the preparation stays)
    for (int k : {int(kCntPieces), int(kCntDropped), int(kCntSubtets), int(kCntDist),
                  int(kCntCutPts), int(kCntPlanes)})
      if ((st = hip_check(hipMemsetAsync(counters + k, 0, sizeof(unsigned long long), s),
                          "memset")))
        return st;
    if ((st = hip_check(hipMemsetAsync(counters + kCntChunkPool, 0,
                                       kMaxChunks * sizeof(unsigned long long), s),
                        "memset")))
      return st;
    // Chunks with pairs, in order.  Per chunk: the clip's classes 12 and 16
    // run on the side stream beside class 10 (they fill its tail), and the
    // next chunk's pair order is made on the side stream while this chunk
    // integrates (the order and the sort scratch are free once the clip has
    // read them; the store is reused only after the integration).
    int live[kMaxChunks];
    int n_live = 0;
    for (int ch = 0; ch < nchunk; ++ch)
      if (pat[ch + 1] > pat[ch]) live[n_live++] = ch;
    auto order_chunk = [&](int ch, hipStream_t q) -> int {
      // the next chunk's order runs beside the integration: its span is
      // shared with it
      ProfScope ps(q == s ? "pair_order" : "pair_order_beside_integrate", q);
      const int64_t tc0 = tc_at[ch], items = tc_at[ch + 1] - tc_at[ch];
      const int64_t ob = ceil_div(items, kOrderItems);
      k_order_count<<<unsigned(ob), kOrderItems, 0, q>>>(tc0, items, c->rng.as<CellRange>(), ohist);
      int r = hip_check(hipGetLastError(), "order count launch");
      if (r) return r;
      if ((r = scan_i32_to_i64(c, ohist, ofirst, 256 * ob, q))) return r;
      k_order_scatter<<<unsigned(ob), kOrderItems, 0, q>>>(
          tc0, items, n_t, c->rng.as<CellRange>(), c->pair_off.as<int64_t>(), ofirst,
          c->order.as<PairDesc>(), c->owner.as<int32_t>());
      return hip_check(hipGetLastError(), "order scatter launch");
    };
    if (n_live > 0 && (st = order_chunk(live[0], s))) return st;
    for (int li = 0; li < n_live; ++li) {
      const int ch = live[li];
      const int64_t p0 = pat[ch], nc = pat[ch + 1] - pat[ch];
      const int64_t* cls_start = ofirst;  // key-major: class k starts at 64 k blocks
      const int64_t ntiles = ceil_div(tc_at[ch + 1] - tc_at[ch], kOrderItems);
      {
        // (II) clip the chunk's pairs, one launch per cut class (fewer vertex
        // slots per lane, more resident waves); each launch reads its
        // class's stretch of the order from the prefix sum of the key counts
        ProfScope ps("clip", s);
        if ((st = hip_check(hipEventRecord(c->ev_fork, s), "event")) ||
            (st = hip_check(hipStreamWaitEvent(c->side, c->ev_fork, 0), "stream wait")))
          return st;
        if (!masses_done) {
          // the solid masses need only the tet volumes: on the second stream
          // ahead of the first clip's classes 12 and 16, in the wave slots
          // the LDS-bound clip leaves free (joined with the clip below)
          if ((st = solid_masses(c, c->side))) return st;
          masses_done = true;
        }
        for (int k = 2; k >= 0; --k) {
          hipStream_t ks = k == 0 ? s : c->side;
          const int resident =
              k == 0 ? resident_blocks(k_clip<T, 10>)
                     : (k == 1 ? resident_blocks(k_clip<T, 12>) : resident_blocks(k_clip<T, kMaxV>));
          const int64_t nb = std::min<int64_t>(ceil_div(nc, kWave), resident);
#define IBVT_CLIP_ARGS                                                                          \
  cls_start + 64 * k * ntiles, cls_start + 64 * (k + 1) * ntiles, c->order.as<PairDesc>(),    \
      c->tetrec.as<double>(), c->lat.as<double>(), c->ld, 1e-14, c->pool.as<T>(), c->pool_cap,  \
      c->pinfo.as<uint64_t>(), counters + kCntChunkPool + ch, flags, counters
          if (k == 0) k_clip<T, 10><<<dim3(unsigned(nb)), kWave, 0, ks>>>(IBVT_CLIP_ARGS);
          else if (k == 1) k_clip<T, 12><<<dim3(unsigned(nb)), kWave, 0, ks>>>(IBVT_CLIP_ARGS);
          else k_clip<T, kMaxV><<<dim3(unsigned(nb)), kWave, 0, ks>>>(IBVT_CLIP_ARGS);
#undef IBVT_CLIP_ARGS
        }
        if ((st = hip_check(hipGetLastError(), "clip launch"))) return st;
        if ((st = hip_check(hipEventRecord(c->ev_join, c->side), "event")) ||
            (st = hip_check(hipStreamWaitEvent(s, c->ev_join, 0), "stream wait")))
          return st;
      }
      const bool next = li + 1 < n_live;
      if (next) {
        if ((st = hip_check(hipEventRecord(c->ev_fork, s), "event")) ||
            (st = hip_check(hipStreamWaitEvent(c->side, c->ev_fork, 0), "stream wait")) ||
            (st = order_chunk(live[li + 1], c->side)) ||
            (st = hip_check(hipEventRecord(c->ev_sorted, c->side), "event")))
          return st;
      }
      {
        // (III) integrate the chunk's sub-tetrahedra, summed per pair (pairs
        // whose records did not fit the store read as empty)
        ProfScope ps("integrate", s);
        k_integrate<T><<<dim3(unsigned(ceil_div(nc, kWave))), kWave, 0, s>>>(
            chunk_max, p0, p0 + nc, n_t, c->pinfo.as<uint64_t>(), c->pool.as<T>(),
            c->owner.as<int32_t>(), c->pair_off.as<int64_t>(), c->rng.as<CellRange>(),
            c->tetrec.as<double>(), c->lat.as<double>(), c->ld, c->keep.as<uint8_t>(),
            c->pval.as<T>(), c->pmom.as<T>(), c->dual ? 1 : 0);
      }
      if ((st = hip_check(hipGetLastError(), "integrate launch"))) return st;
      {
        // (IV) the rows of B^d that take pairs of this chunk: the rows of
        // the components its items belong to (on this stream: beside the
        // next chunk's clip they slow it by more than they take)
        ProfScope ps("rows_gather", s);
        const int64_t d_lo = tc_at[ch] / n_t, d_hi = (tc_at[ch + 1] - 1) / n_t;
        const int64_t w_begin = d_lo * n_v, n_rows = (d_hi - d_lo + 1) * n_v;
        k_rows<T><<<blocks_for(ceil_div(n_rows, kRowsPerWave) * kWave, 256), 256, 0, s>>>(
            n_v, n_t, ch, tc_at[ch], tc_at[ch + 1], p0, chunk_max, w_begin, n_rows,
            c->vt_ptr.as<int64_t>(), c->vt_tet.as<int32_t>(), c->tets.as<int32_t>(),
            c->rng.as<CellRange>(), c->pair_off.as<int64_t>(), c->keep.as<uint8_t>(),
            c->pval.as<T>(), c->ld, c->rowbox.as<RowBox>(), c->rowtmpoff.as<int64_t>(),
            c->rowtmpcol.as<int32_t>(), c->rowtmpval.as<T>(), c->rownnz.as<int64_t>(),
            c->rowspilloff.as<int64_t>(), spill_acc, spill_flg);
      }
      if ((st = hip_check(hipGetLastError(), "rows launch"))) return st;
      if (next && (st = hip_check(hipStreamWaitEvent(s, c->ev_sorted, 0), "stream wait")))
        return st;
    }

    // read-back 2: records each chunk asked for, flags
    int64_t rb2[kMaxChunks];
    {
      const int64_t* src[kMaxChunks];
      for (int k = 0; k < nchunk; ++k)
        src[k] = reinterpret_cast<const int64_t*>(counters + kCntChunkPool + k);
      if ((st = read_counts(c, src, nchunk, rb2, s))) return st;
    }
    if ((st = flags_status(c->host_flags))) return st;
    c->pool_needed = 0;
    for (int k = 0; k < nchunk; ++k) c->pool_needed = std::max(c->pool_needed, rb2[k]);
    if (c->pool_needed <= c->pool_cap) break;
    if (attempt == 1) return set_error(IBVT_E_CAPACITY, "piece store could not be sized");
  }
  // (IV) global assembly: rows of B^d (gathered per chunk above)
  for (int d = 0; d < 3; ++d) {
    c->B[d].nrows = n_v;
    if ((st = scan_i64(c, c->rownnz.as<int64_t>() + d * n_v, c->B[d].rowptr.as<int64_t>(), n_v, s)))
      return st;
  }
  // read-back 3: nonzeros of the three components, flags
  int64_t nnzs[3] = {0, 0, 0};
  {
    const int64_t* src[3] = {c->B[0].rowptr.as<int64_t>() + n_v, c->B[1].rowptr.as<int64_t>() + n_v,
                             c->B[2].rowptr.as<int64_t>() + n_v};
    if ((st = read_counts(c, src, 3, nnzs, s))) return st;
  }
  if ((st = flags_status(c->host_flags))) return st;
  for (int d = 0; d < 3; ++d) {
    const int64_t nnz = nnzs[d];
    c->B[d].nnz = nnz;
    if (nnz >= (int64_t(1) << 31) - 1)
      return set_error(IBVT_E_CAPACITY, "more than 2^31 nonzeros in one component of B");
    if ((st = ensure(c, c->B[d].col, size_t(nnz + 1) * sizeof(int32_t)))) return st;
    if ((st = ensure(c, c->B[d].val, size_t(nnz + 1) * sizeof(T)))) return st;
  }
  {
    ProfScope ps("rows_compact", s);
    k_rows_compact<T><<<blocks_for(3 * n_v * kCompactLanes, 256), 256, 0, s>>>(
        n_v, c->rowtmpoff.as<int64_t>(), c->rowtmpcol.as<int32_t>(), c->rowtmpval.as<T>(),
        c->B[0].rowptr.as<int64_t>(), c->B[1].rowptr.as<int64_t>(), c->B[2].rowptr.as<int64_t>(),
        c->B[0].col.as<int32_t>(), c->B[1].col.as<int32_t>(), c->B[2].col.as<int32_t>(),
        c->B[0].val.as<T>(), c->B[1].val.as<T>(), c->B[2].val.as<T>());
  }
  if ((st = hip_check(hipGetLastError(), "rows compact launch"))) return st;
  for (int d = 0; d < 3; ++d) {
    ProfScope ps("transpose", s);
    if ((st = transpose_one<T>(c, d, s))) return st;
  }
  // masses, unless they ran beside the first clip (no pairs at all)
  if (!masses_done && (st = solid_masses(c, s))) return st;
  // read-back 4: the counters of the assembly, flags
  int64_t cnt[kCntSlots];
  {
    const int64_t* src[kCntSlots];
    for (int k = 0; k < kCntSlots; ++k) src[k] = reinterpret_cast<const int64_t*>(counters + k);
    if ((st = read_counts(c, src, kCntSlots, cnt, s))) return st;
  }
  c->stats.pairs = n_pairs;
  c->stats.pieces = cnt[kCntPieces];
  c->stats.dropped = cnt[kCntDropped];
  c->stats.zero_tets = cnt[kCntZeroTets];
  c->stats.subtets = cnt[kCntSubtets];
  c->stats.dist_evals = cnt[kCntDist];
  c->stats.cut_points = cnt[kCntCutPts];
  c->stats.plane_cuts = cnt[kCntPlanes];
  c->stats.assemblies += 1;
  if ((st = flags_status(c->host_flags))) return st;
  c->mom_valid = c->store_pieces;
  if (!c->store_pieces) {
    // memory-saving mode: no piece store kept; the reverse mode clips again
    // (the stream is idle after the read-back)
    release(c, c->pool);
    release(c, c->pmom);
    c->pool_cap = 0;
  }
  return IBVT_OK;
}

}  // namespace

int solid_masses(ibvt_coupling* c, hipStream_t s) {
  const int64_t n_v = c->n_vert;
  ProfScope ps("masses", s);
  if (c->precision == IBVT_FP32_MIXED)
    k_lumped<float><<<blocks_for(n_v, 256), 256, 0, s>>>(
        n_v, c->vt_ptr.as<int64_t>(), c->vt_tet.as<int32_t>(), c->tetvol.as<double>(),
        c->mlump.as<double>(), c->minv.as<float>());
  else
    k_lumped<double><<<blocks_for(n_v, 256), 256, 0, s>>>(
        n_v, c->vt_ptr.as<int64_t>(), c->vt_tet.as<int32_t>(), c->tetvol.as<double>(),
        c->mlump.as<double>(), c->minv.as<double>());
  if (c->has_M) {
    k_mass_values<<<blocks_for(n_v * kMassLanes, 256), 256, 0, s>>>(
        n_v, c->vt_ptr.as<int64_t>(), c->vt_tet.as<int32_t>(), c->tets.as<int32_t>(),
        c->tetvol.as<double>(), c->M.rowptr.as<int64_t>(), c->M.col.as<int32_t>(),
        c->M.val.as<double>(), c->precision == IBVT_FP32_MIXED ? c->Mval32.as<float>() : nullptr,
        c->Mdiag_inv.as<double>());
  }
  return hip_check(hipGetLastError(), "mass launch");
}

int build_topology(ibvt_coupling* c, hipStream_t s) {
  const int64_t n_t = c->n_tet, n_v = c->n_vert;
  int st;
  if ((st = ensure(c, c->flags_dev, 64))) return st;
  if ((st = ensure(c, c->counters, kCntSlots * sizeof(unsigned long long)))) return st;
  if ((st = ensure(c, c->vt_ptr, size_t(n_v + 1) * sizeof(int64_t)))) return st;
  const int K = c->dim + 1;  // vertices per element
  if ((st = ensure(c, c->vt_tet, size_t(K * n_t + 1) * sizeof(int32_t)))) return st;
  if ((st = ensure(c, c->rownnz, size_t(3 * n_v + 1) * sizeof(int64_t)))) return st;
  unsigned* flags = c->flags_dev.as<unsigned>();
  if ((st = hip_check(hipMemsetAsync(flags, 0, sizeof(unsigned), s), "memset"))) return st;
  auto* deg = c->rownnz.as<unsigned long long>();  // scratch: degrees, then cursors
  if ((st = hip_check(hipMemsetAsync(deg, 0, size_t(n_v + 1) * sizeof(int64_t), s), "memset")))
    return st;
  if (K == 4) k_vt_count<4><<<blocks_for(n_t, 256), 256, 0, s>>>(n_t, n_v, c->tets.as<int32_t>(), deg, flags);
  else k_vt_count<3><<<blocks_for(n_t, 256), 256, 0, s>>>(n_t, n_v, c->tets.as<int32_t>(), deg, flags);
  if ((st = check_flags(c, s))) return st;
  if ((st = scan_i64(c, c->rownnz.as<int64_t>(), c->vt_ptr.as<int64_t>(), n_v, s))) return st;
  if ((st = hip_check(hipMemsetAsync(deg, 0, size_t(n_v + 1) * sizeof(int64_t), s), "memset")))
    return st;
  if (K == 4)
    k_vt_fill<4><<<blocks_for(n_t, 256), 256, 0, s>>>(n_t, c->tets.as<int32_t>(),
                                                      c->vt_ptr.as<int64_t>(), deg,
                                                      c->vt_tet.as<int32_t>());
  else
    k_vt_fill<3><<<blocks_for(n_t, 256), 256, 0, s>>>(n_t, c->tets.as<int32_t>(),
                                                      c->vt_ptr.as<int64_t>(), deg,
                                                      c->vt_tet.as<int32_t>());
  k_sort_segments_i32<<<blocks_for(n_v, 256), 256, 0, s>>>(n_v, c->vt_ptr.as<int64_t>(),
                                                           c->vt_tet.as<int32_t>());
  if ((st = hip_check(hipGetLastError(), "topology launch"))) return st;
  if (c->has_M) {
    auto pattern = [&](bool fill) {
      const int64_t* vp = c->vt_ptr.as<int64_t>();
      const int32_t* vt = c->vt_tet.as<int32_t>();
      const int32_t* el = c->tets.as<int32_t>();
      int64_t* cnt = fill ? nullptr : c->rownnz.as<int64_t>();
      const int64_t* rp = fill ? c->M.rowptr.as<int64_t>() : nullptr;
      int32_t* col = fill ? c->M.col.as<int32_t>() : nullptr;
      const unsigned nb = blocks_for(n_v, 256);
      if (K == 4 && !fill) k_mass_pattern<4, false><<<nb, 256, 0, s>>>(n_v, vp, vt, el, cnt, rp, col);
      if (K == 4 && fill) k_mass_pattern<4, true><<<nb, 256, 0, s>>>(n_v, vp, vt, el, cnt, rp, col);
      if (K == 3 && !fill) k_mass_pattern<3, false><<<nb, 256, 0, s>>>(n_v, vp, vt, el, cnt, rp, col);
      if (K == 3 && fill) k_mass_pattern<3, true><<<nb, 256, 0, s>>>(n_v, vp, vt, el, cnt, rp, col);
    };
    pattern(false);
    if ((st = ensure(c, c->M.rowptr, size_t(n_v + 1) * sizeof(int64_t)))) return st;
    if ((st = scan_i64(c, c->rownnz.as<int64_t>(), c->M.rowptr.as<int64_t>(), n_v, s))) return st;
    int64_t nnz = 0;
    if ((st = read_back(c, &nnz, c->M.rowptr.as<int64_t>() + n_v, sizeof(int64_t), s))) return st;
    c->M.nrows = n_v;
    c->M.nnz = nnz;
    if ((st = ensure(c, c->M.col, size_t(nnz + 1) * sizeof(int32_t)))) return st;
    if ((st = ensure(c, c->M.val, size_t(nnz + 1) * sizeof(double)))) return st;
    if ((st = ensure(c, c->Mval32, size_t(nnz + 1) * sizeof(float)))) return st;
    if ((st = ensure(c, c->Mdiag_inv, size_t(n_v + 1) * sizeof(double)))) return st;
    pattern(true);
    if ((st = hip_check(hipGetLastError(), "mass pattern launch"))) return st;
  }
  return IBVT_OK;
}

namespace {
int assemble_grid(ibvt_coupling* c, hipStream_t s);
}  // namespace

// Every assembly starts by marking the handle unusable and marks it usable
// only when every step has succeeded, so that a failed reassembly (a solid
// leaving the lattice, a capacity error) cannot leave transfers running on a
// mix of old matrices and new per-pair data.
int assemble_all(ibvt_coupling* c, hipStream_t s) {
  c->ready = false;
  c->mom_valid = false;
  c->tcorder_valid = false;
  const int st = c->dim == 2 ? assemble_all_2d(c, s)
                 : c->unstructured ? assemble_all_unstructured(c, s)
                                   : assemble_grid(c, s);
  if (st) {
    c->mom_valid = false;
    return st;
  }
  c->ready = true;
  return IBVT_OK;
}

namespace {
int assemble_grid(ibvt_coupling* c, hipStream_t s) {
  const int64_t n_t = c->n_tet, n_v = c->n_vert;
  int st;
  // the clip's pair descriptors pack the tet and cell indices
  if (n_t >= kMaxDescTets) return set_error(IBVT_E_UNSUPPORTED, "2^30 or more tets");
  for (int k = 0; k < 9; ++k)
    if (c->ld.n[k] > (1 << kCellBits))
      return set_error(IBVT_E_UNSUPPORTED, "more than 2^21 lattice cells along one axis");
  if ((st = ensure(c, c->tetvol, size_t(n_t + 1) * sizeof(double)))) return st;
  if ((st = ensure(c, c->tetrec, size_t(n_t + 1) * kTetRec * sizeof(double)))) return st;
  if ((st = ensure(c, c->tetgrad, size_t(n_t + 1) * 12 * sizeof(double)))) return st;
  if ((st = ensure(c, c->rng, size_t(3 * n_t + 1) * sizeof(CellRange)))) return st;
  if ((st = ensure(c, c->cnt, size_t(3 * n_t + 1) * sizeof(int64_t)))) return st;
  if ((st = ensure(c, c->pair_off, size_t(3 * n_t + 1) * sizeof(int64_t)))) return st;
  if ((st = ensure(c, c->mlump, size_t(n_v + 1) * sizeof(double)))) return st;
  for (int d = 0; d < 3; ++d)
    if ((st = ensure(c, c->B[d].rowptr, size_t(n_v + 1) * sizeof(int64_t)))) return st;
  if (c->precision == IBVT_FP32_MIXED) {
    if ((st = ensure(c, c->minv, size_t(n_v + 1) * sizeof(float)))) return st;
    return assemble_typed<float>(c, s);
  }
  if ((st = ensure(c, c->minv, size_t(n_v + 1) * sizeof(double)))) return st;
  return assemble_typed<double>(c, s);
}
}  // namespace

}  // namespace ibvt
