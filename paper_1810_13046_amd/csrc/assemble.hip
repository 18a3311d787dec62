// Assembly of the mortar matrices B^d (Section 2.3, steps (I)-(IV)).
//
//  k_tet_prep      per tet: bounding box -> cell index range on each
//                  component's lattice (replaces the tree search: on a
//                  rectilinear grid the overlap candidates of a tet are an
//                  index box), volume, validity checks.
//  scan            candidate (tet, component, cell) pair offsets.
//  k_clip<T>       one lane per pair: clip the tet by the cell's six planes
//                  in double and integrate λ_i N_j on the piece (32 values).
//  k_rows<T,FILL>  one wavefront per (solid vertex, component): gathers the
//                  pieces of the vertex's incident tets into a dense node box
//                  held in registers, in a fixed order (deterministic, no
//                  atomics on values), and writes the CSR row (count pass,
//                  then fill pass).
//  transpose       B^dT over the touched fluid nodes (integer atomics for
//                  positions, then each row sorted by vertex index, so the
//                  result does not depend on timing).
//  masses          lumped m_i = Σ_{T∋i} |T|/4 and the consistent P1 mass
//                  matrix |T|(1+δ_il)/20 (Section 2.1), per vertex in
//                  incident-tet order.
#include "geometry.hpp"
#include "internal.hpp"

#include <climits>

namespace ibvt {

namespace {

constexpr int kRowSlots = 4;  // box nodes per lane per pass in k_rows

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

__global__ void k_vt_count(int64_t n_t, int64_t n_v, const int32_t* __restrict__ tets,
                           unsigned long long* __restrict__ deg, unsigned* flags) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= n_t) return;
  int v[4];
  bool bad = false;
  for (int k = 0; k < 4; ++k) {
    v[k] = tets[4 * t + k];
    bad |= (v[k] < 0) || (int64_t(v[k]) >= n_v);
  }
  for (int a = 0; a < 4; ++a)
    for (int b = a + 1; b < 4; ++b) bad |= (v[a] == v[b]);
  if (bad) {
    atomicOr(flags, kFlagValence);
    return;
  }
  for (int k = 0; k < 4; ++k) atomicAdd(&deg[v[k]], 1ull);
}

__global__ void k_vt_fill(int64_t n_t, const int32_t* __restrict__ tets,
                          const int64_t* __restrict__ vt_ptr, unsigned long long* __restrict__ cur,
                          int32_t* __restrict__ vt_tet) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= n_t) return;
  for (int k = 0; k < 4; ++k) {
    const int v = tets[4 * t + k];
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

// Consistent-mass pattern: distinct vertices of the incident tets.
template <bool FILL>
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
      for (int q = 0; q < 4; ++q) {
        const int v = tets[4 * t + q];
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
                           int64_t* __restrict__ cnt, unsigned* flags,
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
    }
  }
  const uint64_t zm = ballot64(zero);
  if (lane_id() == 0 && zm) atomicAdd(&counters[kCntZeroTets], (unsigned long long)popc64(zm));
}

__global__ void k_owner(int64_t n_tc, const int64_t* __restrict__ off, int32_t* __restrict__ owner) {
  const int64_t tc = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (tc >= n_tc) return;
  for (int64_t p = off[tc]; p < off[tc + 1]; ++p) owner[p] = int32_t(tc);
}

// ---------------------------------------------------------------------------
// clip + integrate, one lane per (tet, component, cell) pair
// ---------------------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(kWave) void k_clip(
    int64_t n_pairs, int64_t n_t, const int32_t* __restrict__ owner,
    const int64_t* __restrict__ pair_off, const CellRange* __restrict__ rng,
    const double* __restrict__ X, const int32_t* __restrict__ tets, const double* __restrict__ lat,
    LatDesc ld, double drop_rel, T* __restrict__ pval, uint8_t* __restrict__ keep,
    unsigned* flags, unsigned long long* counters) {
  __shared__ double sx[kMaxV * kWave], sy[kMaxV * kWave], sz[kMaxV * kWave];
  __shared__ uint32_t snb[kMaxV * kWave];
  const int lane = threadIdx.x;
  const PolyView P{sx + lane, sy + lane, sz + lane, snb + lane, kWave};
  unsigned long long nk = 0, nd = 0, ns = 0;
  bool fail = false;
  for (int64_t p = int64_t(blockIdx.x) * kWave + lane; p < n_pairs;
       p += int64_t(gridDim.x) * kWave) {
    const int64_t tc = owner[p];
    const int d = int(tc / n_t);
    const int64_t t = tc - int64_t(d) * n_t;
    const CellRange r = rng[tc];
    const int64_t q = p - pair_off[tc];
    const int ci[3] = {r.lo[0] + int(q % r.n[0]), r.lo[1] + int((q / r.n[0]) % r.n[1]),
                       r.lo[2] + int(q / (int64_t(r.n[0]) * r.n[1]))};
    TetGeom G;
    for (int k = 0; k < 4; ++k) {
      const int64_t v = tets[4 * t + k];
      G.V[k][0] = X[3 * v + 0];
      G.V[k][1] = X[3 * v + 1];
      G.V[k][2] = X[3 * v + 2];
    }
    tet_geom(G);
    double lo[3], hi[3];
    for (int e = 0; e < 3; ++e) {
      const double* L = lat + ld.off[3 * d + e];
      lo[e] = L[ci[e]];
      hi[e] = L[ci[e] + 1];
    }
    double vol6;
    T acc[32];
    int nsub = 0;
    const bool ok = clip_integrate<T>(P, G, lo, hi, vol6, acc, nsub);
    ns += unsigned(nsub);
    if (!ok) {
      fail = true;
      keep[p] = 0;
      continue;
    }
    const double cv = (hi[0] - lo[0]) * (hi[1] - lo[1]) * (hi[2] - lo[2]);
    const double vol = vol6 * cv / 6.0;
    const bool kp = vol > drop_rel * (fabs(G.det) / 6.0);
    keep[p] = kp ? 1 : 0;
    if (kp) {
      ++nk;
      const T sc = T(-cv / 6.0);
      T* out = pval + p * 32;
#pragma unroll
      for (int k = 0; k < 32; ++k) out[k] = acc[k] * sc;
    } else if (vol > 0.0) {
      ++nd;
    }
  }
  nk = wave_sum(nk);
  nd = wave_sum(nd);
  ns = wave_sum(ns);
  const uint64_t fm = ballot64(fail);
  if (lane == 0) {
    if (nk) atomicAdd(&counters[kCntPieces], nk);
    if (nd) atomicAdd(&counters[kCntDropped], nd);
    if (ns) atomicAdd(&counters[kCntSubtets], ns);
    if (fm) atomicOr(flags, kFlagCapacity);
  }
}

// ---------------------------------------------------------------------------
// row gather: one wavefront per (vertex, component)
// ---------------------------------------------------------------------------

template <typename T>
struct RowOut {
  const int64_t* rowptr[3];
  int32_t* col[3];
  T* val[3];
};

template <typename T, bool FILL>
__global__ __launch_bounds__(256) void k_rows(
    int64_t n_v, int64_t n_t, const int64_t* __restrict__ vt_ptr,
    const int32_t* __restrict__ vt_tet, const int32_t* __restrict__ tets,
    const CellRange* __restrict__ rng, const int64_t* __restrict__ pair_off,
    const uint8_t* __restrict__ keep, const T* __restrict__ pval, LatDesc ld,
    int64_t* __restrict__ rownnz, RowOut<T> out) {
  const int64_t wid = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / kWave;
  const int lane = lane_id();
  if (wid >= 3 * n_v) return;
  const int d = int(wid / n_v);
  const int64_t i = wid - int64_t(d) * n_v;
  const int64_t beg = vt_ptr[i], end = vt_ptr[i + 1];
  int bmin[3] = {INT_MAX, INT_MAX, INT_MAX}, bmax[3] = {INT_MIN, INT_MIN, INT_MIN};
  for (int64_t k = beg + lane; k < end; k += kWave) {
    const CellRange r = rng[int64_t(d) * n_t + vt_tet[k]];
    if (int64_t(r.n[0]) * r.n[1] * r.n[2] == 0) continue;
    for (int e = 0; e < 3; ++e) {
      bmin[e] = min(bmin[e], r.lo[e]);
      bmax[e] = max(bmax[e], r.lo[e] + r.n[e]);
    }
  }
  for (int e = 0; e < 3; ++e) {
    bmin[e] = wave_min(bmin[e]);
    bmax[e] = wave_max(bmax[e]);
  }
  if (bmin[0] > bmax[0]) {
    if (!FILL && lane == 0) rownnz[wid] = 0;
    return;
  }
  const int sx = bmax[0] - bmin[0] + 1, sy = bmax[1] - bmin[1] + 1, sz = bmax[2] - bmin[2] + 1;
  const int64_t total = int64_t(sx) * sy * sz;
  const int64_t NX = ld.n[3 * d + 0], NY = ld.n[3 * d + 1];
  int64_t outpos = FILL ? out.rowptr[d][i] : 0;
  int64_t count = 0;
  for (int64_t c0 = 0; c0 < total; c0 += int64_t(kWave) * kRowSlots) {
    T acc[kRowSlots];
    int nx[kRowSlots], ny[kRowSlots], nz[kRowSlots];
    uint32_t valid = 0, touched = 0;
#pragma unroll
    for (int rr = 0; rr < kRowSlots; ++rr) {
      acc[rr] = T(0);
      const int64_t lin = c0 + int64_t(rr) * kWave + lane;
      if (lin < total) valid |= 1u << rr;
      nx[rr] = bmin[0] + int(lin % sx);
      ny[rr] = bmin[1] + int((lin / sx) % sy);
      nz[rr] = bmin[2] + int(lin / (int64_t(sx) * sy));
    }
    const int active = int(min<int64_t>(kRowSlots, ceil_div(total - c0, kWave)));
    for (int64_t k = beg; k < end; ++k) {
      const int64_t t = vt_tet[k];
      const int64_t tc = int64_t(d) * n_t + t;
      const CellRange r = rng[tc];
      const int ncell = r.n[0] * r.n[1] * r.n[2];
      if (!ncell) continue;
      int li = 0;
      for (int q = 1; q < 4; ++q)
        if (tets[4 * t + q] == int32_t(i)) li = q;
      const int64_t base = pair_off[tc];
      for (int q = 0; q < ncell; ++q) {
        if (!keep[base + q]) continue;
        const int cx = r.lo[0] + q % r.n[0];
        const int cy = r.lo[1] + (q / r.n[0]) % r.n[1];
        const int cz = r.lo[2] + q / (r.n[0] * r.n[1]);
        const T* pv = pval + (base + q) * 32 + li * 8;
#pragma unroll
        for (int rr = 0; rr < kRowSlots; ++rr) {
          if (rr >= active) break;
          const unsigned dx = unsigned(nx[rr] - cx), dy = unsigned(ny[rr] - cy),
                         dz = unsigned(nz[rr] - cz);
          if (((valid >> rr) & 1u) && dx <= 1u && dy <= 1u && dz <= 1u) {
            touched |= 1u << rr;
            if (FILL) acc[rr] += pv[dx + 2 * dy + 4 * dz];
          }
        }
      }
    }
#pragma unroll
    for (int rr = 0; rr < kRowSlots; ++rr) {
      const bool tch = (touched >> rr) & 1u;
      const uint64_t m = ballot64(tch);
      if (FILL) {
        if (tch) {
          const int64_t pos = outpos + rank_below(m);
          out.col[d][pos] = int32_t(nx[rr] + NX * (ny[rr] + NY * int64_t(nz[rr])));
          out.val[d][pos] = acc[rr];
        }
        outpos += popc64(m);
      } else {
        count += popc64(m);
      }
    }
  }
  if (!FILL && lane == 0) rownnz[wid] = count;
}

// ---------------------------------------------------------------------------
// transpose
// ---------------------------------------------------------------------------

__global__ void k_mark(int64_t nnz, const int32_t* __restrict__ col, int32_t* __restrict__ mark) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k < nnz) mark[col[k]] = 1;
}

__global__ void k_compact(int64_t n, const int32_t* __restrict__ mark,
                          const int64_t* __restrict__ cidx, int32_t* __restrict__ rowmap) {
  const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j < n && mark[j]) rowmap[cidx[j]] = int32_t(j);
}

__global__ void k_tcount(int64_t nnz, const int32_t* __restrict__ col,
                         const int64_t* __restrict__ cidx, unsigned long long* __restrict__ cnt) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k < nnz) atomicAdd(&cnt[cidx[col[k]]], 1ull);
}

template <typename T>
__global__ void k_tfill(int64_t n_rows, const int64_t* __restrict__ rowptr,
                        const int32_t* __restrict__ col, const T* __restrict__ val,
                        const int64_t* __restrict__ cidx, const int64_t* __restrict__ trowptr,
                        unsigned long long* __restrict__ cur, int32_t* __restrict__ tcol,
                        T* __restrict__ tval) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n_rows) return;
  for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
    const int64_t r = cidx[col[k]];
    const int64_t pos = trowptr[r] + int64_t(atomicAdd(&cur[r], 1ull));
    tcol[pos] = int32_t(i);
    tval[pos] = val[k];
  }
}

template <typename T>
__global__ void k_tsort(int64_t n_rows, const int64_t* __restrict__ ptr, int32_t* __restrict__ key,
                        T* __restrict__ val) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n_rows) return;
  const int64_t b = ptr[i], e = ptr[i + 1];
  for (int64_t k = b + 1; k < e; ++k) {
    const int32_t x = key[k];
    const T v = val[k];
    int64_t j = k - 1;
    while (j >= b && key[j] > x) {
      key[j + 1] = key[j];
      val[j + 1] = val[j];
      --j;
    }
    key[j + 1] = x;
    val[j + 1] = v;
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

__global__ void k_mass_values(int64_t n_v, const int64_t* __restrict__ vt_ptr,
                              const int32_t* __restrict__ vt_tet, const int32_t* __restrict__ tets,
                              const double* __restrict__ tetvol, const int64_t* __restrict__ rowptr,
                              const int32_t* __restrict__ col, double* __restrict__ val,
                              float* __restrict__ val32, double* __restrict__ dinv) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n_v) return;
  const int64_t rb = rowptr[i], re = rowptr[i + 1];
  for (int64_t k = rb; k < re; ++k) val[k] = 0.0;
  for (int64_t k = vt_ptr[i]; k < vt_ptr[i + 1]; ++k) {
    const int64_t t = vt_tet[k];
    const double w = tetvol[t] / 20.0;
    for (int q = 0; q < 4; ++q) {
      const int l = tets[4 * t + q];
      int64_t lo = rb, hi = re;  // binary search for column l
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (col[mid] < l) lo = mid + 1; else hi = mid;
      }
      val[lo] += (int64_t(l) == i) ? 2.0 * w : w;
    }
  }
  double diag = 0.0;
  for (int64_t k = rb; k < re; ++k) {
    if (int64_t(col[k]) == i) diag = val[k];
    if (val32) val32[k] = float(val[k]);
  }
  dinv[i] = (diag > 0.0) ? 1.0 / diag : 0.0;
}

inline unsigned blocks_for(int64_t n, int threads) {
  return unsigned(ceil_div(n > 0 ? n : 1, threads));
}

int read_back(ibvt_coupling* c, void* host, const void* dev, size_t bytes, hipStream_t s) {
  int st = hip_check(hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, s), "read back");
  if (st) return st;
  return hip_check(hipStreamSynchronize(s), "stream sync");
}

int check_flags(ibvt_coupling* c, hipStream_t s) {
  unsigned f = 0;
  int st = read_back(c, &f, c->flags_dev.p, sizeof(unsigned), s);
  if (st) return st;
  if (f & kFlagNonFinite) return set_error(IBVT_E_INVALID, "non-finite vertex coordinate");
  if (f & kFlagValence) return set_error(IBVT_E_INVALID, "tet vertex index out of range or repeated");
  if (f & kFlagOutOfGrid)
    return set_error(IBVT_E_OUT_OF_GRID, "a tet's bounding box leaves a velocity lattice's node hull");
  if (f & kFlagCapacity)
    return set_error(IBVT_E_CAPACITY, "clipped piece exceeded the 16-vertex capacity");
  return IBVT_OK;
}

template <typename T>
int transpose_one(ibvt_coupling* c, int d, hipStream_t s) {
  const int64_t nf = c->n_fluid[d];
  const ibvt::Csr& B = c->B[d];
  ibvt::Csr& Bt = c->Bt[d];
  int st;
  if ((st = hip_check(hipMemsetAsync(c->mark.p, 0, size_t(nf) * sizeof(int32_t), s), "memset")))
    return st;
  if (B.nnz)
    k_mark<<<blocks_for(B.nnz, 256), 256, 0, s>>>(B.nnz, B.col.as<int32_t>(), c->mark.as<int32_t>());
  if ((st = scan_i32_to_i64(c, c->mark.as<int32_t>(), c->cidx.as<int64_t>(), nf, s))) return st;
  int64_t touched = 0;
  if ((st = read_back(c, &touched, c->cidx.as<int64_t>() + nf, sizeof(int64_t), s))) return st;
  Bt.nrows = touched;
  Bt.nnz = B.nnz;
  if ((st = ensure(c, Bt.rowptr, size_t(touched + 1) * sizeof(int64_t)))) return st;
  if ((st = ensure(c, Bt.rowmap, size_t(touched + 1) * sizeof(int32_t)))) return st;
  if ((st = ensure(c, Bt.col, size_t(B.nnz + 1) * sizeof(int32_t)))) return st;
  if ((st = ensure(c, Bt.val, size_t(B.nnz + 1) * sizeof(T)))) return st;
  if ((st = ensure(c, c->tcount, size_t(touched + 1) * sizeof(int64_t)))) return st;
  k_compact<<<blocks_for(nf, 256), 256, 0, s>>>(nf, c->mark.as<int32_t>(), c->cidx.as<int64_t>(),
                                                Bt.rowmap.as<int32_t>());
  auto* cnt = c->tcount.as<unsigned long long>();
  if ((st = hip_check(hipMemsetAsync(cnt, 0, size_t(touched + 1) * sizeof(int64_t), s), "memset")))
    return st;
  if (B.nnz)
    k_tcount<<<blocks_for(B.nnz, 256), 256, 0, s>>>(B.nnz, B.col.as<int32_t>(),
                                                    c->cidx.as<int64_t>(), cnt);
  if ((st = scan_i64(c, c->tcount.as<int64_t>(), Bt.rowptr.as<int64_t>(), touched, s))) return st;
  if ((st = hip_check(hipMemsetAsync(cnt, 0, size_t(touched + 1) * sizeof(int64_t), s), "memset")))
    return st;
  k_tfill<T><<<blocks_for(c->n_vert, 256), 256, 0, s>>>(
      c->n_vert, B.rowptr.as<int64_t>(), B.col.as<int32_t>(), B.val.as<T>(), c->cidx.as<int64_t>(),
      Bt.rowptr.as<int64_t>(), cnt, Bt.col.as<int32_t>(), Bt.val.as<T>());
  k_tsort<T><<<blocks_for(touched, 256), 256, 0, s>>>(touched, Bt.rowptr.as<int64_t>(),
                                                      Bt.col.as<int32_t>(), Bt.val.as<T>());
  return hip_check(hipGetLastError(), "transpose launch");
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
      c->tetvol.as<double>(), c->rng.as<CellRange>(), c->cnt.as<int64_t>(), flags, counters);
  }
  if ((st = hip_check(hipGetLastError(), "prep launch"))) return st;
  if ((st = scan_i64(c, c->cnt.as<int64_t>(), c->pair_off.as<int64_t>(), 3 * n_t, s))) return st;
  if ((st = check_flags(c, s))) return st;
  int64_t n_pairs = 0;
  if ((st = read_back(c, &n_pairs, c->pair_off.as<int64_t>() + 3 * n_t, sizeof(int64_t), s)))
    return st;
  if (n_pairs >= (int64_t(1) << 40))
    return set_error(IBVT_E_CAPACITY, "too many (tet, cell) pairs");
  c->n_pairs = n_pairs;
  if ((st = ensure(c, c->owner, size_t(n_pairs + 1) * sizeof(int32_t)))) return st;
  if ((st = ensure(c, c->keep, size_t(n_pairs + 1)))) return st;
  if ((st = ensure(c, c->pval, size_t(n_pairs + 1) * 32 * sizeof(T)))) return st;
  k_owner<<<blocks_for(3 * n_t, 256), 256, 0, s>>>(3 * n_t, c->pair_off.as<int64_t>(),
                                                   c->owner.as<int32_t>());
  // (II)+(III) clip and integrate every pair
  if (n_pairs > 0) {
    const int64_t nb = std::min<int64_t>(ceil_div(n_pairs, kWave), int64_t(1) << 22);
    ProfScope ps("clip_integrate", s);
    k_clip<T><<<dim3(unsigned(nb)), kWave, 0, s>>>(
        n_pairs, n_t, c->owner.as<int32_t>(), c->pair_off.as<int64_t>(), c->rng.as<CellRange>(),
        c->X.as<double>(), c->tets.as<int32_t>(), c->lat.as<double>(), c->ld, 1e-14,
        c->pval.as<T>(), c->keep.as<uint8_t>(), flags, counters);
  }
  if ((st = hip_check(hipGetLastError(), "clip launch"))) return st;
  // (IV) global assembly: rows of B^d
  RowOut<T> ro{};
  const unsigned row_blocks = blocks_for(3 * n_v * kWave, 256);
  {
    ProfScope ps("rows_count", s);
    k_rows<T, false><<<row_blocks, 256, 0, s>>>(
        n_v, n_t, c->vt_ptr.as<int64_t>(), c->vt_tet.as<int32_t>(), c->tets.as<int32_t>(),
        c->rng.as<CellRange>(), c->pair_off.as<int64_t>(), c->keep.as<uint8_t>(), c->pval.as<T>(),
        c->ld, c->rownnz.as<int64_t>(), ro);
  }
  if ((st = hip_check(hipGetLastError(), "rows launch"))) return st;
  for (int d = 0; d < 3; ++d) {
    c->B[d].nrows = n_v;
    if ((st = scan_i64(c, c->rownnz.as<int64_t>() + d * n_v, c->B[d].rowptr.as<int64_t>(), n_v, s)))
      return st;
  }
  if ((st = check_flags(c, s))) return st;
  for (int d = 0; d < 3; ++d) {
    int64_t nnz = 0;
    if ((st = read_back(c, &nnz, c->B[d].rowptr.as<int64_t>() + n_v, sizeof(int64_t), s)))
      return st;
    c->B[d].nnz = nnz;
    if ((st = ensure(c, c->B[d].col, size_t(nnz + 1) * sizeof(int32_t)))) return st;
    if ((st = ensure(c, c->B[d].val, size_t(nnz + 1) * sizeof(T)))) return st;
    ro.rowptr[d] = c->B[d].rowptr.as<int64_t>();
    ro.col[d] = c->B[d].col.as<int32_t>();
    ro.val[d] = c->B[d].val.as<T>();
  }
  {
    ProfScope ps("rows_fill", s);
    k_rows<T, true><<<row_blocks, 256, 0, s>>>(
        n_v, n_t, c->vt_ptr.as<int64_t>(), c->vt_tet.as<int32_t>(), c->tets.as<int32_t>(),
        c->rng.as<CellRange>(), c->pair_off.as<int64_t>(), c->keep.as<uint8_t>(), c->pval.as<T>(),
        c->ld, c->rownnz.as<int64_t>(), ro);
  }
  if ((st = hip_check(hipGetLastError(), "rows fill launch"))) return st;
  for (int d = 0; d < 3; ++d) {
    ProfScope ps("transpose", s);
    if ((st = transpose_one<T>(c, d, s))) return st;
  }
  // masses
  {
    ProfScope ps("masses", s);
  k_lumped<T><<<blocks_for(n_v, 256), 256, 0, s>>>(n_v, c->vt_ptr.as<int64_t>(),
                                                   c->vt_tet.as<int32_t>(), c->tetvol.as<double>(),
                                                   c->mlump.as<double>(), c->minv.as<T>());
  if (c->has_M) {
    k_mass_values<<<blocks_for(n_v, 256), 256, 0, s>>>(
        n_v, c->vt_ptr.as<int64_t>(), c->vt_tet.as<int32_t>(), c->tets.as<int32_t>(),
        c->tetvol.as<double>(), c->M.rowptr.as<int64_t>(), c->M.col.as<int32_t>(),
        c->M.val.as<double>(), c->precision == IBVT_FP32_MIXED ? c->Mval32.as<float>() : nullptr,
        c->Mdiag_inv.as<double>());
  }
  }
  if ((st = hip_check(hipGetLastError(), "mass launch"))) return st;
  unsigned long long cnt[kCntSlots];
  if ((st = read_back(c, cnt, counters, sizeof(cnt), s))) return st;
  c->stats.pairs = n_pairs;
  c->stats.pieces = int64_t(cnt[kCntPieces]);
  c->stats.dropped = int64_t(cnt[kCntDropped]);
  c->stats.zero_tets = int64_t(cnt[kCntZeroTets]);
  c->stats.subtets = int64_t(cnt[kCntSubtets]);
  c->stats.assemblies += 1;
  return check_flags(c, s);
}

}  // namespace

int build_topology(ibvt_coupling* c, hipStream_t s) {
  const int64_t n_t = c->n_tet, n_v = c->n_vert;
  int st;
  if ((st = ensure(c, c->flags_dev, 64))) return st;
  if ((st = ensure(c, c->counters, kCntSlots * sizeof(unsigned long long)))) return st;
  if ((st = ensure(c, c->vt_ptr, size_t(n_v + 1) * sizeof(int64_t)))) return st;
  if ((st = ensure(c, c->vt_tet, size_t(4 * n_t + 1) * sizeof(int32_t)))) return st;
  if ((st = ensure(c, c->rownnz, size_t(3 * n_v + 1) * sizeof(int64_t)))) return st;
  unsigned* flags = c->flags_dev.as<unsigned>();
  if ((st = hip_check(hipMemsetAsync(flags, 0, sizeof(unsigned), s), "memset"))) return st;
  auto* deg = c->rownnz.as<unsigned long long>();  // scratch: degrees, then cursors
  if ((st = hip_check(hipMemsetAsync(deg, 0, size_t(n_v + 1) * sizeof(int64_t), s), "memset")))
    return st;
  k_vt_count<<<blocks_for(n_t, 256), 256, 0, s>>>(n_t, n_v, c->tets.as<int32_t>(), deg, flags);
  if ((st = check_flags(c, s))) return st;
  if ((st = scan_i64(c, c->rownnz.as<int64_t>(), c->vt_ptr.as<int64_t>(), n_v, s))) return st;
  if ((st = hip_check(hipMemsetAsync(deg, 0, size_t(n_v + 1) * sizeof(int64_t), s), "memset")))
    return st;
  k_vt_fill<<<blocks_for(n_t, 256), 256, 0, s>>>(n_t, c->tets.as<int32_t>(), c->vt_ptr.as<int64_t>(),
                                                 deg, c->vt_tet.as<int32_t>());
  k_sort_segments_i32<<<blocks_for(n_v, 256), 256, 0, s>>>(n_v, c->vt_ptr.as<int64_t>(),
                                                           c->vt_tet.as<int32_t>());
  if ((st = hip_check(hipGetLastError(), "topology launch"))) return st;
  if (c->has_M) {
    k_mass_pattern<false><<<blocks_for(n_v, 256), 256, 0, s>>>(
        n_v, c->vt_ptr.as<int64_t>(), c->vt_tet.as<int32_t>(), c->tets.as<int32_t>(),
        c->rownnz.as<int64_t>(), nullptr, nullptr);
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
    k_mass_pattern<true><<<blocks_for(n_v, 256), 256, 0, s>>>(
        n_v, c->vt_ptr.as<int64_t>(), c->vt_tet.as<int32_t>(), c->tets.as<int32_t>(), nullptr,
        c->M.rowptr.as<int64_t>(), c->M.col.as<int32_t>());
    if ((st = hip_check(hipGetLastError(), "mass pattern launch"))) return st;
  }
  return IBVT_OK;
}

int assemble_all(ibvt_coupling* c, hipStream_t s) {
  const int64_t n_t = c->n_tet, n_v = c->n_vert;
  int st;
  int64_t nf_max = std::max(c->n_fluid[0], std::max(c->n_fluid[1], c->n_fluid[2]));
  if ((st = ensure(c, c->tetvol, size_t(n_t + 1) * sizeof(double)))) return st;
  if ((st = ensure(c, c->rng, size_t(3 * n_t + 1) * sizeof(CellRange)))) return st;
  if ((st = ensure(c, c->cnt, size_t(3 * n_t + 1) * sizeof(int64_t)))) return st;
  if ((st = ensure(c, c->pair_off, size_t(3 * n_t + 1) * sizeof(int64_t)))) return st;
  if ((st = ensure(c, c->mark, size_t(nf_max + 1) * sizeof(int32_t)))) return st;
  if ((st = ensure(c, c->cidx, size_t(nf_max + 1) * sizeof(int64_t)))) return st;
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

}  // namespace ibvt
