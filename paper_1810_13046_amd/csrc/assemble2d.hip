// The planar coupling: Q1 (bilinear) hats on a staggered rectilinear 2D grid
// against P1 triangles, the setting of the paper's 2D experiments (Section
// 4), with the operators of Section 2.3 taken over areas:
//   B^d_ij = ∫ λ_i N^d_j dA (d = 0, 1), S = P1 mass |T|(1+δ_il)/12 or its
//   row sums |T|/3, dual multipliers ψ_i = 4λ_i − 1 (S = diag(m)).
//
//  k_tri_prep   per triangle: bounding box -> cell range on each component's
//               lattice, area, record (vertices, determinant), ∇λ.
//  k_pairs2<T>  one lane per (triangle, component, cell) pair: the ten
//               moments ∫∫ s^a t^b (a+b <= 3) of the piece in the cell's
//               centred unit coordinates, by Green's theorem over the piece
//               boundary (no polygon is built), then the 3 x 4 values
//               ∫ λ_i N_j from the moments.  The moments and values are
//               computed in double in both precisions (only the stored
//               values are float in mixed precision): the planar pieces are
//               cheap, and thin triangles expanded about the cell centre
//               lose several digits in float.
//  k_rows2<T>   one lane per (vertex, component): sums the vertex's pieces
//               into its node box in a fixed order and compacts the row.
//  transpose and the applies are shared with the 3D path (component count
//  from the handle).
//  reverse mode: k_shape2 turns the kept moments into the per-piece shape
//  terms, k_pair_sums2 adds them per (component, triangle), k_grad2 sums
//  those per vertex with the mass term.
#include "internal.hpp"
#include "plane.hpp"

#include <climits>

namespace ibvt {

namespace {

inline unsigned blocks_for(int64_t n, int threads) {
  return unsigned(ceil_div(n > 0 ? n : 1, threads));
}

__device__ __forceinline__ int upper_bound2(const double* L, int n, double x) {
  int lo = 0, hi = n;  // first index with L[idx] > x
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (L[mid] <= x) lo = mid + 1; else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ int lower_bound2(const double* L, int n, double x) {
  int lo = 0, hi = n;  // first index with L[idx] >= x
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (L[mid] < x) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// ---------------------------------------------------------------------------
// per-triangle preparation
// ---------------------------------------------------------------------------

__global__ void k_tri_prep(int64_t n_t, const double* __restrict__ X,
                           const int32_t* __restrict__ tris, const double* __restrict__ lat,
                           LatDesc ld, double* __restrict__ area, CellRange* __restrict__ rng,
                           int64_t* __restrict__ cnt, double* __restrict__ trirec,
                           double* __restrict__ grad, unsigned* flags,
                           unsigned long long* counters) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  bool zero = false;
  if (t < n_t) {
    double P[3][2];
    bool finite = true;
    for (int k = 0; k < 3; ++k) {
      const int64_t v = tris[3 * t + k];
      for (int e = 0; e < 2; ++e) {
        P[k][e] = X[2 * v + e];
        finite &= isfinite(P[k][e]);
      }
    }
    double mn[2], mx[2];
    for (int e = 0; e < 2; ++e) {
      mn[e] = fmin(fmin(P[0][e], P[1][e]), P[2][e]);
      mx[e] = fmax(fmax(P[0][e], P[1][e]), P[2][e]);
    }
    const double det = (P[1][0] - P[0][0]) * (P[2][1] - P[0][1]) -
                       (P[1][1] - P[0][1]) * (P[2][0] - P[0][0]);
    area[t] = finite ? 0.5 * fabs(det) : 0.0;
    double r[kTriRec] = {P[0][0], P[0][1], P[1][0], P[1][1], P[2][0], P[2][1], det, 0.0};
    store_row<kTriRec>(trirec + t * kTriRec, r);
    // ∇λ_i = (y_{i+1} - y_{i+2}, x_{i+2} - x_{i+1}) / det
    double g[6] = {0, 0, 0, 0, 0, 0};
    if (finite && det != 0.0) {
      for (int i = 0; i < 3; ++i) {
        const int i1 = (i + 1) % 3, i2 = (i + 2) % 3;
        g[2 * i] = (P[i1][1] - P[i2][1]) / det;
        g[2 * i + 1] = (P[i2][0] - P[i1][0]) / det;
      }
    }
    for (int k = 0; k < 6; ++k) grad[6 * t + k] = g[k];
    zero = finite && (det == 0.0);
    if (!finite) atomicOr(flags, kFlagNonFinite);
    for (int d = 0; d < 2; ++d) {
      CellRange rg;
      bool ok = finite && !zero;
      for (int e = 0; e < 2; ++e) {
        const double* L = lat + ld.off[3 * d + e];
        const int n = ld.n[3 * d + e];
        if (!(mn[e] >= L[0] && mx[e] <= L[n - 1])) {
          if (finite) atomicOr(flags, kFlagOutOfGrid);
          ok = false;
          rg.lo[e] = 0;
          rg.n[e] = 0;
          continue;
        }
        int lo = upper_bound2(L, n, mn[e]) - 1;
        lo = min(max(lo, 0), n - 2);
        int hi = lower_bound2(L, n, mx[e]) - 1;
        hi = min(max(hi, lo), n - 2);
        rg.lo[e] = lo;
        rg.n[e] = hi - lo + 1;
      }
      rg.lo[2] = 0;
      rg.n[2] = 1;
      if (!ok) rg.n[0] = rg.n[1] = rg.n[2] = 0;
      rng[d * n_t + t] = rg;
      const int64_t c = int64_t(rg.n[0]) * rg.n[1];
      cnt[d * n_t + t] = c;
      if (c > kMaxTetCells) atomicOr(flags, kFlagTetSpan);
    }
  }
  const uint64_t zm = ballot64(zero);
  if (lane_id() == 0 && zm) atomicAdd(&counters[kCntZeroTets], (unsigned long long)popc64(zm));
}

__global__ void k_owner2(int64_t n_tc, const int64_t* __restrict__ off,
                         int32_t* __restrict__ owner) {
  const int64_t tc = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (tc >= n_tc) return;
  for (int64_t p = off[tc]; p < off[tc + 1]; ++p) owner[p] = int32_t(tc);
}

// Cell of pair p in the planar layout (component d, triangle t, cell ci).
__device__ __forceinline__ void pair_cell2(int64_t p, int64_t n_t, const int32_t* owner,
                                           const int64_t* pair_off, const CellRange* rng,
                                           const double* lat, const LatDesc& ld, int& d,
                                           int64_t& t, int ci[2], double lo[2], double hi[2]) {
  const int64_t tc = owner[p];
  d = int(tc >= n_t);
  t = tc - int64_t(d) * n_t;
  const CellRange r = rng[tc];
  const uint32_t q = uint32_t(p - pair_off[tc]);
  const uint32_t n0 = uint32_t(r.n[0]);
  const uint32_t qy = q / n0;
  ci[0] = r.lo[0] + int(q - qy * n0);
  ci[1] = r.lo[1] + int(qy);
  for (int e = 0; e < 2; ++e) {
    const double* L = lat + ld.off[3 * d + e];
    lo[e] = L[ci[e]];
    hi[e] = L[ci[e] + 1];
  }
}

// One lane per pair: the piece moments (kept for the reverse mode) and the
// twelve values ∫ λ_i N_j, written to pval[pair][i*4 + corner]; with dual
// set, the dual multipliers' values 4 b_i - Σ_k b_k.
template <typename T>
__global__ __launch_bounds__(256) void k_pairs2(
    int64_t n_pairs, int64_t n_t, const int32_t* __restrict__ owner,
    const int64_t* __restrict__ pair_off, const CellRange* __restrict__ rng,
    const double* __restrict__ trirec, const double* __restrict__ lat, LatDesc ld,
    double drop_rel, uint8_t* __restrict__ keep, T* __restrict__ pval,
    double* __restrict__ pmom, int dual, unsigned long long* counters) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  bool kept = false, dropped = false;
  if (p < n_pairs) {
    int d, ci[2];
    int64_t t;
    double lo[2], hi[2];
    pair_cell2(p, n_t, owner, pair_off, rng, lat, ld, d, t, ci, lo, hi);
    double r[kTriRec];
    load_row<kTriRec>(trirec + t * kTriRec, r);
    double V[3][2];
    ccw_vertices(r, V);
    double m[kMom2];
    double au;
    piece_moments2<double>(V, lo, hi, m, au);
    const double parea = au * (hi[0] - lo[0]) * (hi[1] - lo[1]);
    kept = parea > drop_rel * 0.5 * fabs(r[6]);
    dropped = !kept && parea > 0.0;
    double out[12];
    if (kept) {
      piece_values2<double>(r, lo, hi, m, dual, out);
    } else {
#pragma unroll
      for (int k = 0; k < 12; ++k) out[k] = 0.0;
    }
    keep[p] = kept ? 1 : 0;
    T vals[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) vals[k] = T(out[k]);
    store_row<12>(pval + p * 12, vals);
    double mp[kMom2Pad];
#pragma unroll
    for (int k = 0; k < kMom2; ++k) mp[k] = kept ? m[k] : 0.0;
    mp[10] = mp[11] = 0.0;
    store_row<kMom2Pad>(pmom + p * kMom2Pad, mp);
  }
  const uint64_t km = ballot64(kept), dm = ballot64(dropped);
  if (lane_id() == 0) {
    if (km) atomicAdd(&counters[kCntPieces], (unsigned long long)popc64(km));
    if (dm) atomicAdd(&counters[kCntDropped], (unsigned long long)popc64(dm));
  }
}

// ---------------------------------------------------------------------------
// rows of B^d: one lane per (vertex, component)
// ---------------------------------------------------------------------------

// Node box of row w = d*n_v + i: the union of the incident triangles' cell
// ranges, as lo[2], extent[2] (nodes) in box[2w .. 2w+3]; cap[w] = its size.
__global__ void k_row_box2(int64_t n_v, int64_t n_t, const int64_t* __restrict__ vt_ptr,
                           const int32_t* __restrict__ vt_tri, const CellRange* __restrict__ rng,
                           int32_t* __restrict__ box, int64_t* __restrict__ cap) {
  const int64_t w = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (w >= 2 * n_v) return;
  const int d = int(w >= n_v);
  const int64_t i = w - int64_t(d) * n_v;
  int bmin[2] = {INT_MAX, INT_MAX}, bmax[2] = {INT_MIN, INT_MIN};
  for (int64_t k = vt_ptr[i]; k < vt_ptr[i + 1]; ++k) {
    const CellRange r = rng[int64_t(d) * n_t + vt_tri[k]];
    if (int64_t(r.n[0]) * r.n[1] == 0) continue;
    for (int e = 0; e < 2; ++e) {
      bmin[e] = min(bmin[e], r.lo[e]);
      bmax[e] = max(bmax[e], r.lo[e] + r.n[e]);
    }
  }
  int64_t sz = 1;
  for (int e = 0; e < 2; ++e) {
    const bool any = bmin[e] <= bmax[e];
    box[4 * w + e] = any ? bmin[e] : 0;
    box[4 * w + 2 + e] = any ? bmax[e] - bmin[e] + 1 : 0;
    sz *= any ? bmax[e] - bmin[e] + 1 : 0;
  }
  cap[w] = sz;
}

// Gathers the kept pieces of the incident triangles (ascending) in cell
// order into the row's node box at tmp_off[w] (sum order fixed, so the
// result does not depend on timing), then compacts the touched nodes in
// column order to the front of that space.
template <typename T>
__global__ void k_rows2(int64_t n_v, int64_t n_t, const int64_t* __restrict__ vt_ptr,
                        const int32_t* __restrict__ vt_tri, const int32_t* __restrict__ tris,
                        const CellRange* __restrict__ rng, const int64_t* __restrict__ pair_off,
                        const uint8_t* __restrict__ keep, const T* __restrict__ pval, LatDesc ld,
                        const int32_t* __restrict__ box, const int64_t* __restrict__ tmp_off,
                        int32_t* __restrict__ tmp_col, T* __restrict__ tmp_val,
                        int64_t* __restrict__ rownnz) {
  const int64_t w = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (w >= 2 * n_v) return;
  const int d = int(w >= n_v);
  const int64_t i = w - int64_t(d) * n_v;
  const int bx0 = box[4 * w], by0 = box[4 * w + 1], bnx = box[4 * w + 2], bny = box[4 * w + 3];
  const int64_t base = tmp_off[w];
  const int64_t cap = int64_t(bnx) * bny;
  const int nx = ld.n[3 * d];
  for (int64_t k = 0; k < cap; ++k) {
    tmp_col[base + k] = -1;
    tmp_val[base + k] = T(0);
  }
  for (int64_t k = vt_ptr[i]; k < vt_ptr[i + 1]; ++k) {
    const int64_t t = vt_tri[k];
    const int la = tris[3 * t + 1] == int32_t(i) ? 1 : (tris[3 * t + 2] == int32_t(i) ? 2 : 0);
    const int64_t tc = int64_t(d) * n_t + t;
    const CellRange r = rng[tc];
    const int64_t p0 = pair_off[tc], p1 = pair_off[tc + 1];
    for (int64_t p = p0; p < p1; ++p) {
      if (!keep[p]) continue;
      const int q = int(p - p0);
      const int cx = r.lo[0] + q % r.n[0], cy = r.lo[1] + q / r.n[0];
      const T* v = pval + p * 12 + la * 4;
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int a = 0; a < 2; ++a) {
          const int64_t kb = int64_t(cx + a - bx0) + int64_t(bnx) * (cy + b - by0);
          tmp_val[base + kb] += v[a + 2 * b];
          tmp_col[base + kb] = (cx + a) + nx * (cy + b);
        }
    }
  }
  int64_t out = 0;
  for (int64_t k = 0; k < cap; ++k) {
    const int32_t c = tmp_col[base + k];
    if (c < 0) continue;
    tmp_col[base + out] = c;
    tmp_val[base + out] = tmp_val[base + k];
    ++out;
  }
  rownnz[w] = out;
}

template <typename T>
__global__ void k_rows_compact2(int64_t n_v, const int64_t* __restrict__ tmp_off,
                                const int32_t* __restrict__ tmp_col, const T* __restrict__ tmp_val,
                                const int64_t* __restrict__ rp0, const int64_t* __restrict__ rp1,
                                int32_t* __restrict__ c0, int32_t* __restrict__ c1,
                                T* __restrict__ v0, T* __restrict__ v1) {
  const int64_t w = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (w >= 2 * n_v) return;
  const int d = int(w >= n_v);
  const int64_t i = w - int64_t(d) * n_v;
  const int64_t* rp = d ? rp1 : rp0;
  int32_t* col = d ? c1 : c0;
  T* val = d ? v1 : v0;
  const int64_t src = tmp_off[w], dst = rp[i], n = rp[i + 1] - rp[i];
  for (int64_t k = 0; k < n; ++k) {
    col[dst + k] = tmp_col[src + k];
    val[dst + k] = tmp_val[src + k];
  }
}

// ---------------------------------------------------------------------------
// masses
// ---------------------------------------------------------------------------

template <typename T>
__global__ void k_lumped2(int64_t n_v, const int64_t* __restrict__ vt_ptr,
                          const int32_t* __restrict__ vt_tri, const double* __restrict__ area,
                          double* __restrict__ m, T* __restrict__ minv) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n_v) return;
  double s = 0.0;
  for (int64_t k = vt_ptr[i]; k < vt_ptr[i + 1]; ++k) s += area[vt_tri[k]];
  s /= 3.0;
  m[i] = s;
  minv[i] = (s > 0.0) ? T(1.0 / s) : T(0);
}

// Consistent mass rows M_il = Σ_{T ∋ i, l} |T|(1 + δ_il)/12, one lane per
// vertex, incident triangles in ascending order.
__global__ void k_mass_values2(int64_t n_v, const int64_t* __restrict__ vt_ptr,
                               const int32_t* __restrict__ vt_tri, const int32_t* __restrict__ tris,
                               const double* __restrict__ area, const int64_t* __restrict__ rowptr,
                               const int32_t* __restrict__ col, double* __restrict__ val,
                               float* __restrict__ val32, double* __restrict__ dinv) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n_v) return;
  const int64_t rb = rowptr[i], re = rowptr[i + 1];
  for (int64_t c = rb; c < re; ++c) val[c] = 0.0;
  for (int64_t k = vt_ptr[i]; k < vt_ptr[i + 1]; ++k) {
    const int64_t t = vt_tri[k];
    const double wk = area[t] / 12.0;
    for (int q = 0; q < 3; ++q) {
      const int l = tris[3 * t + q];
      for (int64_t c = rb; c < re; ++c)
        if (col[c] == l) val[c] += (int64_t(l) == i) ? 2.0 * wk : wk;
    }
  }
  double diag = 0.0;
  for (int64_t c = rb; c < re; ++c) {
    if (val32) val32[c] = float(val[c]);
    if (int64_t(col[c]) == i) diag = val[c];
  }
  dinv[i] = (diag > 0.0) ? 1.0 / diag : 0.0;
}

// ---------------------------------------------------------------------------
// reverse mode: shape derivative
// ---------------------------------------------------------------------------

// Per kept piece and component, with w = Σ_i z_i λ_i (dual: z_i replaced by
// 4 z_i - Σ_k z_k) and U = Σ_j u_j N_j on the cell,
//   G[a][k] = ∂_k λ_a ∫ w U + ∫ λ_a w ∂_k U      (a = 0..2, k = x, y),
// from the piece moments, in double; written to pg[pair][a*2 + k].
template <typename T>
__global__ __launch_bounds__(256) void k_shape2(
    int64_t n_pairs, int64_t n_t, int64_t n_v, const int32_t* __restrict__ owner,
    const int64_t* __restrict__ pair_off, const CellRange* __restrict__ rng,
    const uint8_t* __restrict__ keep, const double* __restrict__ pmom,
    const double* __restrict__ trirec, const int32_t* __restrict__ tris,
    const double* __restrict__ lat, LatDesc ld, const T* __restrict__ z, const T* u0,
    const T* u1, double* __restrict__ pg, int dual) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= n_pairs) return;
  double* out = pg + p * 6;
  if (!keep[p]) {
#pragma unroll
    for (int k = 0; k < 6; ++k) out[k] = 0.0;
    return;
  }
  int d, ci[2];
  int64_t t;
  double lo[2], hi[2];
  pair_cell2(p, n_t, owner, pair_off, rng, lat, ld, d, t, ci, lo, hi);
  double r[kTriRec];
  load_row<kTriRec>(trirec + t * kTriRec, r);
  double m[kMom2Pad];
  load_row<kMom2Pad>(pmom + p * kMom2Pad, m);
  const double hx = hi[0] - lo[0], hy = hi[1] - lo[1];
  double l0[3];
  bary_at(r, 0.5 * (lo[0] + hi[0]), 0.5 * (lo[1] + hi[1]), l0);
  const double idet = 1.0 / r[6];
  double la0[3], las[3], lat_[3];
  double gx[3], gy[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const int i1 = (i + 1) % 3, i2 = (i + 2) % 3;
    gx[i] = (r[2 * i1 + 1] - r[2 * i2 + 1]) * idet;
    gy[i] = (r[2 * i2] - r[2 * i1]) * idet;
    la0[i] = l0[i];
    las[i] = gx[i] * hx;
    lat_[i] = gy[i] * hy;
  }
  double zl[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) zl[i] = double(z[int64_t(d) * n_v + tris[3 * t + i]]);
  if (dual) {
    const double sz = zl[0] + zl[1] + zl[2];
#pragma unroll
    for (int i = 0; i < 3; ++i) zl[i] = 4.0 * zl[i] - sz;
  }
  double w0 = 0, w1 = 0, w2 = 0;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    w0 += zl[i] * la0[i];
    w1 += zl[i] * las[i];
    w2 += zl[i] * lat_[i];
  }
  const T* u = d ? u1 : u0;
  const int nx = ld.n[3 * d];
  const int64_t j00 = int64_t(ci[0]) + int64_t(nx) * ci[1];
  const double c00 = u[j00], c10 = u[j00 + 1], c01 = u[j00 + nx], c11 = u[j00 + nx + 1];
  // U = e0 + es s + et t + est s t
  const double e0 = 0.25 * (c00 + c10 + c01 + c11);
  const double es = 0.5 * (c10 + c11 - c00 - c01);
  const double et = 0.5 * (c01 + c11 - c00 - c10);
  const double est = c00 + c11 - c10 - c01;
  // moments: 0:1 1:s 2:t 3:s² 4:st 5:t² 6:s³ 7:s²t 8:st² 9:t³
  const double wU = w0 * (e0 * m[0] + es * m[1] + et * m[2] + est * m[4]) +
               w1 * (e0 * m[1] + es * m[3] + et * m[4] + est * m[7]) +
               w2 * (e0 * m[2] + es * m[4] + et * m[5] + est * m[8]);
  const double A = hx * hy;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    // λ_a w = q00 + q10 s + q01 t + q20 s² + q11 st + q02 t²
    const double q00 = la0[a] * w0, q10 = la0[a] * w1 + las[a] * w0, q01 = la0[a] * w2 + lat_[a] * w0;
    const double q20 = las[a] * w1, q11 = las[a] * w2 + lat_[a] * w1, q02 = lat_[a] * w2;
    const double Q = q00 * m[0] + q10 * m[1] + q01 * m[2] + q20 * m[3] + q11 * m[4] + q02 * m[5];
    const double Qt = q00 * m[2] + q10 * m[4] + q01 * m[5] + q20 * m[7] + q11 * m[8] + q02 * m[9];
    const double Qs = q00 * m[1] + q10 * m[3] + q01 * m[4] + q20 * m[6] + q11 * m[7] + q02 * m[8];
    // ∂_x U = (es + est t)/hx, ∂_y U = (et + est s)/hy; dA = hx hy ds dt
    out[2 * a] = gx[a] * A * wU + hy * (es * Q + est * Qt);
    out[2 * a + 1] = gy[a] * A * wU + hx * (et * Q + est * Qs);
  }
}

// Mass term coefficient per triangle (summed over both components):
// |T| s_T with s_T = Σ_d (z·u + Σz Σu)/12 (consistent) or z·u/3 (lumped).
template <typename T>
__global__ void k_mass_coef2(int64_t n_t, int64_t n_v, const int32_t* __restrict__ tris,
                             const double* __restrict__ area, const T* __restrict__ z,
                             const T* __restrict__ us, int mass, double* __restrict__ out) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= n_t) return;
  double sT = 0.0;
  for (int d = 0; d < 2; ++d) {
    double zs = 0, uss = 0, zu = 0;
    for (int q = 0; q < 3; ++q) {
      const int64_t v = tris[3 * t + q];
      const double zq = double(z[int64_t(d) * n_v + v]), uq = double(us[int64_t(d) * n_v + v]);
      zs += zq;
      uss += uq;
      zu += zq * uq;
    }
    sT += (mass == 1) ? (zu + zs * uss) / 12.0 : zu / 3.0;
  }
  out[t] = area[t] * sT;
}

// Per (component, triangle) sums of the pair terms, pairs in order.
__global__ void k_pair_sums2(int64_t n_tc, const int64_t* __restrict__ pair_off,
                             const double* __restrict__ pg, double* __restrict__ pgt) {
  const int64_t w = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (w >= n_tc) return;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (int64_t p = pair_off[w]; p < pair_off[w + 1]; ++p)
#pragma unroll
    for (int k = 0; k < 6; ++k) acc[k] += pg[p * 6 + k];
#pragma unroll
  for (int k = 0; k < 6; ++k) pgt[w * 6 + k] = acc[k];
}

// gX[a] += alpha (Σ over incident triangles and components of the summed
// pair terms - mcoef_T ∇λ_a), one lane per vertex, fixed order.
__global__ void k_grad2(int64_t n_v, int64_t n_t, const int64_t* __restrict__ vt_ptr,
                        const int32_t* __restrict__ vt_tri, const int32_t* __restrict__ tris,
                        const double* __restrict__ pgt, const double* __restrict__ grad,
                        const double* __restrict__ mcoef, double alpha,
                        double* __restrict__ gX) {
  const int64_t a = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (a >= n_v) return;
  double g0 = 0.0, g1 = 0.0;
  for (int64_t k = vt_ptr[a]; k < vt_ptr[a + 1]; ++k) {
    const int64_t t = vt_tri[k];
    const int la = tris[3 * t + 1] == int32_t(a) ? 1 : (tris[3 * t + 2] == int32_t(a) ? 2 : 0);
    for (int d = 0; d < 2; ++d) {
      const int64_t tc = int64_t(d) * n_t + t;
      g0 += pgt[tc * 6 + 2 * la];
      g1 += pgt[tc * 6 + 2 * la + 1];
    }
    if (mcoef) {
      g0 -= mcoef[t] * grad[6 * t + 2 * la];
      g1 -= mcoef[t] * grad[6 * t + 2 * la + 1];
    }
  }
  gX[2 * a] += alpha * g0;
  gX[2 * a + 1] += alpha * g1;
}

// ---------------------------------------------------------------------------
// host drivers
// ---------------------------------------------------------------------------

template <typename T>
int assemble2_typed(ibvt_coupling* c, hipStream_t s) {
  const int64_t n_t = c->n_tet, n_v = c->n_vert;
  int st;
  unsigned* flags = c->flags_dev.as<unsigned>();
  auto* counters = c->counters.as<unsigned long long>();
  if ((st = hip_check(hipMemsetAsync(flags, 0, sizeof(unsigned), s), "memset"))) return st;
  if ((st = hip_check(hipMemsetAsync(counters, 0, kCntSlots * sizeof(unsigned long long), s),
                      "memset")))
    return st;
  {
    ProfScope ps("tri_prep", s);
    k_tri_prep<<<blocks_for(n_t, 256), 256, 0, s>>>(
        n_t, c->X.as<double>(), c->tets.as<int32_t>(), c->lat.as<double>(), c->ld,
        c->tetvol.as<double>(), c->rng.as<CellRange>(), c->cnt.as<int64_t>(),
        c->tetrec.as<double>(), c->tetgrad.as<double>(), flags, counters);
  }
  if ((st = hip_check(hipGetLastError(), "prep launch"))) return st;
  if ((st = scan_i64(c, c->cnt.as<int64_t>(), c->pair_off.as<int64_t>(), 2 * n_t, s))) return st;
  if ((st = check_flags(c, s))) return st;
  int64_t n_pairs = 0;
  if ((st = read_back(c, &n_pairs, c->pair_off.as<int64_t>() + 2 * n_t, sizeof(int64_t), s)))
    return st;
  if (n_pairs >= (int64_t(1) << 31) - 1)
    return set_error(IBVT_E_CAPACITY, "2^31 or more (triangle, cell) pairs");
  c->n_pairs = n_pairs;
  if ((st = ensure(c, c->owner, size_t(n_pairs + 1) * sizeof(int32_t)))) return st;
  if ((st = ensure(c, c->keep, size_t(n_pairs + 1)))) return st;
  if ((st = ensure(c, c->pval, size_t(n_pairs + 1) * 12 * sizeof(T)))) return st;
  if ((st = ensure(c, c->pmom, size_t(n_pairs + 1) * kMom2Pad * sizeof(double)))) return st;
  c->mom_valid = false;
  k_owner2<<<blocks_for(2 * n_t, 256), 256, 0, s>>>(2 * n_t, c->pair_off.as<int64_t>(),
                                                    c->owner.as<int32_t>());
  if (n_pairs > 0) {
    ProfScope ps("pairs2d", s);
    k_pairs2<T><<<blocks_for(n_pairs, 256), 256, 0, s>>>(
        n_pairs, n_t, c->owner.as<int32_t>(), c->pair_off.as<int64_t>(), c->rng.as<CellRange>(),
        c->tetrec.as<double>(), c->lat.as<double>(), c->ld, 1e-14, c->keep.as<uint8_t>(),
        c->pval.as<T>(), c->pmom.as<double>(), c->dual ? 1 : 0, counters);
  }
  if ((st = hip_check(hipGetLastError(), "pairs launch"))) return st;
  // rows
  if ((st = ensure(c, c->rowbox, size_t(2 * n_v + 1) * 4 * sizeof(int32_t)))) return st;
  if ((st = ensure(c, c->rowcap, size_t(2 * n_v + 1) * sizeof(int64_t)))) return st;
  if ((st = ensure(c, c->rowtmpoff, size_t(2 * n_v + 1) * sizeof(int64_t)))) return st;
  {
    ProfScope ps("rows_box", s);
    k_row_box2<<<blocks_for(2 * n_v, 256), 256, 0, s>>>(
        n_v, n_t, c->vt_ptr.as<int64_t>(), c->vt_tet.as<int32_t>(), c->rng.as<CellRange>(),
        c->rowbox.as<int32_t>(), c->rowcap.as<int64_t>());
  }
  if ((st = scan_i64(c, c->rowcap.as<int64_t>(), c->rowtmpoff.as<int64_t>(), 2 * n_v, s)))
    return st;
  int64_t tmp_total = 0;
  if ((st = read_back(c, &tmp_total, c->rowtmpoff.as<int64_t>() + 2 * n_v, sizeof(int64_t), s)))
    return st;
  if ((st = ensure(c, c->rowtmpcol, size_t(tmp_total + 1) * sizeof(int32_t)))) return st;
  if ((st = ensure(c, c->rowtmpval, size_t(tmp_total + 1) * sizeof(T)))) return st;
  {
    ProfScope ps("rows_gather", s);
    k_rows2<T><<<blocks_for(2 * n_v, 128), 128, 0, s>>>(
        n_v, n_t, c->vt_ptr.as<int64_t>(), c->vt_tet.as<int32_t>(), c->tets.as<int32_t>(),
        c->rng.as<CellRange>(), c->pair_off.as<int64_t>(), c->keep.as<uint8_t>(),
        c->pval.as<T>(), c->ld, c->rowbox.as<int32_t>(), c->rowtmpoff.as<int64_t>(),
        c->rowtmpcol.as<int32_t>(), c->rowtmpval.as<T>(), c->rownnz.as<int64_t>());
  }
  if ((st = hip_check(hipGetLastError(), "rows launch"))) return st;
  for (int d = 0; d < 2; ++d) {
    c->B[d].nrows = n_v;
    if ((st = scan_i64(c, c->rownnz.as<int64_t>() + d * n_v, c->B[d].rowptr.as<int64_t>(), n_v,
                       s)))
      return st;
  }
  for (int d = 0; d < 2; ++d) {
    int64_t nnz = 0;
    if ((st = read_back(c, &nnz, c->B[d].rowptr.as<int64_t>() + n_v, sizeof(int64_t), s)))
      return st;
    c->B[d].nnz = nnz;
    if (nnz >= (int64_t(1) << 31) - 1)
      return set_error(IBVT_E_CAPACITY, "more than 2^31 nonzeros in one component of B");
    if ((st = ensure(c, c->B[d].col, size_t(nnz + 1) * sizeof(int32_t)))) return st;
    if ((st = ensure(c, c->B[d].val, size_t(nnz + 1) * sizeof(T)))) return st;
  }
  {
    ProfScope ps("rows_compact", s);
    k_rows_compact2<T><<<blocks_for(2 * n_v, 256), 256, 0, s>>>(
        n_v, c->rowtmpoff.as<int64_t>(), c->rowtmpcol.as<int32_t>(), c->rowtmpval.as<T>(),
        c->B[0].rowptr.as<int64_t>(), c->B[1].rowptr.as<int64_t>(), c->B[0].col.as<int32_t>(),
        c->B[1].col.as<int32_t>(), c->B[0].val.as<T>(), c->B[1].val.as<T>());
  }
  if ((st = hip_check(hipGetLastError(), "rows compact launch"))) return st;
  for (int d = 0; d < 2; ++d) {
    ProfScope ps("transpose", s);
    if ((st = transpose_one<T>(c, d, s))) return st;
  }
  {
    ProfScope ps("masses", s);
    k_lumped2<T><<<blocks_for(n_v, 256), 256, 0, s>>>(n_v, c->vt_ptr.as<int64_t>(),
                                                      c->vt_tet.as<int32_t>(),
                                                      c->tetvol.as<double>(), c->mlump.as<double>(),
                                                      c->minv.as<T>());
    if (c->has_M)
      k_mass_values2<<<blocks_for(n_v, 256), 256, 0, s>>>(
          n_v, c->vt_ptr.as<int64_t>(), c->vt_tet.as<int32_t>(), c->tets.as<int32_t>(),
          c->tetvol.as<double>(), c->M.rowptr.as<int64_t>(), c->M.col.as<int32_t>(),
          c->M.val.as<double>(), c->precision == IBVT_FP32_MIXED ? c->Mval32.as<float>() : nullptr,
          c->Mdiag_inv.as<double>());
  }
  if ((st = hip_check(hipGetLastError(), "mass launch"))) return st;
  unsigned long long cnt[kCntSlots];
  if ((st = read_back(c, cnt, counters, sizeof(cnt), s))) return st;
  c->stats.pairs = n_pairs;
  c->stats.pieces = int64_t(cnt[kCntPieces]);
  c->stats.dropped = int64_t(cnt[kCntDropped]);
  c->stats.zero_tets = int64_t(cnt[kCntZeroTets]);
  c->stats.subtets = 0;
  c->stats.dist_evals = 0;
  c->stats.cut_points = 0;
  c->mom_valid = true;
  c->stats.assemblies += 1;
  return check_flags(c, s);
}

template <typename T>
int shape2_typed(ibvt_coupling* c, const T* z, const T* u0, const T* u1, const T* us, int mass,
                 double alpha, double* gX, hipStream_t s) {
  const int64_t n_t = c->n_tet, n_v = c->n_vert, n_pairs = c->n_pairs;
  int st;
  const size_t pg_bytes = (size_t(n_pairs + 1) * 6 * sizeof(double) + 255) & ~size_t(255);
  if ((st = ensure(c, c->work2, pg_bytes + size_t(2 * n_t + 1) * 6 * sizeof(double)))) return st;
  if ((st = ensure(c, c->mcoef, size_t(n_t + 1) * sizeof(double)))) return st;
  double* pg = c->work2.as<double>();
  double* pgt = reinterpret_cast<double*>(c->work2.as<char>() + pg_bytes);
  {
    ProfScope ps("shape2d", s);
    if (n_pairs > 0)
      k_shape2<T><<<blocks_for(n_pairs, 256), 256, 0, s>>>(
          n_pairs, n_t, n_v, c->owner.as<int32_t>(), c->pair_off.as<int64_t>(),
          c->rng.as<CellRange>(), c->keep.as<uint8_t>(), c->pmom.as<double>(), c->tetrec.as<double>(),
          c->tets.as<int32_t>(), c->lat.as<double>(), c->ld, z, u0, u1, pg, c->dual ? 1 : 0);
    if (n_t > 0)
      k_pair_sums2<<<blocks_for(2 * n_t, 256), 256, 0, s>>>(2 * n_t, c->pair_off.as<int64_t>(), pg,
                                                             pgt);
    const double* mc = nullptr;
    if (mass >= 0) {
      k_mass_coef2<T><<<blocks_for(n_t, 256), 256, 0, s>>>(n_t, n_v, c->tets.as<int32_t>(),
                                                           c->tetvol.as<double>(), z, us, mass,
                                                           c->mcoef.as<double>());
      mc = c->mcoef.as<double>();
    }
    k_grad2<<<blocks_for(n_v, 256), 256, 0, s>>>(n_v, n_t, c->vt_ptr.as<int64_t>(),
                                                 c->vt_tet.as<int32_t>(), c->tets.as<int32_t>(),
                                                 pgt, c->tetgrad.as<double>(), mc, alpha, gX);
  }
  return hip_check(hipGetLastError(), "shape launch");
}

}  // namespace

int assemble_all_2d(ibvt_coupling* c, hipStream_t s) {
  const int64_t n_t = c->n_tet, n_v = c->n_vert;
  int st;
  if ((st = ensure(c, c->tetvol, size_t(n_t + 1) * sizeof(double)))) return st;
  if ((st = ensure(c, c->tetrec, size_t(n_t + 1) * kTriRec * sizeof(double)))) return st;
  if ((st = ensure(c, c->tetgrad, size_t(n_t + 1) * 6 * sizeof(double)))) return st;
  if ((st = ensure(c, c->rng, size_t(2 * n_t + 1) * sizeof(CellRange)))) return st;
  if ((st = ensure(c, c->cnt, size_t(2 * n_t + 1) * sizeof(int64_t)))) return st;
  if ((st = ensure(c, c->pair_off, size_t(2 * n_t + 1) * sizeof(int64_t)))) return st;
  if ((st = ensure(c, c->mlump, size_t(n_v + 1) * sizeof(double)))) return st;
  for (int d = 0; d < 2; ++d)
    if ((st = ensure(c, c->B[d].rowptr, size_t(n_v + 1) * sizeof(int64_t)))) return st;
  if (c->precision == IBVT_FP32_MIXED) {
    if ((st = ensure(c, c->minv, size_t(n_v + 1) * sizeof(float)))) return st;
    return assemble2_typed<float>(c, s);
  }
  if ((st = ensure(c, c->minv, size_t(n_v + 1) * sizeof(double)))) return st;
  return assemble2_typed<double>(c, s);
}

int shape_gradient_2d(ibvt_coupling* c, const void* z, const void* const u[3], const void* us,
                      int mass, double alpha, double* gX, hipStream_t s) {
  if (!c->mom_valid) return set_error(IBVT_E_INVALID, "no piece moments: assemble first");
  if (c->precision == IBVT_FP32_MIXED)
    return shape2_typed<float>(c, static_cast<const float*>(z), static_cast<const float*>(u[0]),
                               static_cast<const float*>(u[1]), static_cast<const float*>(us),
                               mass, alpha, gX, s);
  return shape2_typed<double>(c, static_cast<const double*>(z), static_cast<const double*>(u[0]),
                              static_cast<const double*>(u[1]), static_cast<const double*>(us),
                              mass, alpha, gX, s);
}

}  // namespace ibvt
