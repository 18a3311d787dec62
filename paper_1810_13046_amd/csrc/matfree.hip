// The coupling without stored matrices (IBVT_NO_STORE_B): every product with
// B^d or B^dT, and the shape derivative, clips and integrates the pieces
// again (Section 2.3, steps (II)-(III)) instead of reading an assembled
// matrix, so the handle holds per-tet data and the solid masses only.
//
// One lane per (component d, tet t) walks the tet's cells in index order
// (the order of its pairs in the assembled coupling), clips each cell in
// double (vertex graph in LDS), integrates the product's integrand on the
// piece exactly, already contracted with the field (∫ λ_i U with U = Σ_j
// x_j N_j for B x, ∫ w N_j with w = Σ_i y_i λ_i for B^T y: 4 or 8 sums per
// piece instead of the 32 ∫ λ_i N_j), and applies the assembly's drop rule
// (pieces of volume <= 1e-14 |T| are left out).  The (component, tet) items are ordered once per assembly by the
// vertex slots their cells need (the most planes any of their cells cuts:
// <= 3, 4, >= 5 → 10, 12, 16 slots, one launch each) and, within a class,
// by their cell count, so the lanes of a wave walk similar loops; then:
//   k_mf_tet_apply    B x:   pt[(d,t)][i] = Σ_cells Σ_j b_ij x_d[node_j]
//                     (sums in double), then k_mf_rows adds them per vertex
//                     over its incident tets in a fixed order and scales by
//                     1/m when asked;
//   k_mf_tet_spread   B^T y: out_d[node_j] += α Σ_i b_ij y_d[v_i] with
//                     device-scope atomic adds (the summation order of a
//                     node then depends on timing: results agree with the
//                     assembled product to rounding, not bit for bit);
//   k_mf_tet_shape    the per-(component, tet) shape terms
//                     Σ_cells [∫ λ_a w ∂_k U + ∂_k λ_a ∫ w U] (the same
//                     integrand as the re-clipping path of grad.hip), which
//                     shape_gather turns into g_X.
#include "geometry.hpp"
#include "internal.hpp"

namespace ibvt {

namespace {

constexpr double kDropRel = 1e-14;

// Per-lane set-up of one (component, tet): its geometry and cell range.
struct TetCells {
  int d;
  int64_t t;
  CellRange r;
  int64_t count;
};

__device__ __forceinline__ bool tet_cells(int64_t w, int64_t n_t, const CellRange* rng,
                                          TetCells& tc) {
  tc.d = int(w / n_t);
  tc.t = w - int64_t(tc.d) * n_t;
  tc.r = rng[w];
  tc.count = int64_t(tc.r.n[0]) * tc.r.n[1] * tc.r.n[2];
  return tc.count > 0;
}

// Entry (component d, axis e) of a lattice descriptor array, by selects on
// d (a runtime index into the kernel argument would copy it to scratch).
__device__ __forceinline__ int32_t ld_at(const int32_t a[9], int d, int e) {
  return d == 0 ? a[e] : (d == 1 ? a[3 + e] : a[6 + e]);
}

// Cell q of the range (x fastest) and its box.
__device__ __forceinline__ void range_cell(const CellRange& r, int64_t q, const double* lat,
                                           const LatDesc& ld, int d, int ci[3], double lo[3],
                                           double hi[3]) {
  const int64_t qy = q / r.n[0], qz = qy / r.n[1];
  ci[0] = r.lo[0] + int(q - qy * r.n[0]);
  ci[1] = r.lo[1] + int(qy - qz * r.n[1]);
  ci[2] = r.lo[2] + int(qz);
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    const double* L = lat + ld_at(ld.off, d, e);
    lo[e] = L[ci[e]];
    hi[e] = L[ci[e] + 1];
  }
}

// Dual multipliers: w = Σ_i z_i ψ_i = Σ_i (5 z_i − Σ_k z_k) λ_i.
template <typename T>
__device__ __forceinline__ void dual_weights_mf(T zl[4]) {
  const T s = zl[0] + zl[1] + zl[2] + zl[3];
#pragma unroll
  for (int k = 0; k < 4; ++k) zl[k] = T(5) * zl[k] - s;
}

// Σ_j u_j N_j at cell-local point p (corner j = a + 2b + 4c).
template <typename T>
__device__ __forceinline__ T trilinear(const T u[8], T px, T py, T pz) {
  const T x0 = u[0] + px * (u[1] - u[0]), x1 = u[2] + px * (u[3] - u[2]);
  const T x2 = u[4] + px * (u[5] - u[4]), x3 = u[6] + px * (u[7] - u[6]);
  const T y0 = x0 + py * (x1 - x0), y1 = x2 + py * (x3 - x2);
  return y0 + pz * (y1 - y0);
}

__device__ __forceinline__ bool piece_kept(double vol6, const double lo[3], const double hi[3],
                                           const TetGeom& G) {
  const double cv = (hi[0] - lo[0]) * (hi[1] - lo[1]) * (hi[2] - lo[2]);
  return vol6 * cv / 6.0 > kDropRel * (fabs(G.det) / 6.0);
}

__device__ __forceinline__ void load_tet(const double* tetrec, int64_t t, TetGeom& G) {
  double r[kTetRec];
  load_row<kTetRec>(tetrec + t * kTetRec, r);
  for (int k = 0; k < 4; ++k)
    for (int e = 0; e < 3; ++e) G.V[k][e] = r[3 * k + e];
  tet_geom(G);
}

// linear index of corner j = a + 2b + 4c of cell ci on a lattice NX x NY x .
__device__ __forceinline__ int64_t corner_node(const int ci[3], int j, int64_t NX, int64_t NY) {
  return (ci[0] + (j & 1)) + NX * ((ci[1] + ((j >> 1) & 1)) + NY * int64_t(ci[2] + (j >> 2)));
}

// One slot class of the (component, tet) order: items order[*first ..
// *end) (device pointers: the class bounds stay on the device).
struct TcList {
  const int32_t* order;
  const int64_t* first;
  const int64_t* end;
};

// The class's items, one per lane, in batches of 64 over a grid sized to
// the resident waves: ITEM_LOOP(lst, w) { body for item w }.  (A plain loop:
// a lambda capturing the kernel's parameters by reference would give them
// addresses, and the compiler then copies them to scratch.)
#define ITEM_LOOP(lst, w)                                                                  \
  for (int64_t i0_ = int64_t(blockIdx.x) * kWave, f_ = *(lst).first,                        \
               n_ = *(lst).end - *(lst).first;                                              \
       i0_ < n_; i0_ += int64_t(gridDim.x) * kWave)                                        \
    if (const int64_t i_ = i0_ + threadIdx.x; i_ < n_)                                      \
      if (const int64_t w = int64_t((lst).order[f_ + i_]); true)

template <typename T, int MAXV>
__global__ __launch_bounds__(kWave) void k_mf_tet_apply(
    TcList lst, int64_t n_t, const CellRange* __restrict__ rng, const double* __restrict__ tetrec,
    const double* __restrict__ lat, LatDesc ld, const T* x0, const T* x1, const T* x2, int dual,
    T* __restrict__ pt, unsigned* flags) {
  __shared__ double sx[MAXV * kWave], sy[MAXV * kWave], sz[MAXV * kWave];
  __shared__ uint32_t snb[MAXV * kWave];
  const int lane = threadIdx.x;
  const PolyView P{sx + lane, sy + lane, sz + lane, snb + lane, kWave, (1u << MAXV) - 1u};
  bool fail = false;
  ITEM_LOOP(lst, w) {
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    TetCells tc;
    if (tet_cells(w, n_t, rng, tc)) {
      TetGeom G;
      load_tet(tetrec, tc.t, G);
      const T* x = tc.d == 0 ? x0 : (tc.d == 1 ? x1 : x2);
      const int64_t NX = ld_at(ld.n, tc.d, 0), NY = ld_at(ld.n, tc.d, 1);
      for (int64_t q = 0; q < tc.count; ++q) {
        int ci[3];
        double lo[3], hi[3];
        range_cell(tc.r, q, lat, ld, tc.d, ci, lo, hi);
        T xl[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) xl[j] = x[corner_node(ci, j, NX, NY)];
        // Σ_j b_ij x_j = ∫ λ_i U with U = Σ_j x_j N_j: four sums per piece
        T LA[4], LG[4][3], b4[4] = {T(0), T(0), T(0), T(0)};
        double vol6 = 0.0;
        const bool ok = clip_fan_local<T, MAXV>(
            P, G, lo, hi, LA, LG, vol6, [&](const T (&y)[4][3], double det) {
              subtet_quad<T>(y, T(det), [&](T px, T py, T pz, T w) {
                const T wu = w * trilinear<T>(xl, px, py, pz);
#pragma unroll
                for (int i = 0; i < 4; ++i)
                  b4[i] += wu * (LA[i] + LG[i][0] * px + LG[i][1] * py + LG[i][2] * pz);
              });
            });
        if (!ok) {
          fail = true;
          continue;
        }
        if (!piece_kept(vol6, lo, hi, G)) continue;
        const T sc = T(-(hi[0] - lo[0]) * (hi[1] - lo[1]) * (hi[2] - lo[2]) / 6.0);
#pragma unroll
        for (int i = 0; i < 4; ++i) b4[i] *= sc;
        if (dual) {
          // ψ_i = 5 λ_i − Σ_k λ_k
          const T sum = b4[0] + b4[1] + b4[2] + b4[3];
#pragma unroll
          for (int i = 0; i < 4; ++i) b4[i] = T(5) * b4[i] - sum;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[i] += double(b4[i]);
      }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) pt[w * 4 + i] = T(acc[i]);
  }
  const uint64_t fm = ballot64(fail);
  if (lane == 0 && fm) atomicOr(flags, kFlagCapacity);
}

// y[d·n_v + i] = s_i Σ_{t ∋ i} pt[(d, t)][local index of i in t], incident
// tets in ascending order; s_i = 1/m_i or 1.
template <typename T>
__global__ __launch_bounds__(256) void k_mf_rows(int64_t n_v, int64_t n_t, int ncomp,
                                                 const int64_t* __restrict__ vt_ptr,
                                                 const int32_t* __restrict__ vt_tet,
                                                 const int32_t* __restrict__ tets,
                                                 const T* __restrict__ pt,
                                                 const T* __restrict__ scale, T* __restrict__ y) {
  const int64_t w = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (w >= int64_t(ncomp) * n_v) return;
  const int d = int(w / n_v);
  const int64_t i = w - int64_t(d) * n_v;
  double s = 0.0;
  for (int64_t k = vt_ptr[i]; k < vt_ptr[i + 1]; ++k) {
    const int64_t t = vt_tet[k];
    const int4 tv = *reinterpret_cast<const int4*>(tets + 4 * t);
    const int li =
        (tv.y == int32_t(i)) ? 1 : (tv.z == int32_t(i)) ? 2 : (tv.w == int32_t(i)) ? 3 : 0;
    s += double(pt[(int64_t(d) * n_t + t) * 4 + li]);
  }
  T v = T(s);
  if (scale) v *= scale[i];
  y[w] = v;
}

template <typename T, int MAXV>
__global__ __launch_bounds__(kWave) void k_mf_tet_spread(
    TcList lst, int64_t n_t, int64_t n_v, const CellRange* __restrict__ rng,
    const double* __restrict__ tetrec, const int32_t* __restrict__ tets,
    const double* __restrict__ lat, LatDesc ld, const T* __restrict__ ys, double alpha, int dual,
    T* o0, T* o1, T* o2, unsigned* flags) {
  __shared__ double sx[MAXV * kWave], sy[MAXV * kWave], sz[MAXV * kWave];
  __shared__ uint32_t snb[MAXV * kWave];
  const int lane = threadIdx.x;
  const PolyView P{sx + lane, sy + lane, sz + lane, snb + lane, kWave, (1u << MAXV) - 1u};
  bool fail = false;
  ITEM_LOOP(lst, w) {
    TetCells tc;
    if (!tet_cells(w, n_t, rng, tc)) continue;
    TetGeom G;
    load_tet(tetrec, tc.t, G);
    T zl[4];
    const int4 tv = *reinterpret_cast<const int4*>(tets + 4 * tc.t);
    const int32_t vv[4] = {tv.x, tv.y, tv.z, tv.w};
#pragma unroll
    for (int k = 0; k < 4; ++k) zl[k] = ys[int64_t(tc.d) * n_v + vv[k]];
    if (dual) dual_weights_mf<T>(zl);
    T* out = tc.d == 0 ? o0 : (tc.d == 1 ? o1 : o2);
    const int64_t NX = ld_at(ld.n, tc.d, 0), NY = ld_at(ld.n, tc.d, 1);
    for (int64_t q = 0; q < tc.count; ++q) {
      int ci[3];
      double lo[3], hi[3];
      range_cell(tc.r, q, lat, ld, tc.d, ci, lo, hi);
      // Σ_i y_i b_ij = ∫ w N_j with w = Σ_i y_i λ_i (dual: the weights of
      // ψ): eight sums per piece
      T LA[4], LG[4][3], b8[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) b8[j] = T(0);
      double vol6 = 0.0;
      const bool ok = clip_fan_local<T, MAXV>(
          P, G, lo, hi, LA, LG, vol6, [&](const T (&y)[4][3], double det) {
            subtet_quad<T>(y, T(det), [&](T px, T py, T pz, T w) {
              T wv = T(0);
#pragma unroll
              for (int i = 0; i < 4; ++i)
                wv += zl[i] * (LA[i] + LG[i][0] * px + LG[i][1] * py + LG[i][2] * pz);
              wv *= w;
              const T hx0 = T(1) - px, hy0 = T(1) - py, hz0 = T(1) - pz;
              const T n00 = hx0 * hy0, n10 = px * hy0, n01 = hx0 * py, n11 = px * py;
              b8[0] += wv * n00 * hz0;
              b8[1] += wv * n10 * hz0;
              b8[2] += wv * n01 * hz0;
              b8[3] += wv * n11 * hz0;
              b8[4] += wv * n00 * pz;
              b8[5] += wv * n10 * pz;
              b8[6] += wv * n01 * pz;
              b8[7] += wv * n11 * pz;
            });
          });
      if (!ok) {
        fail = true;
        continue;
      }
      if (!piece_kept(vol6, lo, hi, G)) continue;
      const T sc = T(-(hi[0] - lo[0]) * (hi[1] - lo[1]) * (hi[2] - lo[2]) / 6.0);
#pragma unroll
      for (int j = 0; j < 8; ++j)
        unsafeAtomicAdd(out + corner_node(ci, j, NX, NY), T(alpha * double(sc * b8[j])));
    }
  }
  const uint64_t fm = ballot64(fail);
  if (lane == 0 && fm) atomicOr(flags, kFlagCapacity);
}

template <typename T, int MAXV>
__global__ __launch_bounds__(kWave) void k_mf_tet_shape(
    TcList lst, int64_t n_t, int64_t n_v, const CellRange* __restrict__ rng,
    const double* __restrict__ tetrec, const int32_t* __restrict__ tets,
    const double* __restrict__ lat, LatDesc ld, const T* __restrict__ z, const T* u0,
    const T* u1, const T* u2, int dual, double* __restrict__ pgt, unsigned* flags) {
  __shared__ double sx[MAXV * kWave], sy[MAXV * kWave], sz[MAXV * kWave];
  __shared__ uint32_t snb[MAXV * kWave];
  const int lane = threadIdx.x;
  const PolyView P{sx + lane, sy + lane, sz + lane, snb + lane, kWave, (1u << MAXV) - 1u};
  bool fail = false;
  ITEM_LOOP(lst, w) {
    double acc[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = 0.0;
    TetCells tc;
    if (tet_cells(w, n_t, rng, tc)) {
      TetGeom G;
      load_tet(tetrec, tc.t, G);
      T zl[4];
      const int4 tv = *reinterpret_cast<const int4*>(tets + 4 * tc.t);
      const int32_t vv[4] = {tv.x, tv.y, tv.z, tv.w};
#pragma unroll
      for (int k = 0; k < 4; ++k) zl[k] = z[int64_t(tc.d) * n_v + vv[k]];
      if (dual) dual_weights_mf<T>(zl);
      const T* u = tc.d == 0 ? u0 : (tc.d == 1 ? u1 : u2);
      const int64_t NX = ld_at(ld.n, tc.d, 0), NY = ld_at(ld.n, tc.d, 1);
      for (int64_t q = 0; q < tc.count; ++q) {
        int ci[3];
        double lo[3], hi[3];
        range_cell(tc.r, q, lat, ld, tc.d, ci, lo, hi);
        T ul[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) ul[j] = u[corner_node(ci, j, NX, NY)];
        T LA[4], LG[4][3], A[12], Bs = T(0);
#pragma unroll
        for (int k = 0; k < 12; ++k) A[k] = T(0);
        double vol6 = 0.0;
        const bool ok = clip_fan_local<T, MAXV>(P, G, lo, hi, LA, LG, vol6,
                                          [&](const T (&y)[4][3], double det) {
                                            subtet_grad<T>(y, T(det), LA, LG, zl, ul, A, Bs);
                                          });
        if (!ok) {
          fail = true;
          continue;
        }
        const double cv = (hi[0] - lo[0]) * (hi[1] - lo[1]) * (hi[2] - lo[2]);
        if (!(vol6 * cv / 6.0 > kDropRel * (fabs(G.det) / 6.0))) continue;
        const double sc = -cv / 6.0;
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int k = 0; k < 3; ++k)
            acc[a * 3 + k] +=
                double(T(sc * (double(A[a * 3 + k]) / (hi[k] - lo[k]) + G.g[a][k] * double(Bs))));
      }
    }
    store_row<12>(pgt + w * 12, acc);
  }
  const uint64_t fm = ballot64(fail);
  if (lane == 0 && fm) atomicOr(flags, kFlagCapacity);
}

// Sort key of (component, tet) w: class · 64 + min(cells, 63).  A cell of
// the range is cut by at most min(n_e − 1, 2) planes of axis e (one where
// the range has two cells, two inside a longer one), so the item's class is
// that of its most-cut cell: <= 3 planes → 0 (10 slots), 4 → 1 (12),
// >= 5 → 2 (16), the classes of the assembly's pair order.
__global__ void k_mf_key(int64_t n_tc, const CellRange* __restrict__ rng,
                         uint8_t* __restrict__ key) {
  const int64_t w = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (w >= n_tc) return;
  const CellRange r = rng[w];
  int cuts = 0;
  int64_t cells = 1;
  for (int e = 0; e < 3; ++e) {
    cuts += min(max(r.n[e] - 1, 0), 2);
    cells *= r.n[e];
  }
  const int cls = cuts <= 3 ? 0 : (cuts == 4 ? 1 : 2);
  key[w] = uint8_t(cls * 64 + int(min<int64_t>(max<int64_t>(cells, 0), 63)));
}

// bounds[k] = first position of class k in the order, bounds[3] = n_tc.
__global__ void k_mf_bounds(const int64_t* __restrict__ starts, int64_t ntiles,
                            int64_t* __restrict__ bounds) {
  const int k = threadIdx.x;
  if (k < 4) bounds[k] = starts[int64_t(64 * k) * ntiles];
}

constexpr int kMfClasses = 3;
constexpr int kMfSlots[kMfClasses] = {10, 12, 16};

// Resident waves of one class kernel: LDS per wave is 28 bytes per slot and
// lane (160 KB per CU), over 256 CUs, a few rounds deep so the tail of
// the walk balances.
inline unsigned class_blocks(int64_t n_tc, int k) {
  const int64_t per_cu = (160 * 1024) / (int64_t(kMfSlots[k]) * 28 * kWave);
  const int64_t want = 256 * per_cu * 4;
  return unsigned(std::max<int64_t>(1, std::min<int64_t>(want, ceil_div(n_tc, kWave))));
}

inline int64_t* class_bounds(ibvt_coupling* c) {
  const size_t ob = (size_t(3 * c->n_tet) * sizeof(int32_t) + 255) & ~size_t(255);
  return reinterpret_cast<int64_t*>(c->order.as<char>() + ob);
}

inline TcList class_list(ibvt_coupling* c, int k) {
  const int64_t* b = class_bounds(c);
  return TcList{c->order.as<int32_t>(), b + k, b + k + 1};
}

// Launch kernel kern<MAXV> for the three slot classes on stream s.
#define IBVT_MF_CLASSES(KERN, T, ...)                                                   \
  do {                                                                                  \
    KERN<T, 10><<<class_blocks(3 * n_t, 0), kWave, 0, s>>>(class_list(c, 0), __VA_ARGS__); \
    KERN<T, 12><<<class_blocks(3 * n_t, 1), kWave, 0, s>>>(class_list(c, 1), __VA_ARGS__); \
    KERN<T, 16><<<class_blocks(3 * n_t, 2), kWave, 0, s>>>(class_list(c, 2), __VA_ARGS__); \
  } while (0)

template <typename T>
int apply_B_typed(ibvt_coupling* c, const void* const x[3], void* y, bool lumped_scale,
                  hipStream_t s) {
  const int64_t n_t = c->n_tet, n_v = c->n_vert;
  T* pt = c->pval.as<T>();  // 3 n_t x 4, sized by the assembly
  ProfScope ps("mf_apply", s);
  if (n_t > 0)
    IBVT_MF_CLASSES(k_mf_tet_apply, T,
        n_t, c->rng.as<CellRange>(), c->tetrec.as<double>(), c->lat.as<double>(), c->ld,
        static_cast<const T*>(x[0]), static_cast<const T*>(x[1]), static_cast<const T*>(x[2]),
        c->dual ? 1 : 0, pt, c->flags_dev.as<unsigned>());
  k_mf_rows<T><<<unsigned(ceil_div(3 * n_v, 256)), 256, 0, s>>>(
      n_v, n_t, 3, c->vt_ptr.as<int64_t>(), c->vt_tet.as<int32_t>(), c->tets.as<int32_t>(), pt,
      lumped_scale ? c->minv.as<T>() : nullptr, static_cast<T*>(y));
  return hip_check(hipGetLastError(), "matrix-free apply launch");
}

template <typename T>
int apply_Bt_typed(ibvt_coupling* c, const void* ys, void* const out[3], double alpha,
                   hipStream_t s) {
  const int64_t n_t = c->n_tet;
  ProfScope ps("mf_spread", s);
  if (n_t > 0)
    IBVT_MF_CLASSES(k_mf_tet_spread, T,
        n_t, c->n_vert, c->rng.as<CellRange>(), c->tetrec.as<double>(), c->tets.as<int32_t>(),
        c->lat.as<double>(), c->ld, static_cast<const T*>(ys), alpha, c->dual ? 1 : 0,
        static_cast<T*>(out[0]), static_cast<T*>(out[1]), static_cast<T*>(out[2]),
        c->flags_dev.as<unsigned>());
  return hip_check(hipGetLastError(), "matrix-free spread launch");
}

template <typename T>
int shape_typed_mf(ibvt_coupling* c, const void* z, const void* const u[3], const void* us,
                   int mass, double alpha, double* gX, hipStream_t s) {
  const int64_t n_t = c->n_tet;
  int st = ensure(c, c->work2, size_t(3 * n_t + 1) * 12 * sizeof(double));
  if (st) return st;
  double* pgt = c->work2.as<double>();
  unsigned* flags = c->flags_dev.as<unsigned>();
  if ((st = hip_check(hipMemsetAsync(flags, 0, sizeof(unsigned), s), "memset"))) return st;
  {
    ProfScope ps("mf_shape", s);
    if (n_t > 0)
      IBVT_MF_CLASSES(k_mf_tet_shape, T,
          n_t, c->n_vert, c->rng.as<CellRange>(), c->tetrec.as<double>(), c->tets.as<int32_t>(),
          c->lat.as<double>(), c->ld, static_cast<const T*>(z), static_cast<const T*>(u[0]),
          static_cast<const T*>(u[1]), static_cast<const T*>(u[2]), c->dual ? 1 : 0, pgt, flags);
  }
  if ((st = hip_check(hipGetLastError(), "matrix-free shape launch"))) return st;
  if ((st = shape_gather(c, pgt, z, us, mass, alpha, gX, c->tetgrad.as<double>(), 12, s)))
    return st;
  return check_flags(c, s);
}

}  // namespace

#undef IBVT_MF_CLASSES
#undef ITEM_LOOP

// The (component, tet) order of the products (slot class, then cell
// count); kept with the coupling until it is freed or reassembled.
int matfree_order(ibvt_coupling* c, hipStream_t s) {
  const int64_t n_tc = 3 * c->n_tet;
  const size_t ob = (size_t(n_tc) * sizeof(int32_t) + 255) & ~size_t(255);
  int st = ensure(c, c->order, ob + 4 * sizeof(int64_t));
  if (st) return st;
  const size_t kb = (size_t(n_tc + 1) + 255) & ~size_t(255);
  if ((st = ensure(c, c->pscan, kb + sort_pass_bytes(std::max<int64_t>(n_tc, 1), 8)))) return st;
  uint8_t* keys = c->pscan.as<uint8_t>();
  void* scratch = c->pscan.as<char>() + kb;
  int64_t* bounds = class_bounds(c);
  if (n_tc == 0)
    return hip_check(hipMemsetAsync(bounds, 0, 4 * sizeof(int64_t), s), "memset");
  k_mf_key<<<unsigned(ceil_div(n_tc, 256)), 256, 0, s>>>(n_tc, c->rng.as<CellRange>(), keys);
  if ((st = hip_check(hipGetLastError(), "matrix-free key launch"))) return st;
  if ((st = order_by_byte_key(c, n_tc, keys, c->order.as<int32_t>(), scratch, s))) return st;
  k_mf_bounds<<<1, kWave, 0, s>>>(sort_digit_starts(scratch, n_tc, 8, 4), sort_tiles(n_tc, 4),
                                  bounds);
  return hip_check(hipGetLastError(), "matrix-free bounds launch");
}

// A piece never needs more than the 16 vertex slots of the re-clipping
// kernels; were a walk to fail, the kernels flag it on the device, and the
// shape gradient (which synchronises) reports it.
int apply_B_matfree(ibvt_coupling* c, const void* const x[3], void* y, bool lumped_scale,
                    hipStream_t s) {
  if (c->precision == IBVT_FP32_MIXED) return apply_B_typed<float>(c, x, y, lumped_scale, s);
  return apply_B_typed<double>(c, x, y, lumped_scale, s);
}

int apply_Bt_matfree(ibvt_coupling* c, const void* ys, void* const out[3], double alpha,
                     hipStream_t s) {
  if (c->precision == IBVT_FP32_MIXED) return apply_Bt_typed<float>(c, ys, out, alpha, s);
  return apply_Bt_typed<double>(c, ys, out, alpha, s);
}

int shape_gradient_matfree(ibvt_coupling* c, const void* z, const void* const u[3],
                           const void* us, int mass, double alpha, double* gX, hipStream_t s) {
  if (c->precision == IBVT_FP32_MIXED)
    return shape_typed_mf<float>(c, z, u, us, mass, alpha, gX, s);
  return shape_typed_mf<double>(c, z, u, us, mass, alpha, gX, s);
}

}  // namespace ibvt
