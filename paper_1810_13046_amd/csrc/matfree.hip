// The coupling without stored matrices (IBVT_NO_STORE_B): every product with
// B^d or B^dT, and the shape derivative, clips and integrates the pieces
// again (Section 2.3, steps (II)-(III)) instead of reading an assembled
// matrix, so the handle holds per-tet data and the solid masses only.
//
// One lane per (component d, tet t) walks the tet's cells in index order
// (the order of its pairs in the assembled coupling), clips each cell in
// double (vertex graph in LDS), integrates λ_i N_j on the piece exactly and
// applies the assembly's drop rule (pieces of volume <= 1e-14 |T| are left
// out), then:
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

// Cell q of the range (x fastest) and its box.
__device__ __forceinline__ void range_cell(const CellRange& r, int64_t q, const double* lat,
                                           const LatDesc& ld, int d, int ci[3], double lo[3],
                                           double hi[3]) {
  const int64_t qy = q / r.n[0], qz = qy / r.n[1];
  ci[0] = r.lo[0] + int(q - qy * r.n[0]);
  ci[1] = r.lo[1] + int(qy - qz * r.n[1]);
  ci[2] = r.lo[2] + int(qz);
  for (int e = 0; e < 3; ++e) {
    const double* L = lat + ld.off[3 * d + e];
    lo[e] = L[ci[e]];
    hi[e] = L[ci[e] + 1];
  }
}

// b[i][j] = ∫ λ_i N_j over tet ∩ box (ψ_i = 5λ_i − Σ_k λ_k for the dual
// basis); keep = the piece passes the drop rule.  False on a capacity or
// walk failure.
template <typename T>
__device__ __forceinline__ bool piece_values(const PolyView& P, const TetGeom& G,
                                             const double lo[3], const double hi[3], int dual,
                                             T b[4][8], bool& keep) {
  double vol6 = 0.0;
  T acc[32];
  int nsub = 0;
  keep = false;
  if (!clip_integrate<T>(P, G, lo, hi, vol6, acc, nsub)) return false;
  const double cv = (hi[0] - lo[0]) * (hi[1] - lo[1]) * (hi[2] - lo[2]);
  keep = vol6 * cv / 6.0 > kDropRel * (fabs(G.det) / 6.0);
  const T sc = T(-cv / 6.0);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 8; ++j) b[i][j] = sc * acc[i * 8 + j];
  if (dual) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const T s = b[0][j] + b[1][j] + b[2][j] + b[3][j];
#pragma unroll
      for (int i = 0; i < 4; ++i) b[i][j] = T(5) * b[i][j] - s;
    }
  }
  return true;
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

template <typename T>
__global__ __launch_bounds__(kWave) void k_mf_tet_apply(
    int64_t n_t, const CellRange* __restrict__ rng, const double* __restrict__ tetrec,
    const double* __restrict__ lat, LatDesc ld, const T* x0, const T* x1, const T* x2, int dual,
    T* __restrict__ pt, unsigned* flags) {
  __shared__ double sx[kMaxV * kWave], sy[kMaxV * kWave], sz[kMaxV * kWave];
  __shared__ uint32_t snb[kMaxV * kWave];
  const int lane = threadIdx.x;
  const PolyView P{sx + lane, sy + lane, sz + lane, snb + lane, kWave};
  const int64_t w = int64_t(blockIdx.x) * kWave + lane;
  bool fail = false;
  if (w < 3 * n_t) {
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    TetCells tc;
    if (tet_cells(w, n_t, rng, tc)) {
      TetGeom G;
      load_tet(tetrec, tc.t, G);
      const T* x = tc.d == 0 ? x0 : (tc.d == 1 ? x1 : x2);
      const int64_t NX = ld.n[3 * tc.d + 0], NY = ld.n[3 * tc.d + 1];
      for (int64_t q = 0; q < tc.count; ++q) {
        int ci[3];
        double lo[3], hi[3];
        range_cell(tc.r, q, lat, ld, tc.d, ci, lo, hi);
        T b[4][8];
        bool keep;
        if (!piece_values<T>(P, G, lo, hi, dual, b, keep)) {
          fail = true;
          continue;
        }
        if (!keep) continue;
        T xl[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) xl[j] = x[corner_node(ci, j, NX, NY)];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          T s = T(0);
#pragma unroll
          for (int j = 0; j < 8; ++j) s += b[i][j] * xl[j];
          acc[i] += double(s);
        }
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

template <typename T>
__global__ __launch_bounds__(kWave) void k_mf_tet_spread(
    int64_t n_t, int64_t n_v, const CellRange* __restrict__ rng, const double* __restrict__ tetrec,
    const int32_t* __restrict__ tets, const double* __restrict__ lat, LatDesc ld,
    const T* __restrict__ ys, double alpha, int dual, T* o0, T* o1, T* o2, unsigned* flags) {
  __shared__ double sx[kMaxV * kWave], sy[kMaxV * kWave], sz[kMaxV * kWave];
  __shared__ uint32_t snb[kMaxV * kWave];
  const int lane = threadIdx.x;
  const PolyView P{sx + lane, sy + lane, sz + lane, snb + lane, kWave};
  const int64_t w = int64_t(blockIdx.x) * kWave + lane;
  bool fail = false;
  TetCells tc;
  if (w < 3 * n_t && tet_cells(w, n_t, rng, tc)) {
    TetGeom G;
    load_tet(tetrec, tc.t, G);
    T zl[4];
    const int4 tv = *reinterpret_cast<const int4*>(tets + 4 * tc.t);
    const int32_t vv[4] = {tv.x, tv.y, tv.z, tv.w};
#pragma unroll
    for (int k = 0; k < 4; ++k) zl[k] = ys[int64_t(tc.d) * n_v + vv[k]];
    T* out = tc.d == 0 ? o0 : (tc.d == 1 ? o1 : o2);
    const int64_t NX = ld.n[3 * tc.d + 0], NY = ld.n[3 * tc.d + 1];
    for (int64_t q = 0; q < tc.count; ++q) {
      int ci[3];
      double lo[3], hi[3];
      range_cell(tc.r, q, lat, ld, tc.d, ci, lo, hi);
      T b[4][8];
      bool keep;
      if (!piece_values<T>(P, G, lo, hi, dual, b, keep)) {
        fail = true;
        continue;
      }
      if (!keep) continue;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const T s = b[0][j] * zl[0] + b[1][j] * zl[1] + b[2][j] * zl[2] + b[3][j] * zl[3];
        unsafeAtomicAdd(out + corner_node(ci, j, NX, NY), T(alpha * double(s)));
      }
    }
  }
  const uint64_t fm = ballot64(fail);
  if (lane == 0 && fm) atomicOr(flags, kFlagCapacity);
}

// Dual multipliers: w = Σ_i z_i ψ_i = Σ_i (5 z_i − Σ_k z_k) λ_i.
template <typename T>
__device__ __forceinline__ void dual_weights_mf(T zl[4]) {
  const T s = zl[0] + zl[1] + zl[2] + zl[3];
#pragma unroll
  for (int k = 0; k < 4; ++k) zl[k] = T(5) * zl[k] - s;
}

template <typename T>
__global__ __launch_bounds__(kWave) void k_mf_tet_shape(
    int64_t n_t, int64_t n_v, const CellRange* __restrict__ rng, const double* __restrict__ tetrec,
    const int32_t* __restrict__ tets, const double* __restrict__ lat, LatDesc ld,
    const T* __restrict__ z, const T* u0, const T* u1, const T* u2, int dual,
    double* __restrict__ pgt, unsigned* flags) {
  __shared__ double sx[kMaxV * kWave], sy[kMaxV * kWave], sz[kMaxV * kWave];
  __shared__ uint32_t snb[kMaxV * kWave];
  const int lane = threadIdx.x;
  const PolyView P{sx + lane, sy + lane, sz + lane, snb + lane, kWave};
  const int64_t w = int64_t(blockIdx.x) * kWave + lane;
  bool fail = false;
  if (w < 3 * n_t) {
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
      const int64_t NX = ld.n[3 * tc.d + 0], NY = ld.n[3 * tc.d + 1];
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
        const bool ok = clip_fan_local<T>(P, G, lo, hi, LA, LG, vol6,
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

inline unsigned tet_blocks(int64_t n_t) { return unsigned(ceil_div(3 * n_t > 0 ? 3 * n_t : 1, kWave)); }

template <typename T>
int apply_B_typed(ibvt_coupling* c, const void* const x[3], void* y, bool lumped_scale,
                  hipStream_t s) {
  const int64_t n_t = c->n_tet, n_v = c->n_vert;
  T* pt = c->pval.as<T>();  // 3 n_t x 4, sized by the assembly
  ProfScope ps("mf_apply", s);
  if (n_t > 0)
    k_mf_tet_apply<T><<<tet_blocks(n_t), kWave, 0, s>>>(
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
    k_mf_tet_spread<T><<<tet_blocks(n_t), kWave, 0, s>>>(
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
      k_mf_tet_shape<T><<<tet_blocks(n_t), kWave, 0, s>>>(
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
