// Shape derivative of the transfers with respect to the solid vertex
// positions X (reverse mode).
//
// B_ij(X) = Σ_T ∫_T λ_i N_j: the P1 hats λ_i move with the vertices while the
// Q1 hats N_j stay on the grid.  Moving vertex a of T along e_k moves the
// points of T by λ_a e_k, so
//   ∂B_ij/∂X_{a,k} = Σ_{T∋a} ∫_T (λ_a λ_i ∂_k N_j + ∂_k λ_a λ_i N_j)
// and, contracted with z (solid) and u (fluid), with w = Σ z_i λ_i and
// U = Σ u_j N_j (the Q1 interpolant):
//   z^T (∂B/∂X_{a,k}) u = Σ_{T∋a} [ ∫ λ_a w ∂_k U + ∂_k λ_a ∫ w U ].
// The bracket is a polynomial integral of degree <= 4 on each (tet,
// component, cell) piece: k_shape_tet takes it from the piece moments kept
// by the assembly and sums it over the pieces of each (component, tet);
// k_shape_pairs (when no moments are kept) clips every piece again and
// integrates it, and k_pair_sums adds those per (component, tet);
// k_grad_gather sums the per-tet terms per vertex in a fixed order and
// subtracts the mass term  z^T (∂S/∂X) u_s, with ∂|T|/∂X_a = |T| ∇λ_a
// (S consistent: |T|(1+δ_il)/20 per tet; lumped: |T|/4 on the diagonal).
#include "geometry.hpp"
#include "internal.hpp"

namespace ibvt {

namespace {

// Dual multipliers (eq. biorth): w = Σ_i z_i ψ_i with ψ_i = 5λ_i − 1 on the
// tet equals Σ_i (5 z_i − Σ_k z_k) λ_i, so the shape terms keep their form
// with these vertex weights.
template <typename T>
__device__ __forceinline__ void dual_weights(T zl[4]) {
  const T s = zl[0] + zl[1] + zl[2] + zl[3];
#pragma unroll
  for (int k = 0; k < 4; ++k) zl[k] = T(5) * zl[k] - s;
}

template <typename T>
__global__ __launch_bounds__(kWave) void k_shape_pairs(
    int64_t n_pairs, int64_t n_t, int64_t n_v, const int32_t* __restrict__ owner,
    const int64_t* __restrict__ pair_off, const CellRange* __restrict__ rng,
    const uint8_t* __restrict__ keep, const double* __restrict__ X,
    const int32_t* __restrict__ tets, const double* __restrict__ lat, LatDesc ld,
    const T* __restrict__ z, const T* u0, const T* u1, const T* u2, T* __restrict__ pg,
    int dual, unsigned* flags) {
  __shared__ double sx[kMaxV * kWave], sy[kMaxV * kWave], sz[kMaxV * kWave];
  __shared__ uint32_t snb[kMaxV * kWave];
  const int lane = threadIdx.x;
  const PolyView P{sx + lane, sy + lane, sz + lane, snb + lane, kWave};
  bool fail = false;
  for (int64_t p = int64_t(blockIdx.x) * kWave + lane; p < n_pairs;
       p += int64_t(gridDim.x) * kWave) {
    T* out = pg + p * 12;
    if (!keep[p]) {
#pragma unroll
      for (int k = 0; k < 12; ++k) out[k] = T(0);
      continue;
    }
    int d, ci[3];
    int64_t t;
    double lo[3], hi[3];
    pair_cell(p, n_t, owner, pair_off, rng, lat, ld, d, t, ci, lo, hi);
    TetGeom G;
    T zl[4];
    for (int k = 0; k < 4; ++k) {
      const int64_t v = tets[4 * t + k];
      G.V[k][0] = X[3 * v + 0];
      G.V[k][1] = X[3 * v + 1];
      G.V[k][2] = X[3 * v + 2];
      zl[k] = z[int64_t(d) * n_v + v];
    }
    if (dual) dual_weights<T>(zl);
    tet_geom(G);
    const T* u = (d == 0) ? u0 : (d == 1 ? u1 : u2);
    const int64_t NX = ld.n[3 * d + 0], NY = ld.n[3 * d + 1];
    T ul[8];
    for (int c = 0; c < 2; ++c)
      for (int b = 0; b < 2; ++b)
        for (int a = 0; a < 2; ++a)
          ul[a + 2 * b + 4 * c] = u[(ci[0] + a) + NX * ((ci[1] + b) + NY * int64_t(ci[2] + c))];
    T LA[4], LG[4][3], A[12], Bs = T(0);
    for (int k = 0; k < 12; ++k) A[k] = T(0);
    double vol6;
    const bool ok = clip_fan_local<T>(P, G, lo, hi, LA, LG, vol6, [&](const T (&y)[4][3], double det) {
      subtet_grad<T>(y, T(det), LA, LG, zl, ul, A, Bs);
    });
    if (!ok) {
      fail = true;
      for (int k = 0; k < 12; ++k) out[k] = T(0);
      continue;
    }
    const double cv = (hi[0] - lo[0]) * (hi[1] - lo[1]) * (hi[2] - lo[2]);
    const double sc = -cv / 6.0;
    for (int a = 0; a < 4; ++a)
      for (int k = 0; k < 3; ++k)
        out[a * 3 + k] = T(sc * (double(A[a * 3 + k]) / (hi[k] - lo[k]) + G.g[a][k] * double(Bs)));
  }
  const uint64_t fm = ballot64(fail);
  if (lane == 0 && fm) atomicOr(flags, kFlagCapacity);
}

// Pair terms from the stored piece moments (no clipping, no quadrature),
// summed over the pieces of each (component, tet): one lane per (component,
// tet) walks the tet's pairs in cell order, so the tet's geometry, vertex
// weights and lattice are set up once per lane.  The lanes take the items
// in the order of their pair counts (order[]), so the walks of a wave have
// about the same length.  Sums in double to pgt[(d, t)][12] (vertex a,
// axis k at a*3 + k).  With TWO, a second
// contraction (solid weights z2, fluid field v, factor alpha2) is added from
// the same moments: both adjoints' terms in one pass over the store.
template <typename T, bool TWO>
__global__ __launch_bounds__(256) void k_shape_tet(
    int64_t n_t, int64_t n_v, const int64_t* __restrict__ pair_off,
    const CellRange* __restrict__ rng, const uint8_t* __restrict__ keep,
    const T* __restrict__ pmom, const double* __restrict__ tetrec,
    const double* __restrict__ lat, const int32_t* __restrict__ tets, LatDesc ld,
    const T* __restrict__ z, const T* u0, const T* u1, const T* u2, const T* __restrict__ z2,
    const T* v0, const T* v1, const T* v2, double alpha2, const int32_t* __restrict__ order,
    double* __restrict__ pgt, int dual) {
  const int64_t item = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (item >= 3 * n_t) return;
  const int64_t w = order[item];
  const int d = int(w / n_t);
  const int64_t t = w - int64_t(d) * n_t;
  double acc[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = 0.0;
  const int64_t p0 = pair_off[w], p1 = pair_off[w + 1];
  if (p1 > p0) {
    const int4 tv = *reinterpret_cast<const int4*>(tets + 4 * t);
    const T* zd = z + int64_t(d) * n_v;
    T zl[4] = {zd[tv.x], zd[tv.y], zd[tv.z], zd[tv.w]};
    if (dual) dual_weights<T>(zl);
    const T* u = (d == 0) ? u0 : (d == 1 ? u1 : u2);
    T zl2[4] = {T(0), T(0), T(0), T(0)};
    const T* v = (d == 0) ? v0 : (d == 1 ? v1 : v2);
    if (TWO) {
      const T* z2d = z2 + int64_t(d) * n_v;
      zl2[0] = z2d[tv.x];
      zl2[1] = z2d[tv.y];
      zl2[2] = z2d[tv.z];
      zl2[3] = z2d[tv.w];
      if (dual) dual_weights<T>(zl2);
    }
    const int64_t NX = ld.n[3 * d + 0], NY = ld.n[3 * d + 1];
    const double* L0 = lat + ld.off[3 * d + 0];
    const double* L1 = lat + ld.off[3 * d + 1];
    const double* L2 = lat + ld.off[3 * d + 2];
    double rec[kTetRec];
    load_row<kTetRec>(tetrec + t * kTetRec, rec);
    TetGeom G;
    for (int k = 0; k < 4; ++k)
      for (int e = 0; e < 3; ++e) G.V[k][e] = rec[3 * k + e];
    tet_geom(G);
    const CellRange r = rng[w];
    for (int64_t p = p0; p < p1; ++p) {
      if (!keep[p]) continue;
      const uint32_t q = uint32_t(p - p0);
      const uint32_t qy = q / uint32_t(r.n[0]);
      const uint32_t qz = qy / uint32_t(r.n[1]);
      const int ci[3] = {r.lo[0] + int(q - qy * uint32_t(r.n[0])),
                         r.lo[1] + int(qy - qz * uint32_t(r.n[1])), r.lo[2] + int(qz)};
      const double lo[3] = {L0[ci[0]], L1[ci[1]], L2[ci[2]]};
      const double hi[3] = {L0[ci[0] + 1], L1[ci[1] + 1], L2[ci[2] + 1]};
      const int64_t n000 = ci[0] + NX * (ci[1] + NY * int64_t(ci[2]));
      T ul[8];
#pragma unroll
      for (int j = 0; j < 8; ++j)
        ul[j] = u[n000 + (j & 1) + NX * (((j >> 1) & 1) + NY * (j >> 2))];
      T LA[4], LG[4][3];
      cell_lambda<T>(G, lo, hi, LA, LG);
      T M[kMomPad];
      load_row<kMomPad>(pmom + p * kMomPad, M);
      T A[12], Bs;
      mom_shape<T>(M, LA, LG, zl, ul, A, Bs);
      // ∂/∂x_k = (1/h_k) ∂/∂ξ_k; ∇λ_a = (cell-local gradient)/h
      const T sc = T(-(hi[0] - lo[0]) * (hi[1] - lo[1]) * (hi[2] - lo[2]) / 6.0);
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const T ih = T(1.0 / (hi[k] - lo[k]));
#pragma unroll
        for (int a = 0; a < 4; ++a) acc[a * 3 + k] += double(sc * ih * (A[a * 3 + k] + LG[a][k] * Bs));
      }
      if (TWO) {
        T vl[8];
#pragma unroll
        for (int j = 0; j < 8; ++j)
          vl[j] = v[n000 + (j & 1) + NX * (((j >> 1) & 1) + NY * (j >> 2))];
        mom_shape<T>(M, LA, LG, zl2, vl, A, Bs);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const T ih = T(1.0 / (hi[k] - lo[k]));
#pragma unroll
          for (int a = 0; a < 4; ++a)
            acc[a * 3 + k] += alpha2 * double(sc * ih * (A[a * 3 + k] + LG[a][k] * Bs));
        }
      }
    }
  }
  store_row<12>(pgt + w * 12, acc);
}

// Sort key of (component, tet) w: its pair count, clamped to 255.
__global__ void k_tc_key(int64_t n_tc, const int64_t* __restrict__ pair_off,
                         uint8_t* __restrict__ key) {
  const int64_t w = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (w < n_tc) key[w] = uint8_t(min<int64_t>(pair_off[w + 1] - pair_off[w], 255));
}

// Per (component, tet) sums of the per-pair terms of k_shape_pairs.
template <typename T>
__global__ __launch_bounds__(256) void k_pair_sums(int64_t n_tc, const int64_t* __restrict__ pair_off,
                                                   const T* __restrict__ pg,
                                                   double* __restrict__ pgt) {
  const int64_t w = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (w >= n_tc) return;
  double acc[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = 0.0;
  for (int64_t p = pair_off[w]; p < pair_off[w + 1]; ++p)
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] += double(pg[p * 12 + k]);
  store_row<12>(pgt + w * 12, acc);
}

// Mass term coefficient per (component d, tet t): |T| · z_T^T S_T u_s,T with
// S_T = (1 + δ_il)/20 (consistent) or δ_il/4 (lumped) — the derivative of
// z^T S u_s with respect to vertex a of T is this times ∇λ_a.
template <typename T>
__global__ __launch_bounds__(256) void k_mass_coef(int64_t n_t, int64_t n_v,
                                                   const int32_t* __restrict__ tets,
                                                   const double* __restrict__ tetvol,
                                                   const T* __restrict__ z, const T* __restrict__ us,
                                                   int mass, double* __restrict__ out) {
  const int64_t w = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (w >= 3 * n_t) return;
  const int d = int(w / n_t);
  const int64_t t = w - int64_t(d) * n_t;
  const int4 tv = *reinterpret_cast<const int4*>(tets + 4 * t);
  const int32_t vv[4] = {tv.x, tv.y, tv.z, tv.w};
  double zs = 0, uss = 0, zu = 0;
  for (int q = 0; q < 4; ++q) {
    const double zq = double(z[int64_t(d) * n_v + vv[q]]);
    const double uq = double(us[int64_t(d) * n_v + vv[q]]);
    zs += zq;
    uss += uq;
    zu += zq * uq;
  }
  const double sT = (mass == 1) ? (zu + zs * uss) / 20.0 : zu / 4.0;
  out[w] = tetvol[t] * sT;
}

// One wavefront per vertex a: lanes take (incident tet, component) items,
// add the per-tet pair terms and the mass term, then a fixed-order wave
// reduction.  mcoef: per (component, tet) mass coefficients, or null for no
// mass term; tetgrad: ∇λ of every tet (12 doubles at stride gstride).
__global__ __launch_bounds__(256) void k_grad_gather(
    int64_t n_v, int64_t n_t, const int64_t* __restrict__ vt_ptr,
    const int32_t* __restrict__ vt_tet, const int32_t* __restrict__ tets,
    const double* __restrict__ pgt, const double* __restrict__ tetgrad, int gstride,
    const double* __restrict__ mcoef, double alpha, double* __restrict__ gX) {
  const int64_t a = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / kWave;
  const int lane = lane_id();
  if (a >= n_v) return;
  const int64_t beg = vt_ptr[a], end = vt_ptr[a + 1];
  double g[3] = {0, 0, 0};
  for (int64_t it = beg * 3 + lane; it < end * 3; it += kWave) {
    const int64_t k = it / 3;
    const int d = int(it - k * 3);
    const int64_t t = vt_tet[k];
    const int4 tv = *reinterpret_cast<const int4*>(tets + 4 * t);
    const int la = (tv.y == int32_t(a)) ? 1 : (tv.z == int32_t(a)) ? 2 : (tv.w == int32_t(a)) ? 3 : 0;
    const int64_t tc = int64_t(d) * n_t + t;
    for (int e = 0; e < 3; ++e) g[e] += pgt[tc * 12 + la * 3 + e];
    if (mcoef) {
      const double m = mcoef[tc];
      const double* ga = tetgrad + t * gstride + la * 3;
#pragma unroll
      for (int e = 0; e < 3; ++e) g[e] -= m * ga[e];
    }
  }
  for (int e = 0; e < 3; ++e) g[e] = wave_sum(g[e]);
  if (lane == 0)
    for (int e = 0; e < 3; ++e) gX[3 * a + e] += alpha * g[e];
}

// g_X += alpha Σ (per-(component, tet) pair terms pgt − mass term of (z, us)),
// gathered per vertex in a fixed order.
template <typename T>
int gather_typed(ibvt_coupling* c, const double* pgt, const void* z, const void* us, int mass,
                 double alpha, double* gX, const double* grad, int gstride, hipStream_t s) {
  int st;
  double* mcoef = nullptr;
  if (mass >= 0 && c->n_tet > 0) {
    if ((st = ensure(c, c->mcoef, size_t(3 * c->n_tet + 1) * sizeof(double)))) return st;
    mcoef = c->mcoef.as<double>();
    k_mass_coef<T><<<unsigned(ceil_div(3 * c->n_tet, 256)), 256, 0, s>>>(
        c->n_tet, c->n_vert, c->tets.as<int32_t>(), c->tetvol.as<double>(),
        static_cast<const T*>(z), static_cast<const T*>(us), mass, mcoef);
  }
  const unsigned blocks = unsigned(ceil_div(c->n_vert * kWave, 256));
  ProfScope ps_g("grad_gather", s);
  if (c->n_vert > 0)
    k_grad_gather<<<blocks, 256, 0, s>>>(c->n_vert, c->n_tet, c->vt_ptr.as<int64_t>(),
                                         c->vt_tet.as<int32_t>(), c->tets.as<int32_t>(), pgt, grad,
                                         gstride, mcoef, alpha, gX);
  return hip_check(hipGetLastError(), "gather launch");
}

// g_X += alpha (shape terms of (z, u) and the mass term of (z, us)) [+ alpha2
// (shape terms of (z2, v)) when z2 is given; needs the stored moments].
template <typename T>
int shape_typed(ibvt_coupling* c, const void* z, const void* const u[3], const void* us, int mass,
                double alpha, double* gX, hipStream_t s, const void* z2 = nullptr,
                const void* const* v = nullptr, double alpha2 = 0.0) {
  // per (component, tet) sums (double), then the per-pair terms of the
  // re-clipping path
  const size_t tc_bytes = (size_t(3 * c->n_tet + 1) * 12 * sizeof(double) + 255) & ~size_t(255);
  // (stored moments) the sort keys and scratch of the item order
  const int64_t n_tc = 3 * c->n_tet;
  const size_t kb = (size_t(n_tc + 1) + 255) & ~size_t(255);
  const size_t pg_bytes = c->mom_valid ? kb + sort_pass_bytes(std::max<int64_t>(n_tc, 1), 8)
                                       : size_t(c->n_pairs + 1) * 12 * sizeof(T);
  int st = ensure(c, c->work2, tc_bytes + pg_bytes);
  if (st) return st;
  double* pgt = c->work2.as<double>();
  T* pg = reinterpret_cast<T*>(c->work2.as<char>() + tc_bytes);
  unsigned* flags = c->flags_dev.as<unsigned>();
  if ((st = hip_check(hipMemsetAsync(flags, 0, sizeof(unsigned), s), "memset"))) return st;
  if (c->mom_valid && !c->tcorder_valid && n_tc > 0) {
    // once per assembly: the items ordered by their pair counts
    ProfScope ps("shape_order", s);
    if ((st = ensure(c, c->tcorder, size_t(n_tc) * sizeof(int32_t)))) return st;
    uint8_t* keys = c->work2.as<uint8_t>() + tc_bytes;
    k_tc_key<<<unsigned(ceil_div(n_tc, 256)), 256, 0, s>>>(n_tc, c->pair_off.as<int64_t>(), keys);
    if ((st = hip_check(hipGetLastError(), "order key launch"))) return st;
    if ((st = order_by_byte_key(c, n_tc, keys, c->tcorder.as<int32_t>(),
                                c->work2.as<char>() + tc_bytes + kb, s)))
      return st;
    c->tcorder_valid = true;
  }
  if (c->mom_valid) {
    ProfScope ps("shape_moments", s);
    const unsigned nb = unsigned(ceil_div(3 * c->n_tet, 256));
    const T* zz = static_cast<const T*>(z);
    const T* u0 = static_cast<const T*>(u[0]);
    const T* u1 = static_cast<const T*>(u[1]);
    const T* u2 = static_cast<const T*>(u[2]);
    if (c->n_tet > 0 && z2)
      k_shape_tet<T, true><<<nb, 256, 0, s>>>(
          c->n_tet, c->n_vert, c->pair_off.as<int64_t>(), c->rng.as<CellRange>(),
          c->keep.as<uint8_t>(), c->pmom.as<T>(), c->tetrec.as<double>(), c->lat.as<double>(),
          c->tets.as<int32_t>(), c->ld, zz, u0, u1, u2, static_cast<const T*>(z2),
          static_cast<const T*>(v[0]), static_cast<const T*>(v[1]), static_cast<const T*>(v[2]),
          alpha2 / alpha, c->tcorder.as<int32_t>(), pgt, c->dual ? 1 : 0);
    else if (c->n_tet > 0)
      k_shape_tet<T, false><<<nb, 256, 0, s>>>(
          c->n_tet, c->n_vert, c->pair_off.as<int64_t>(), c->rng.as<CellRange>(),
          c->keep.as<uint8_t>(), c->pmom.as<T>(), c->tetrec.as<double>(), c->lat.as<double>(),
          c->tets.as<int32_t>(), c->ld, zz, u0, u1, u2, nullptr, nullptr, nullptr, nullptr, 0.0,
          c->tcorder.as<int32_t>(), pgt, c->dual ? 1 : 0);
  } else {
    const int64_t nb = std::min<int64_t>(ceil_div(c->n_pairs, kWave), int64_t(1) << 22);
    ProfScope ps("shape_pairs", s);
    if (nb > 0)
      k_shape_pairs<T><<<dim3(unsigned(nb)), kWave, 0, s>>>(
        c->n_pairs, c->n_tet, c->n_vert, c->owner.as<int32_t>(), c->pair_off.as<int64_t>(),
        c->rng.as<CellRange>(), c->keep.as<uint8_t>(), c->X.as<double>(), c->tets.as<int32_t>(),
        c->lat.as<double>(), c->ld, static_cast<const T*>(z), static_cast<const T*>(u[0]),
        static_cast<const T*>(u[1]), static_cast<const T*>(u[2]), pg, c->dual ? 1 : 0, flags);
    if (c->n_tet > 0)
      k_pair_sums<T><<<unsigned(ceil_div(3 * c->n_tet, 256)), 256, 0, s>>>(
          3 * c->n_tet, c->pair_off.as<int64_t>(), pg, pgt);
  }
  if ((st = hip_check(hipGetLastError(), "shape launch"))) return st;
  if ((st = gather_typed<T>(c, pgt, z, us, mass, alpha, gX, c->tetgrad.as<double>(), 12, s)))
    return st;
  unsigned f = 0;
  if ((st = hip_check(hipMemcpyAsync(&f, flags, sizeof(f), hipMemcpyDeviceToHost, s), "read")))
    return st;
  if ((st = hip_check(hipStreamSynchronize(s), "sync"))) return st;
  if (f & kFlagCapacity) return set_error(IBVT_E_CAPACITY, "clipped piece exceeded capacity");
  return IBVT_OK;
}

}  // namespace

int shape_gradient(ibvt_coupling* c, const void* z, const void* const u[3], const void* us,
                   int mass, double alpha, double* gX, hipStream_t s) {
  if (c->matrix_free) return shape_gradient_matfree(c, z, u, us, mass, alpha, gX, s);
  if (c->precision == IBVT_FP32_MIXED) return shape_typed<float>(c, z, u, us, mass, alpha, gX, s);
  return shape_typed<double>(c, z, u, us, mass, alpha, gX, s);
}

int shape_gather(ibvt_coupling* c, const double* pgt, const void* z, const void* us, int mass,
                 double alpha, double* gX, const double* grad, int gstride, hipStream_t s) {
  if (c->precision == IBVT_FP32_MIXED)
    return gather_typed<float>(c, pgt, z, us, mass, alpha, gX, grad, gstride, s);
  return gather_typed<double>(c, pgt, z, us, mass, alpha, gX, grad, gstride, s);
}

int shape_gradient_two(ibvt_coupling* c, const void* z, const void* const u[3], const void* us,
                       int mass, const void* z2, const void* const v[3], double alpha2,
                       double* gX, hipStream_t s) {
  if (!c->mom_valid) return set_error(IBVT_E_INVALID, "the piece moments are not stored");
  if (c->precision == IBVT_FP32_MIXED)
    return shape_typed<float>(c, z, u, us, mass, 1.0, gX, s, z2, v, alpha2);
  return shape_typed<double>(c, z, u, us, mass, 1.0, gX, s, z2, v, alpha2);
}

}  // namespace ibvt
