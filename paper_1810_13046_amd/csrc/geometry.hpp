// Tet ∩ cell clipping and exact integration of the mortar products on the
// pieces (Section 2.3, assembly steps (II) and (III): quadrature points in
// the intersection of a solid element with a fluid cell, then the local
// contributions ∫ λ_i N_j).
//
// Clipping keeps the piece as a vertex graph (every vertex has exactly three
// neighbours, listed counter-clockwise seen from outside), the
// representation of Powell & Abel's r3d ("An exact general remeshing scheme
// applied to physically conservative voxelization", J. Comput. Phys. 2015).
// A tet cut by the six planes of a box has at most 10 faces, hence at most
// 2·10 − 4 = 16 vertices; cut points reuse the slots of vertices that leave,
// so 16 slots always suffice.  Signed distances and cut points are double;
// a cut point's coordinate on its plane is set to the plane value, and a
// vertex with distance >= 0 is inside.
//
// Integration: the piece is fanned into sub-tetrahedra from its lowest
// vertex (faces through that vertex are skipped).  The assembly integrates
// the 32 monomial moments of degree <= 4 (no exponent above 3) of each
// sub-tetrahedron with a symmetric 11-point degree-4 rule (subtet_moments),
// from which every integrand λ_i N_j follows; the re-clipping paths (the reverse mode
// without stored moments, the products without stored matrices) integrate
// their degree-4 integrands, already contracted with the fields, directly
// with a symmetric 14-point degree-5 rule (subtet_quad, subtet_grad).
// Coordinates are cell-local
// (ξ = (x − x0)/h ∈ [0, 1]^3), so the Q1 hats are ξ or 1 − ξ per axis and
// float arithmetic keeps its relative precision in the mixed-precision path.
//
// Everything here is __host__ __device__: the storage of the vertex graph
// is a strided view (stride 64 = one slot per lane in LDS on the GPU).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ibvt {

#include "quadrature.inc"

constexpr int kMaxV = 16;
constexpr uint32_t kAllSlots = (1u << kMaxV) - 1u;

__host__ __device__ __forceinline__ int ctz32(uint32_t m) { return __builtin_ctz(m); }
__host__ __device__ __forceinline__ int ctz64(uint64_t m) { return __builtin_ctzll(m); }

__host__ __device__ __forceinline__ int nb_get(uint32_t w, int k) { return (w >> (8 * k)) & 0xff; }
__host__ __device__ __forceinline__ uint32_t nb_set(uint32_t w, int k, int v) {
  return (w & ~(0xffu << (8 * k))) | (uint32_t(v) << (8 * k));
}
__host__ __device__ __forceinline__ uint32_t nb_pack(int a, int b, int c) {
  return uint32_t(a) | (uint32_t(b) << 8) | (uint32_t(c) << 16);
}
__host__ __device__ __forceinline__ int nb_find(uint32_t w, int v) {
  return nb_get(w, 0) == v ? 0 : (nb_get(w, 1) == v ? 1 : 2);
}

// Strided view of one piece's vertex graph (`all` = its usable slots: a
// tet cut by c planes has at most 4 + c faces, hence at most 2(4 + c) − 4
// vertices, and slot reuse never needs more than that).
struct PolyView {
  double* px;
  double* py;
  double* pz;
  uint32_t* pnb;
  int S;
  uint32_t all = kAllSlots;  // mask of the slots this view may use
  __host__ __device__ double& co(int v, int a) const {
    return (a == 0 ? px : (a == 1 ? py : pz))[v * S];
  }
  __host__ __device__ double& x(int v) const { return px[v * S]; }
  __host__ __device__ double& y(int v) const { return py[v * S]; }
  __host__ __device__ double& z(int v) const { return pz[v * S]; }
  __host__ __device__ uint32_t& nb(int v) const { return pnb[v * S]; }
};

// Load a tetrahedron (vertices V, any orientation); `flip` swaps vertices 2
// and 3 so that the stored one is positively oriented.
__host__ __device__ inline uint32_t poly_init_tet(const PolyView& P, const double V[4][3],
                                                  bool flip) {
  for (int v = 0; v < 2; ++v) {
    P.x(v) = V[v][0];
    P.y(v) = V[v][1];
    P.z(v) = V[v][2];
  }
  P.x(2) = flip ? V[3][0] : V[2][0];
  P.y(2) = flip ? V[3][1] : V[2][1];
  P.z(2) = flip ? V[3][2] : V[2][2];
  P.x(3) = flip ? V[2][0] : V[3][0];
  P.y(3) = flip ? V[2][1] : V[3][1];
  P.z(3) = flip ? V[2][2] : V[3][2];
  P.nb(0) = nb_pack(1, 3, 2);
  P.nb(1) = nb_pack(2, 3, 0);
  P.nb(2) = nb_pack(0, 3, 1);
  P.nb(3) = nb_pack(1, 2, 0);
  return 0xFu;
}

// Work counts of the clip (for throughput figures): planes clipped by,
// signed distances evaluated and cut points made.
struct ClipCount {
  uint32_t planes = 0;
  uint32_t dist = 0;
  uint32_t cuts = 0;
};

// sv / den for 0 <= sv <= den, den > 0 (the parameter of a cut point on
// an edge): the hardware reciprocal refined by two Newton steps, within an
// ulp or two of the quotient (device code only).
__device__ __forceinline__ double cut_param(double sv, double den) {
  double r = __builtin_amdgcn_rcp(den);
  r = fma(fma(-den, r, 1.0), r, r);
  r = fma(fma(-den, r, 1.0), r, r);
  return sv * r;
}

// Keep the half-space dist(v) >= 0, dist being the signed distance of the
// point in slot v to the plane; a cut point is placed by interpolation and
// then passed to place(w) (which moves it exactly onto an axis plane, or
// does nothing for a general plane).  `live` is the mask of used slots, all
// below NS.  Returns false if the fixed capacity or a walk bound is
// exceeded.  The distance and adjacency passes run over all NS slots
// (unused ones masked), so their reads are independent of each other.
template <int NS, typename Dist, typename Place>
__host__ __device__ __forceinline__ bool poly_clip_by(const PolyView& P, uint32_t& live,
                                                      Dist&& dist, Place&& place,
                                                      ClipCount* cc) {
  if (cc) {
    cc->planes += 1;
    cc->dist += uint32_t(__builtin_popcount(live));
  }
  uint32_t out = 0;
#pragma unroll
  for (int v = 0; v < NS; ++v) {
    const double s = dist(v);
    if (((live >> v) & 1u) && s < 0.0) out |= 1u << v;
  }
  if (!out) return true;
  if (out == live) {
    live = 0;
    return true;
  }
  const uint32_t in = live & ~out;
  uint32_t adj = 0;  // outside vertices with an inside neighbour
  for (uint32_t m = out; m; m &= m - 1) {
    const int u = ctz32(m);
    const uint32_t w = P.nb(u);
    if (((1u << nb_get(w, 0)) | (1u << nb_get(w, 1)) | (1u << nb_get(w, 2))) & in) adj |= 1u << u;
  }
  // free slots: never used, or outside with no inside neighbour
  uint32_t freem = (~live & P.all) | (out & ~adj);
  uint32_t newm = 0;
  for (uint32_t m = adj; m; m &= m - 1) {
    const int u = ctz32(m);
    const double ux = P.x(u), uy = P.y(u), uz = P.z(u);
    const double su = dist(u);
    const uint32_t unb = P.nb(u);
    bool first = true;
    for (int k = 0; k < 3; ++k) {
      const int v = nb_get(unb, k);
      if (!((in >> v) & 1u)) continue;
      const double vx = P.x(v), vy = P.y(v), vz = P.z(v);
      const double sv = dist(v);
      const double t = cut_param(sv, sv - su);
      int w;
      if (first) {
        w = u;  // v's neighbour entry already names u
        first = false;
      } else {
        if (!freem) return false;
        w = ctz32(freem);
        freem &= freem - 1;
        const uint32_t vw = P.nb(v);
        P.nb(v) = nb_set(vw, nb_find(vw, u), w);
      }
      P.x(w) = vx + t * (ux - vx);
      P.y(w) = vy + t * (uy - vy);
      P.z(w) = vz + t * (uz - vz);
      place(w);
      P.nb(w) = nb_pack(v, v, v);
      newm |= 1u << w;
    }
  }
  // Close the cap: from each new vertex walk around the face on its left
  // until the next new vertex.
  for (uint32_t m = newm; m; m &= m - 1) {
    const int w = ctz32(m);
    int vcur = w;
    int vnext = nb_get(P.nb(w), 0);
    int guard = 0;
    do {
      const uint32_t nw = P.nb(vnext);
      const int np = nb_find(nw, vcur);
      vcur = vnext;
      vnext = nb_get(nw, (np + 1) % 3);
      if (++guard > 3 * kMaxV) return false;
    } while (!((newm >> vcur) & 1u));
    P.nb(w) = nb_set(P.nb(w), 2, vcur);
    P.nb(vcur) = nb_set(P.nb(vcur), 1, w);
  }
  live = in | newm;
  if (cc) cc->cuts += uint32_t(__builtin_popcount(newm));
  return true;
}

// Keep the half-space sgn·(x_a − c) >= 0 (an axis plane; cut points are
// set exactly onto it).
template <int NS = kMaxV>
__host__ __device__ inline bool poly_clip(const PolyView& P, uint32_t& live, int a, double c,
                                          double sgn, ClipCount* cc = nullptr) {
  return poly_clip_by<NS>(
      P, live, [&](int v) { return sgn * (P.co(v, a) - c); }, [&](int w) { P.co(w, a) = c; },
      cc);
}

// Clip by the six planes of the box [lo, hi].  mn/mx bound the original
// tet: the piece never leaves them, so a plane the tet does not straddle is
// skipped, and a box the tet only touches gives an empty piece.
template <int NS = kMaxV>
__host__ __device__ inline bool poly_clip_box(const PolyView& P, uint32_t& live, const double lo[3],
                                              const double hi[3], const double mn[3],
                                              const double mx[3], ClipCount* cc = nullptr) {
  for (int a = 0; a < 3; ++a)
    if (mx[a] <= lo[a] || mn[a] >= hi[a]) {
      live = 0;
      return true;
    }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (live && mn[a] < lo[a] && !poly_clip<NS>(P, live, a, lo[a], 1.0, cc)) return false;
    if (live && mx[a] > hi[a] && !poly_clip<NS>(P, live, a, hi[a], -1.0, cc)) return false;
  }
  return true;
}

// Number of sub-tetrahedra poly_fan will emit: a 3-regular polyhedral graph
// with V vertices has Σ_faces (deg − 2) = 2V − 4; faces through the apex
// are skipped.  Returns -1 if a walk exceeds its bound.
__host__ __device__ inline int poly_fan_count(const PolyView& P, uint32_t live) {
  if (!live) return 0;
  const int apex = ctz32(live);
  int total = 2 * __builtin_popcount(live) - 4;
  const uint32_t aw = P.nb(apex);
  for (int k = 0; k < 3; ++k) {
    int prev = apex, cur = nb_get(aw, k), deg = 1, guard = 0;
    while (cur != apex) {
      const uint32_t cw = P.nb(cur);
      const int nxt = nb_get(cw, (nb_find(cw, prev) + 1) % 3);
      prev = cur;
      cur = nxt;
      ++deg;
      if (++guard > 3 * kMaxV) return -1;
    }
    total -= deg - 2;
  }
  return total;
}

// Call fn(apex, f0, f1, f2) for every sub-tetrahedron of the fan
// decomposition.  Faces are walked with the same rule as the cap closure,
// which traverses every face clockwise seen from outside, so each
// sub-tetrahedron (apex, f0, f1, f2) has a non-positive determinant.
template <typename F>
__host__ __device__ inline bool poly_fan(const PolyView& P, uint32_t live, F&& fn) {
  if (!live) return true;
  const int apex = ctz32(live);
  uint64_t seen = 0;
  for (uint32_t m = live; m; m &= m - 1) {
    const int v = ctz32(m);
    const uint32_t vw = P.nb(v);
    for (int k = 0; k < 3; ++k) {
      if ((seen >> (3 * v + k)) & 1ull) continue;
      // pass 1: mark the face's directed edges, look for the apex
      bool has_apex = (v == apex);
      int prev = v, cur = nb_get(vw, k);
      seen |= 1ull << (3 * v + k);
      int guard = 0;
      while (cur != v) {
        has_apex |= (cur == apex);
        const uint32_t cw = P.nb(cur);
        const int nk = (nb_find(cw, prev) + 1) % 3;
        seen |= 1ull << (3 * cur + nk);
        prev = cur;
        cur = nb_get(cw, nk);
        if (++guard > 3 * kMaxV) return false;
      }
      if (has_apex) continue;
      // pass 2: fan from v
      int f1 = nb_get(vw, k);
      prev = v;
      guard = 0;
      for (;;) {
        const uint32_t cw = P.nb(f1);
        const int f2 = nb_get(cw, (nb_find(cw, prev) + 1) % 3);
        if (f2 == v) break;
        fn(apex, v, f1, f2);
        prev = f1;
        f1 = f2;
        if (++guard > 3 * kMaxV) return false;
      }
    }
  }
  return true;
}

// The 14 points and weights of the symmetric degree-5 rule on the
// sub-tetrahedron with vertices y (cell-local), weights scaled by wscale:
// f(px, py, pz, w) for each point.
template <typename T, typename F>
__host__ __device__ __forceinline__ void subtet_quad(const T y[4][3], T wscale, F&& f) {
  T S[3];
#pragma unroll
  for (int e = 0; e < 3; ++e) S[e] = y[0][e] + y[1][e] + y[2][e] + y[3][e];
  const T a1 = T(kQA1), c1 = T(1.0 - 4.0 * kQA1), w1 = T(kQW1) * wscale;
  const T a2 = T(kQA2), c2 = T(1.0 - 4.0 * kQA2), w2 = T(kQW2) * wscale;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    f(a1 * S[0] + c1 * y[k][0], a1 * S[1] + c1 * y[k][1], a1 * S[2] + c1 * y[k][2], w1);
    f(a2 * S[0] + c2 * y[k][0], a2 * S[1] + c2 * y[k][1], a2 * S[2] + c2 * y[k][2], w2);
  }
  const T pb = T(2.0 * kQB - 0.5), ps = T(0.5 - kQB), w3 = T(kQW3) * wscale;
  const int pk[6] = {0, 0, 0, 1, 1, 2}, pl[6] = {1, 2, 3, 2, 3, 3};
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    const int k = pk[q], l = pl[q];
    f(pb * (y[k][0] + y[l][0]) + ps * S[0], pb * (y[k][1] + y[l][1]) + ps * S[1],
      pb * (y[k][2] + y[l][2]) + ps * S[2], w3);
  }
}

// Shape-derivative integrand on one sub-tetrahedron.  With w = Σ_i z_i λ_i
// (z at the tet's vertices) and U = Σ_j u_j N_j (u at the cell's corners):
//   A[a*3+k] += ∫ λ_a w ∂U/∂ξ_k,   Bs += ∫ w U      (unscaled, cell-local)
template <typename T>
__host__ __device__ __forceinline__ void grad_point(T px, T py, T pz, T wq, const T LA[4],
                                                    const T LG[4][3], const T zl[4],
                                                    const T ul[8], T A[12], T& Bs) {
  T lam[4];
  T w = T(0);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    lam[i] = LA[i] + LG[i][0] * px + LG[i][1] * py + LG[i][2] * pz;
    w += zl[i] * lam[i];
  }
  const T hx1 = px, hx0 = T(1) - px, hy1 = py, hy0 = T(1) - py, hz1 = pz, hz0 = T(1) - pz;
  // differences along each axis of the corner values (corner = a + 2b + 4c)
  const T dx00 = ul[1] - ul[0], dx10 = ul[3] - ul[2], dx01 = ul[5] - ul[4], dx11 = ul[7] - ul[6];
  const T dy00 = ul[2] - ul[0], dy10 = ul[3] - ul[1], dy01 = ul[6] - ul[4], dy11 = ul[7] - ul[5];
  const T dz00 = ul[4] - ul[0], dz10 = ul[5] - ul[1], dz01 = ul[6] - ul[2], dz11 = ul[7] - ul[3];
  const T gx = (dx00 * hy0 + dx10 * hy1) * hz0 + (dx01 * hy0 + dx11 * hy1) * hz1;
  const T gy = (dy00 * hx0 + dy10 * hx1) * hz0 + (dy01 * hx0 + dy11 * hx1) * hz1;
  const T gz = (dz00 * hx0 + dz10 * hx1) * hy0 + (dz01 * hx0 + dz11 * hx1) * hy1;
  const T u00 = ul[0] + px * dx00, u10 = ul[2] + px * dx10;
  const T u01 = ul[4] + px * dx01, u11 = ul[6] + px * dx11;
  const T U = (u00 * hy0 + u10 * hy1) * hz0 + (u01 * hy0 + u11 * hy1) * hz1;
  const T ww = wq * w;
  Bs += ww * U;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const T t = ww * lam[a];
    A[a * 3 + 0] += t * gx;
    A[a * 3 + 1] += t * gy;
    A[a * 3 + 2] += t * gz;
  }
}

template <typename T>
__host__ __device__ inline void subtet_grad(const T y[4][3], T wscale, const T LA[4],
                                            const T LG[4][3], const T zl[4], const T ul[8],
                                            T A[12], T& Bs) {
  T S[3];
#pragma unroll
  for (int e = 0; e < 3; ++e) S[e] = y[0][e] + y[1][e] + y[2][e] + y[3][e];
  const T a1 = T(kQA1), c1 = T(1.0 - 4.0 * kQA1), w1 = T(kQW1) * wscale;
  const T a2 = T(kQA2), c2 = T(1.0 - 4.0 * kQA2), w2 = T(kQW2) * wscale;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    grad_point<T>(a1 * S[0] + c1 * y[k][0], a1 * S[1] + c1 * y[k][1], a1 * S[2] + c1 * y[k][2],
                  w1, LA, LG, zl, ul, A, Bs);
    grad_point<T>(a2 * S[0] + c2 * y[k][0], a2 * S[1] + c2 * y[k][1], a2 * S[2] + c2 * y[k][2],
                  w2, LA, LG, zl, ul, A, Bs);
  }
  const T pb = T(2.0 * kQB - 0.5), ps = T(0.5 - kQB), w3 = T(kQW3) * wscale;
  const int pk[6] = {0, 0, 0, 1, 1, 2}, pl[6] = {1, 2, 3, 2, 3, 3};
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    const int k = pk[q], l = pl[q];
    grad_point<T>(pb * (y[k][0] + y[l][0]) + ps * S[0], pb * (y[k][1] + y[l][1]) + ps * S[1],
                  pb * (y[k][2] + y[l][2]) + ps * S[2], w3, LA, LG, zl, ul, A, Bs);
  }
}

// ---------------------------------------------------------------------------
// Piece moments.  Every integrand of the transfer and of its shape
// derivative is a polynomial of degree <= 4 on a piece (λ_i N_j, λ_a w ∂_k U,
// w U with w, λ linear and N_j, U trilinear) in which no coordinate has an
// exponent above 3 (a trilinear factor and its derivatives have exponents
// <= 1, the linear or quadratic one <= 2), so the 32 moments
//   M_α = ∫_piece s^α,  s = ξ − (½, ½, ½),  |α| <= 4, α_e <= 3
// (cell-local coordinates centred in the cell, which keeps the
// recombination well conditioned) determine all of them.  Moments are summed
// per sub-tetrahedron with the 11-point degree-4 rule and per piece over its
// fan.
// ---------------------------------------------------------------------------
constexpr int kMom = 32;
constexpr int kMomPad = 32;  // per-pair stride of the moment store (16-byte rows)
constexpr int kMomLds = 36;  // row stride of LDS staging (rows apart in the banks)

struct MomTable {
  int idx[5][5][5];
  constexpr MomTable() : idx{} {
    for (int x = 0; x < 5; ++x)
      for (int y = 0; y < 5; ++y)
        for (int z = 0; z < 5; ++z) idx[x][y][z] = -1;
    int n = 0;
    for (int x = 0; x <= 3; ++x)
      for (int y = 0; y <= 4 - x && y <= 3; ++y)
        for (int z = 0; z <= 4 - x - y && z <= 3; ++z) idx[x][y][z] = n++;
  }
};
constexpr MomTable kMomTable{};
static_assert(kMomTable.idx[3][1][0] == kMom - 1 && kMomTable.idx[4][0][0] == -1 &&
                  kMomTable.idx[0][0][3] == 3,
              "moment table");
// position of s_x^a s_y^b s_z^c (a + b + c <= 4, each <= 3) in the moment vector
__host__ __device__ constexpr int mom_idx(int a, int b, int c) { return kMomTable.idx[a][b][c]; }

// M += w · s^α for every α (the moment order is a, then b, then c ascending)
template <typename T>
__host__ __device__ __forceinline__ void mom_point(T sx, T sy, T sz, T w, T M[kMom]) {
  const T x2 = sx * sx, y2 = sy * sy, z2 = sz * sz;
  const T px[4] = {T(1), sx, x2, x2 * sx};
  const T py[4] = {T(1), sy, y2, y2 * sy};
  const T pz[4] = {T(1), sz, z2, z2 * sz};
  int k = 0;
#pragma unroll
  for (int a = 0; a <= 3; ++a) {
    const T wa = w * px[a];
#pragma unroll
    for (int b = 0; b <= 4 - a && b <= 3; ++b) {
      const T wab = wa * py[b];
#pragma unroll
      for (int c = 0; c <= 4 - a - b && c <= 3; ++c) M[k++] += wab * pz[c];
    }
  }
}

// Adds the unscaled moments of one sub-tetrahedron (vertices y in cell-local
// coordinates, weight scale = its determinant) to M, with the 11-point
// degree-4 rule (exact for the moments, which are of degree <= 4).
template <typename T>
__host__ __device__ inline void subtet_moments(const T y[4][3], T wscale, T M[kMom]) {
  T yc[4][3], S[3];
#pragma unroll
  for (int e = 0; e < 3; ++e) {
#pragma unroll
    for (int v = 0; v < 4; ++v) yc[v][e] = y[v][e] - T(0.5);
    S[e] = yc[0][e] + yc[1][e] + yc[2][e] + yc[3][e];
  }
  mom_point<T>(T(0.25) * S[0], T(0.25) * S[1], T(0.25) * S[2], T(kQ4W0) * wscale, M);
  const T a = T(kQ4A), ca = T(1.0 - 4.0 * kQ4A), wa = T(kQ4WA) * wscale;
#pragma unroll
  for (int k = 0; k < 4; ++k)
    mom_point<T>(a * S[0] + ca * yc[k][0], a * S[1] + ca * yc[k][1], a * S[2] + ca * yc[k][2],
                 wa, M);
  const T pb = T(2.0 * kQ4B - 0.5), ps = T(0.5 - kQ4B), wb = T(kQ4WB) * wscale;
  const int pk[6] = {0, 0, 0, 1, 1, 2}, pl[6] = {1, 2, 3, 2, 3, 3};
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    const int k = pk[q], l = pl[q];
    mom_point<T>(pb * (yc[k][0] + yc[l][0]) + ps * S[0], pb * (yc[k][1] + yc[l][1]) + ps * S[1],
                 pb * (yc[k][2] + yc[l][2]) + ps * S[2], wb, M);
  }
}

// Q1 hats in centred coordinates: h_0 = ½ − s, h_1 = ½ + s.  Turns the 8
// values G[a + 2b + 4c] = ∫ s_x^a s_y^b s_z^c f into ∫ h_a h_b h_c f
// (one axis at a time: ∫ h_0 g = ½∫g − ∫ s g, ∫ h_1 g = ½∫g + ∫ s g).
template <typename T>
__host__ __device__ __forceinline__ void hat_butterfly(T G[8]) {
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    const int st = 1 << e;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if (j & st) continue;
      const T g0 = G[j], g1 = G[j + st];
      G[j] = T(0.5) * g0 - g1;
      G[j + st] = T(0.5) * g0 + g1;
    }
  }
}

// ∫ λ_i N_j (i = tet vertex, j = cell corner a + 2b + 4c) from the piece's
// moments M (any memory), with λ_i(ξ) = LA[i] + LG[i]·ξ: calls
// put(i, j, value) with the value unscaled like M.
template <typename T, typename F>
__host__ __device__ inline void mom_to_b(const T* M, const T LA[4], const T LG[4][3], F&& put) {
  T Fv[4][8];  // Fv[0][j] = ∫ N_j, Fv[1 + e][j] = ∫ s_e N_j
#pragma unroll
  for (int f = 0; f < 4; ++f) {
#pragma unroll
    for (int j = 0; j < 8; ++j)
      Fv[f][j] = M[mom_idx((j & 1) + (f == 1), ((j >> 1) & 1) + (f == 2), (j >> 2) + (f == 3))];
    hat_butterfly<T>(Fv[f]);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const T lac = LA[i] + T(0.5) * (LG[i][0] + LG[i][1] + LG[i][2]);
#pragma unroll
    for (int j = 0; j < 8; ++j)
      put(i, j, lac * Fv[0][j] + LG[i][0] * Fv[1][j] + LG[i][1] * Fv[2][j] + LG[i][2] * Fv[3][j]);
  }
}

// Shape-derivative integrands of one piece from its moments: with
// w = Σ_i z_i λ_i and U = Σ_j u_j N_j (u at the cell's corners),
//   A[a*3 + k] = ∫ λ_a w ∂U/∂ξ_k,   Bs = ∫ w U      (unscaled like M).
template <typename T>
__host__ __device__ inline void mom_shape(const T M[kMom], const T LA[4], const T LG[4][3],
                                          const T zl[4], const T ul[8], T A[12], T& Bs) {
  T lac[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) lac[i] = LA[i] + T(0.5) * (LG[i][0] + LG[i][1] + LG[i][2]);
  // w = W0 + WG·s
  T W0 = T(0), WG[3] = {T(0), T(0), T(0)};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    W0 += zl[i] * lac[i];
#pragma unroll
    for (int e = 0; e < 3; ++e) WG[e] += zl[i] * LG[i][e];
  }
  // U = Σ_α Uc[α] s^α over α in {0,1}^3 (u_0 h_0 + u_1 h_1 = ½(u_0 + u_1) + (u_1 − u_0) s)
  T Uc[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) Uc[j] = ul[j];
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    const int st = 1 << e;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if (j & st) continue;
      const T u0 = Uc[j], u1 = Uc[j + st];
      Uc[j] = T(0.5) * (u0 + u1);
      Uc[j + st] = u1 - u0;
    }
  }
  Bs = T(0);
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int a = j & 1, b = (j >> 1) & 1, c = j >> 2;
    Bs += Uc[j] * (W0 * M[mom_idx(a, b, c)] + WG[0] * M[mom_idx(a + 1, b, c)] +
                   WG[1] * M[mom_idx(a, b + 1, c)] + WG[2] * M[mom_idx(a, b, c + 1)]);
  }
  // quadratic monomials β: 1, s_x, s_y, s_z, s_x², s_y², s_z², s_x s_y, s_x s_z, s_y s_z
  constexpr int bx[10] = {0, 1, 0, 0, 2, 0, 0, 1, 1, 0};
  constexpr int by[10] = {0, 0, 1, 0, 0, 2, 0, 1, 0, 1};
  constexpr int bz[10] = {0, 0, 0, 1, 0, 0, 2, 0, 1, 1};
  // E_k[β] = Σ_{α: α_k = 1} Uc[α] M[β + α − e_k]  (= ∫ s^β ∂U/∂s_k)
  T E[3][10];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int q = 0; q < 10; ++q) {
      T acc = T(0);
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        if (!((j >> k) & 1)) continue;
        const int a = (j & 1) - (k == 0), b = ((j >> 1) & 1) - (k == 1), c = (j >> 2) - (k == 2);
        acc += Uc[j] * M[mom_idx(bx[q] + a, by[q] + b, bz[q] + c)];
      }
      E[k][q] = acc;
    }
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    // λ_a w = Σ_β q_β s^β
    T qv[10];
    qv[0] = lac[a] * W0;
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      qv[1 + e] = lac[a] * WG[e] + LG[a][e] * W0;
      qv[4 + e] = LG[a][e] * WG[e];
    }
    qv[7] = LG[a][0] * WG[1] + LG[a][1] * WG[0];
    qv[8] = LG[a][0] * WG[2] + LG[a][2] * WG[0];
    qv[9] = LG[a][1] * WG[2] + LG[a][2] * WG[1];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      T acc = T(0);
#pragma unroll
      for (int q = 0; q < 10; ++q) acc += qv[q] * E[k][q];
      A[a * 3 + k] = acc;
    }
  }
}

// Tet data shared by the clip kernels: vertices, orientation, volume and
// barycentric gradients.
struct TetGeom {
  double V[4][3];
  double det;      // e1 · (e2 × e3), e_k = V_k − V_0
  double g[4][3];  // ∇λ_i
  double mn[3], mx[3];  // bounding box
};

// e1 · (e2 × e3) with e_k = V_k − V_0; c receives the cofactor rows
// (e2 × e3, e3 × e1, e1 × e2).
__host__ __device__ inline double tet_det(const double V[4][3], double c[3][3]) {
  double e[3][3];
  for (int k = 0; k < 3; ++k)
    for (int a = 0; a < 3; ++a) e[k][a] = V[k + 1][a] - V[0][a];
  for (int k = 0; k < 3; ++k) {
    const double* p = e[(k + 1) % 3];
    const double* q = e[(k + 2) % 3];
    c[k][0] = p[1] * q[2] - p[2] * q[1];
    c[k][1] = p[2] * q[0] - p[0] * q[2];
    c[k][2] = p[0] * q[1] - p[1] * q[0];
  }
  return e[0][0] * c[0][0] + e[0][1] * c[0][1] + e[0][2] * c[0][2];
}

__host__ __device__ inline void tet_box(TetGeom& G) {
  for (int a = 0; a < 3; ++a) {
    G.mn[a] = fmin(fmin(G.V[0][a], G.V[1][a]), fmin(G.V[2][a], G.V[3][a]));
    G.mx[a] = fmax(fmax(G.V[0][a], G.V[1][a]), fmax(G.V[2][a], G.V[3][a]));
  }
}

__host__ __device__ inline void tet_geom(TetGeom& G) {
  tet_box(G);
  // cofactor rows: ∇λ_1 = (e2 × e3)/det, ∇λ_2 = (e3 × e1)/det, ∇λ_3 = (e1 × e2)/det
  double c[3][3];
  G.det = tet_det(G.V, c);
  const double inv = (G.det != 0.0) ? 1.0 / G.det : 0.0;
  for (int a = 0; a < 3; ++a) {
    G.g[1][a] = c[0][a] * inv;
    G.g[2][a] = c[1][a] * inv;
    G.g[3][a] = c[2][a] * inv;
    G.g[0][a] = -(G.g[1][a] + G.g[2][a] + G.g[3][a]);
  }
}

// Per-tet record read by every pair of the tet: its four vertices (12
// doubles, 96 bytes; the determinant is recomputed where it is needed).
constexpr int kTetRec = 12;

__host__ __device__ inline void store_tet_rec(const TetGeom& G, double* r) {
  for (int k = 0; k < 4; ++k)
    for (int e = 0; e < 3; ++e) r[3 * k + e] = G.V[k][e];
}

// Vertices, determinant and bounding box from a tet record (gradients unset).
__host__ __device__ inline void load_tet_box(TetGeom& G, const double r[kTetRec]) {
  for (int k = 0; k < 4; ++k)
    for (int e = 0; e < 3; ++e) G.V[k][e] = r[3 * k + e];
  double c[3][3];
  G.det = tet_det(G.V, c);
  tet_box(G);
}

// λ_i in cell-local coordinates: λ_i(ξ) = λ_i(lo) + (∇λ_i ∘ h)·ξ.
template <typename T>
__host__ __device__ inline void cell_lambda(const TetGeom& G, const double lo[3], const double hi[3],
                                            T LA[4], T LG[4][3]) {
  for (int i = 0; i < 4; ++i) {
    double a0 = (i == 0) ? 1.0 : 0.0;
    for (int e = 0; e < 3; ++e) a0 += G.g[i][e] * (lo[e] - G.V[0][e]);
    LA[i] = T(a0);
    for (int e = 0; e < 3; ++e) LG[i][e] = T(G.g[i][e] * (hi[e] - lo[e]));
  }
}

// λ of the tet of record r in the cell-local coordinates of [lo, hi]
// (gradients recomputed from the vertices).
template <typename T>
__host__ __device__ inline void rec_cell_lambda(const double r[kTetRec], const double lo[3],
                                                const double hi[3], T LA[4], T LG[4][3]) {
  TetGeom G;
  for (int k = 0; k < 4; ++k)
    for (int e = 0; e < 3; ++e) G.V[k][e] = r[3 * k + e];
  tet_geom(G);
  cell_lambda<T>(G, lo, hi, LA, LG);
}

// Sub-tetrahedron record of the piece store: its 4 vertices (cell-local),
// kRecord values of type T (whole 16-byte words; the determinant follows
// from the vertices, subtet_det).
constexpr int kRecord = 12;

// Determinant d0 · (d1 × d2), d_k = y_{k+1} − y_0, of a sub-tetrahedron (the
// same expression the clip sums into the piece volume).
template <typename T>
__host__ __device__ __forceinline__ T subtet_det(const T ya[3], const T yv[3], const T y1[3],
                                                 const T y2[3]) {
  const T d0[3] = {yv[0] - ya[0], yv[1] - ya[1], yv[2] - ya[2]};
  const T d1[3] = {y1[0] - ya[0], y1[1] - ya[1], y1[2] - ya[2]};
  const T d2[3] = {y2[0] - ya[0], y2[1] - ya[1], y2[2] - ya[2]};
  return d0[0] * (d1[1] * d2[2] - d1[2] * d2[1]) - d0[1] * (d1[0] * d2[2] - d1[2] * d2[0]) +
         d0[2] * (d1[0] * d2[1] - d1[1] * d2[0]);
}

// Walk the three faces through the apex (the lowest live vertex) once:
// their directed edges are marked in `seen` (they give no sub-tetrahedra),
// and the number of sub-tetrahedra of the fan is returned:
// Σ_faces (deg − 2) = 2V − 4 for a 3-regular polyhedral graph, minus the
// apex faces.  Returns -1 if a walk exceeds its bound.
__host__ __device__ inline int poly_fan_prepare(const PolyView& P, uint32_t live, uint64_t& seen) {
  seen = 0;
  if (!live) return 0;
  const int apex = ctz32(live);
  int total = 2 * __builtin_popcount(live) - 4;
  const uint32_t aw = P.nb(apex);
  for (int k = 0; k < 3; ++k) {
    seen |= 1ull << (3 * apex + k);
    int prev = apex, cur = nb_get(aw, k), deg = 1, guard = 0;
    while (cur != apex) {
      const uint32_t cw = P.nb(cur);
      const int nk = (nb_find(cw, prev) + 1) % 3;
      seen |= 1ull << (3 * cur + nk);
      prev = cur;
      cur = nb_get(cw, nk);
      ++deg;
      if (++guard > 3 * kMaxV) return -1;
    }
    total -= deg - 2;
  }
  return total;
}

// Hand the fan's sub-tetrahedra of a clipped piece to put(k, r) in fan
// order (k = 0, 1, ...; r = the record: cell-local vertices rounded to T);
// vol6 receives the piece's 6·volume in cell-local units (double).  The faces
// not marked in `seen` are walked once each; the apex, the face's first
// vertex and the previous vertex stay in registers, so each sub-tetrahedron
// reads one new vertex.
template <typename T, typename Put>
__host__ __device__ inline bool emit_subtets(const PolyView& P, uint32_t live, uint64_t seen,
                                             const double lo[3], const double hi[3], Put&& put,
                                             double& vol6, int& nsub) {
  vol6 = 0.0;
  nsub = 0;
  if (!live) return true;
  const double ih[3] = {1.0 / (hi[0] - lo[0]), 1.0 / (hi[1] - lo[1]), 1.0 / (hi[2] - lo[2])};
  auto local = [&](int v, double y[3]) {
    y[0] = (P.x(v) - lo[0]) * ih[0];
    y[1] = (P.y(v) - lo[1]) * ih[1];
    y[2] = (P.z(v) - lo[2]) * ih[2];
  };
  const int apex = ctz32(live);
  double ya[3];
  local(apex, ya);
  double vsum = 0.0;
  for (uint32_t m = live; m; m &= m - 1) {
    const int v = ctz32(m);
    if (((seen >> (3 * v)) & 7ull) == 7ull) continue;  // all three faces done
    const uint32_t vw = P.nb(v);
    double yv[3];
    local(v, yv);
    for (int k = 0; k < 3; ++k) {
      if ((seen >> (3 * v + k)) & 1ull) continue;
      seen |= 1ull << (3 * v + k);
      int prev = v, f1 = nb_get(vw, k), guard = 0;
      double y1[3];
      local(f1, y1);
      for (;;) {
        const uint32_t cw = P.nb(f1);
        const int nk = (nb_find(cw, prev) + 1) % 3;
        seen |= 1ull << (3 * f1 + nk);
        const int f2 = nb_get(cw, nk);
        if (f2 == v) break;
        double y2[3];
        local(f2, y2);
        vsum += subtet_det<double>(ya, yv, y1, y2);
        T r[kRecord];
        for (int e = 0; e < 3; ++e) {
          r[e] = T(ya[e]);
          r[3 + e] = T(yv[e]);
          r[6 + e] = T(y1[e]);
          r[9 + e] = T(y2[e]);
        }
        put(nsub, r);
        ++nsub;
        prev = f1;
        f1 = f2;
        y1[0] = y2[0];
        y1[1] = y2[1];
        y1[2] = y2[2];
        if (++guard > 3 * kMaxV) return false;
      }
    }
  }
  vol6 = -vsum;
  return true;
}

// Clip tet ∩ box and call sub(y, det) for every sub-tetrahedron (cell-local
// coordinates as T, determinant as double).  Also returns the λ
// coefficients in cell-local coordinates and 6|piece| (cell-local units).
template <typename T, int NS = kMaxV, typename F>
__host__ __device__ inline bool clip_fan_local(const PolyView& P, const TetGeom& G,
                                               const double lo[3], const double hi[3], T LA[4],
                                               T LG[4][3], double& vol6, F&& sub) {
  vol6 = 0.0;
  uint32_t live = poly_init_tet(P, G.V, G.det < 0.0);
  if (!poly_clip_box<NS>(P, live, lo, hi, G.mn, G.mx)) return false;
  const double ih[3] = {1.0 / (hi[0] - lo[0]), 1.0 / (hi[1] - lo[1]), 1.0 / (hi[2] - lo[2])};
  cell_lambda<T>(G, lo, hi, LA, LG);
  if (!live) return true;
  double vsum = 0.0;
  const bool ok = poly_fan(P, live, [&](int q0, int q1, int q2, int q3) {
    const int qs[4] = {q0, q1, q2, q3};
    double yd[4][3];
    for (int v = 0; v < 4; ++v)
      for (int e = 0; e < 3; ++e) yd[v][e] = (P.co(qs[v], e) - lo[e]) * ih[e];
    double d[3][3];
    for (int v = 0; v < 3; ++v)
      for (int e = 0; e < 3; ++e) d[v][e] = yd[v + 1][e] - yd[0][e];
    const double det = d[0][0] * (d[1][1] * d[2][2] - d[1][2] * d[2][1]) -
                       d[0][1] * (d[1][0] * d[2][2] - d[1][2] * d[2][0]) +
                       d[0][2] * (d[1][0] * d[2][1] - d[1][1] * d[2][0]);
    vsum += det;
    T y[4][3];
    for (int v = 0; v < 4; ++v)
      for (int e = 0; e < 3; ++e) y[v][e] = T(yd[v][e]);
    sub(y, det);
  });
  vol6 = -vsum;
  return ok;
}

}  // namespace ibvt
