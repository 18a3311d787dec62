// Per-pair arithmetic of the coupling with a tetrahedral fluid background:
// a solid tet clipped by the four half-spaces of a fluid tet and the
// products of their P1 hats integrated exactly on the piece.  __host__
// __device__, so that it can also be checked on the host.
#pragma once

#include "geometry.hpp"

namespace ibvt {

// Tet record: vertices (12), ∇λ_0..3 (12), determinant, 3 unused; a hat is
// λ_k(x) = δ_k0 + ∇λ_k·(x − V0).
constexpr int kURec = 28;
// A tet cut by the four planes of another has at most 4 + 4 faces, hence
// at most 2·8 − 4 vertices.
constexpr int kUSlots = 12;
// Per-pair store of ∫ λ_a λ_i (a <= i, 10 values; row stride 12).
constexpr int kULam = 12;

// Index of (a, i), a <= i, in the 10 products ∫ λ_a λ_i.
__host__ __device__ __forceinline__ int lam_index(int a, int i) {
  const int lo = a < i ? a : i, hi = a < i ? i : a;
  return lo * 4 - lo * (lo - 1) / 2 + (hi - lo);
}

// acc[i*4 + j] = ∫ λ_i μ_j over (solid tet rs) ∩ (fluid tet rf), vol the
// piece volume, and with lam also lam[lam_index(a, i)] = ∫ λ_a λ_i (the
// reverse mode's second integral); P must offer kUSlots slots.  The solid
// tet is clipped by the half-spaces μ_k >= 0 (general planes: cut points are
// interpolated) and fanned into sub-tetrahedra.  Every integrand is a
// product of two affine functions, so the piece's moments of degree <= 2
// in y = x − V0 (V0 the solid tet's vertex 0) determine them all: per
// sub-tetrahedron τ, ∫ 1 = |τ|, ∫ y = |τ| (Σ_v y_v)/4 and
// ∫ y_k y_l = |τ|/20 (Σ_v y_vk y_vl + Σ_v y_vk Σ_v y_vl); then with
// λ_i = δ_i0 + g_i·y and μ_j = e_j + h_j·y,
// ∫ λ_i μ_j = δ_i0 e_j M0 + δ_i0 h_j·M1 + e_j g_i·M1 + g_iᵀ M2 h_j.
// Returns false if a capacity or walk bound fails.
__host__ __device__ inline bool tet_pair_values(const PolyView& P, const double (&rs)[kURec],
                                                const double (&rf)[kURec], double (&acc)[16],
                                                double& vol, double* lam = nullptr) {
  for (int k = 0; k < 16; ++k) acc[k] = 0.0;
  if (lam)
    for (int k = 0; k < 10; ++k) lam[k] = 0.0;
  vol = 0.0;
  bool fail = false;
  double V[4][3];
  for (int k = 0; k < 4; ++k)
    for (int e = 0; e < 3; ++e) V[k][e] = rs[3 * k + e];
  uint32_t live = poly_init_tet(P, V, rs[24] < 0.0);
  // half-space of the fluid tet opposite its vertex k: μ_k >= 0 (unrolled, so
  // the record is indexed with constants)
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (live && !fail) {
      const double* gk = rf + 12 + 3 * k;
      const double d0 = (k == 0) ? 1.0 : 0.0;
      auto dist = [&](int v) {
        return d0 + gk[0] * (P.x(v) - rf[0]) + gk[1] * (P.y(v) - rf[1]) +
               gk[2] * (P.z(v) - rf[2]);
      };
      if (!poly_clip_by<kUSlots>(P, live, dist, [](int) {}, nullptr)) fail = true;
    }
  }
  if (!live || fail) return !fail;
  // moments of the piece: M0, M1[3], M2 (xx, xy, xz, yy, yz, zz)
  double m0 = 0.0, m1[3] = {0.0, 0.0, 0.0}, m2[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  const bool ok = poly_fan(P, live, [&](int a, int b, int c, int d) {
    const int vv[4] = {a, b, c, d};
    double y[4][3];
    for (int q = 0; q < 4; ++q) {
      y[q][0] = P.x(vv[q]) - rs[0];
      y[q][1] = P.y(vv[q]) - rs[1];
      y[q][2] = P.z(vv[q]) - rs[2];
    }
    double e1[3], e2[3], e3[3];
    for (int k = 0; k < 3; ++k) {
      e1[k] = y[1][k] - y[0][k];
      e2[k] = y[2][k] - y[0][k];
      e3[k] = y[3][k] - y[0][k];
    }
    const double det = e1[0] * (e2[1] * e3[2] - e2[2] * e3[1]) -
                       e1[1] * (e2[0] * e3[2] - e2[2] * e3[0]) +
                       e1[2] * (e2[0] * e3[1] - e2[1] * e3[0]);
    const double vt = fabs(det) / 6.0;
    double sy[3];
    for (int k = 0; k < 3; ++k) sy[k] = y[0][k] + y[1][k] + y[2][k] + y[3][k];
    m0 += vt;
    for (int k = 0; k < 3; ++k) m1[k] += 0.25 * vt * sy[k];
    const double w = vt / 20.0;
    int o = 0;
    for (int k = 0; k < 3; ++k)
      for (int l = k; l < 3; ++l, ++o) {
        double t = sy[k] * sy[l];
        for (int q = 0; q < 4; ++q) t += y[q][k] * y[q][l];
        m2[o] += w * t;
      }
  });
  if (!ok) return false;
  vol = m0;
  auto quad = [&](const double* g, const double* h) {  // gᵀ M2 h
    return g[0] * (m2[0] * h[0] + m2[1] * h[1] + m2[2] * h[2]) +
           g[1] * (m2[1] * h[0] + m2[3] * h[1] + m2[4] * h[2]) +
           g[2] * (m2[2] * h[0] + m2[4] * h[1] + m2[5] * h[2]);
  };
  auto dot1 = [&](const double* g) { return g[0] * m1[0] + g[1] * m1[1] + g[2] * m1[2]; };
  // μ_j = e_j + h_j·y with e_j = δ_j0 + h_j·(V0s − V0f)
  const double dv[3] = {rs[0] - rf[0], rs[1] - rf[1], rs[2] - rf[2]};
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const double* h = rf + 12 + 3 * j;
    const double ej = (j == 0 ? 1.0 : 0.0) + h[0] * dv[0] + h[1] * dv[1] + h[2] * dv[2];
    const double hm1 = dot1(h);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const double* g = rs + 12 + 3 * i;
      double v = ej * dot1(g) + quad(g, h);
      if (i == 0) v += ej * m0 + hm1;
      acc[4 * i + j] = v;
    }
  }
  if (lam)
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const double* ga = rs + 12 + 3 * a;
#pragma unroll
      for (int i = a; i < 4; ++i) {
        const double* gi = rs + 12 + 3 * i;
        double v = quad(ga, gi);
        if (a == 0) v += dot1(gi);
        if (i == 0) v += dot1(ga);
        if (a == 0 && i == 0) v += m0;
        lam[lam_index(a, i)] = v;
      }
    }
  return true;
}

}  // namespace ibvt
