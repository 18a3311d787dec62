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

// acc[i*4 + j] = ∫ λ_i μ_j over (solid tet rs) ∩ (fluid tet rf), vol the
// piece volume; P must offer kUSlots slots.  The solid tet is clipped by
// the half-spaces μ_k >= 0 (general planes: cut points are interpolated),
// fanned into sub-tetrahedra, and on each ∫ f g = |τ|/20 (Σ_v f_v g_v +
// Σ_v f_v Σ_v g_v) for the affine factors (coordinates relative to the
// solid tet's vertex 0).  Returns false if a capacity or walk bound fails.
__host__ __device__ inline bool tet_pair_values(const PolyView& P, const double (&rs)[kURec],
                                                const double (&rf)[kURec], double (&acc)[16],
                                                double& vol) {
  for (int k = 0; k < 16; ++k) acc[k] = 0.0;
  vol = 0.0;
  bool fail = false;
  double V[4][3];
  for (int k = 0; k < 4; ++k)
    for (int e = 0; e < 3; ++e) V[k][e] = rs[3 * k + e];
  uint32_t live = poly_init_tet(P, V, rs[24] < 0.0);
  // half-space of the fluid tet opposite its vertex k: μ_k >= 0
  for (int k = 0; k < 4 && live && !fail; ++k) {
    const double* gk = rf + 12 + 3 * k;
    const double d0 = (k == 0) ? 1.0 : 0.0;
    auto dist = [&](int v) {
      return d0 + gk[0] * (P.x(v) - rf[0]) + gk[1] * (P.y(v) - rf[1]) +
             gk[2] * (P.z(v) - rf[2]);
    };
    if (!poly_clip_by<kUSlots>(P, live, dist, [](int) {}, nullptr)) fail = true;
  }
  if (live && !fail) {
    const double dv[3] = {rs[0] - rf[0], rs[1] - rf[1], rs[2] - rf[2]};
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
      vol += vt;
      double lam[4][4], mu[4][4], sl[4], sm[4];
      for (int i = 0; i < 4; ++i) {
        const double* gs = rs + 12 + 3 * i;
        const double* gf = rf + 12 + 3 * i;
        sl[i] = sm[i] = 0.0;
        for (int q = 0; q < 4; ++q) {
          lam[i][q] = (i == 0 ? 1.0 : 0.0) + gs[0] * y[q][0] + gs[1] * y[q][1] + gs[2] * y[q][2];
          mu[i][q] = (i == 0 ? 1.0 : 0.0) + gf[0] * (y[q][0] + dv[0]) +
                     gf[1] * (y[q][1] + dv[1]) + gf[2] * (y[q][2] + dv[2]);
          sl[i] += lam[i][q];
          sm[i] += mu[i][q];
        }
      }
      const double w = vt / 20.0;
      for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
          double t = sl[i] * sm[j];
          for (int q = 0; q < 4; ++q) t += lam[i][q] * mu[j][q];
          acc[4 * i + j] += w * t;
        }
    });
    if (!ok) fail = true;
  }
  return !fail;
}

}  // namespace ibvt
