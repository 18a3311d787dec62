// Per-piece arithmetic of the planar coupling (Q1 quadrilateral lattice x
// P1 triangles): moments of a triangle ∩ cell piece by Green's theorem, and
// the values ∫ λ_i N_j from them.  Everything is __host__ __device__ so that
// it can also be checked on the host.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace ibvt {

constexpr int kTriRec = 8;   // x0 y0 x1 y1 x2 y2 det 0
constexpr int kMom2 = 10;    // moments 1 s t s² st t² s³ s²t st² t³
constexpr int kMom2Pad = 12;

// Adds the boundary integrals ∮ s^(a+1) t^b dt of one directed segment
// (s0, t0) -> (s1, t1) to m (the 1/(a+1) factors are applied once at the
// end).  Along the segment the integrand is a polynomial of degree <= 4 in
// the parameter, so the 3-point Gauss–Legendre rule is exact.
template <typename T>
__host__ __device__ __forceinline__ void seg_moments(T s0, T t0, T s1, T t1, T (&m)[kMom2]) {
  const T ds = s1 - s0, dt = t1 - t0;
  const T gu[3] = {T(0.1127016653792583115), T(0.5), T(0.8872983346207416885)};
  const T gw[3] = {T(5.0 / 18.0), T(8.0 / 18.0), T(5.0 / 18.0)};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const T s = s0 + gu[k] * ds, t = t0 + gu[k] * dt;
    const T w = gw[k] * dt;
    const T ws = w * s, ws2 = ws * s, ws3 = ws2 * s, t2 = t * t;
    m[0] += ws;
    m[1] += ws2;
    m[2] += ws * t;
    m[3] += ws3;
    m[4] += ws2 * t;
    m[5] += ws * t2;
    m[6] += ws3 * s;
    m[7] += ws3 * t;
    m[8] += ws2 * t2;
    m[9] += ws * t2 * t;
  }
}

// Moments of (triangle V, counter-clockwise) ∩ (cell [lo, hi]) in the
// centred unit coordinates s = (x - xc)/hx, t = (y - yc)/hy, and the piece
// area in double (the trapezoid sums of the same segments).
//
// Boundary of the convex piece: the parts of the triangle's edges inside the
// closed cell, and the parts of the cell's sides inside the closed triangle;
// the horizontal sides have dt = 0 and contribute nothing.  Edge parts are
// found by intersecting the edge's parameter interval with the four
// half-planes (distance >= 0 is inside; a cut end is placed exactly on its
// line); side parts by intersecting the side's y interval with the
// triangle's three half-planes.  A triangle edge lying on a vertical cell
// line is taken through the cell side instead, once, and only when the
// triangle lies on the cell's side of that line.
template <typename T>
__host__ __device__ inline void piece_moments2(const double (&V)[3][2], const double lo[2], const double hi[2],
                               T (&m)[kMom2], double& area_unit) {
  const double xc = 0.5 * (lo[0] + hi[0]), yc = 0.5 * (lo[1] + hi[1]);
  const double ihx = 1.0 / (hi[0] - lo[0]), ihy = 1.0 / (hi[1] - lo[1]);
#pragma unroll
  for (int k = 0; k < kMom2; ++k) m[k] = T(0);
  area_unit = 0.0;
  auto local_s = [&](double x, int snap) {
    return snap == 0 ? -0.5 : (snap == 1 ? 0.5 : (x - xc) * ihx);
  };
  auto local_t = [&](double y, int snap) {
    return snap == 2 ? -0.5 : (snap == 3 ? 0.5 : (y - yc) * ihy);
  };
  // triangle edges clipped to the closed cell
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    const double px = V[e][0], py = V[e][1];
    const double qx = V[(e + 1) % 3][0], qy = V[(e + 1) % 3][1];
    if (px == qx && (px == lo[0] || px == hi[0])) continue;
    const double fp[4] = {px - lo[0], hi[0] - px, py - lo[1], hi[1] - py};
    const double fq[4] = {qx - lo[0], hi[0] - qx, qy - lo[1], hi[1] - qy};
    double u0 = 0.0, u1 = 1.0;
    int k0 = -1, k1 = -1;
    bool empty = false;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const double a = fp[k], b = fq[k];
      if (a < 0.0 && b < 0.0) {
        empty = true;
      } else if (a < 0.0) {
        const double u = a / (a - b);
        if (u > u0) { u0 = u; k0 = k; }
      } else if (b < 0.0) {
        const double u = a / (a - b);
        if (u < u1) { u1 = u; k1 = k; }
      }
    }
    if (empty || !(u0 < u1)) continue;
    const double x0 = px + u0 * (qx - px), y0 = py + u0 * (qy - py);
    const double x1 = px + u1 * (qx - px), y1 = py + u1 * (qy - py);
    const int sx0 = (k0 == 0 || k0 == 1) ? k0 : -1, sy0 = (k0 == 2 || k0 == 3) ? k0 : -1;
    const int sx1 = (k1 == 0 || k1 == 1) ? k1 : -1, sy1 = (k1 == 2 || k1 == 3) ? k1 : -1;
    const double s0 = local_s(x0, sx0), t0 = local_t(y0, sy0);
    const double s1 = local_s(x1, sx1), t1 = local_t(y1, sy1);
    area_unit += 0.5 * (s0 + s1) * (t1 - t0);
    seg_moments<T>(T(s0), T(t0), T(s1), T(t1), m);
  }
  // the cell's vertical sides clipped to the closed triangle: x = hi (going
  // up, inside is x < hi) and x = lo (going down, inside is x > lo)
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const double c = side == 0 ? hi[0] : lo[0];
    double ylo = lo[1], yhi = hi[1];
    int slo = 2, shi = 3;
    bool empty = false, on_line = false;
    int off_vertex = 0;
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      const double px = V[e][0], py = V[e][1];
      const double qx = V[(e + 1) % 3][0], qy = V[(e + 1) % 3][1];
      // inside (left of p -> q): B (y - py) - D >= 0
      const double B = qx - px, D = (qy - py) * (c - px);
      if (B == 0.0) {
        if (px == c) {
          on_line = true;
          off_vertex = (e + 2) % 3;
        } else if (D > 0.0) {
          empty = true;
        }
      } else {
        const double yb = py + D / B;
        if (B > 0.0) {
          if (yb > ylo) { ylo = yb; slo = -1; }
        } else {
          if (yb < yhi) { yhi = yb; shi = -1; }
        }
      }
    }
    if (on_line) {
      const double xr = V[off_vertex][0];
      if (side == 0 ? !(xr < c) : !(xr > c)) empty = true;
    }
    if (empty || !(ylo < yhi)) continue;
    const double s = side == 0 ? 0.5 : -0.5;
    const double ta = local_t(ylo, slo), tb = local_t(yhi, shi);
    if (side == 0) {
      area_unit += s * (tb - ta);
      seg_moments<T>(T(s), T(ta), T(s), T(tb), m);
    } else {
      area_unit += s * (ta - tb);
      seg_moments<T>(T(s), T(tb), T(s), T(ta), m);
    }
  }
  m[1] *= T(0.5);
  m[3] *= T(1.0 / 3.0);
  m[4] *= T(0.5);
  m[6] *= T(0.25);
  m[7] *= T(1.0 / 3.0);
  m[8] *= T(0.5);
}

// Barycentric coordinates of the point (x, y) in triangle rec (any orientation).
__host__ __device__ __forceinline__ void bary_at(const double (&r)[kTriRec], double x, double y,
                                        double (&l)[3]) {
  const double idet = 1.0 / r[6];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const int i1 = (i + 1) % 3, i2 = (i + 2) % 3;
    l[i] = ((r[2 * i1] - x) * (r[2 * i2 + 1] - y) - (r[2 * i2] - x) * (r[2 * i1 + 1] - y)) * idet;
  }
}

// Hat butterflies: ∫ f N_ab for the four cell corners from the moments
// (F, Fs, Ft, Fst) of f, with N_ab = h_a(s) h_b(t), h_0 = 1/2 - s, h_1 = 1/2 + s.
template <typename T>
__host__ __device__ __forceinline__ void corner_integrals(T F, T Fs, T Ft, T Fst, T (&J)[4]) {
  const T a0 = T(0.5) * F - Fs, a1 = T(0.5) * F + Fs;       // ∫ f h_a
  const T b0 = T(0.5) * Ft - Fst, b1 = T(0.5) * Ft + Fst;   // ∫ f h_a t
  J[0] = T(0.5) * a0 - b0;
  J[1] = T(0.5) * a1 - b1;
  J[2] = T(0.5) * a0 + b0;
  J[3] = T(0.5) * a1 + b1;
}


// The twelve values ∫ λ_i N_j (i*4 + corner) of a piece of triangle r in
// cell [lo, hi] from its moments m; with dual set, the dual multipliers'
// values 4 b_i - Σ_k b_k.
template <typename T>
__host__ __device__ inline void piece_values2(const double (&r)[kTriRec], const double lo[2],
                                              const double hi[2], const T (&m)[kMom2], int dual,
                                              T (&out)[12]) {
  const double hx = hi[0] - lo[0], hy = hi[1] - lo[1];
  double l0[3];
  bary_at(r, 0.5 * (lo[0] + hi[0]), 0.5 * (lo[1] + hi[1]), l0);
  T J1[4], Js[4], Jt[4];
  corner_integrals<T>(m[0], m[1], m[2], m[4], J1);
  corner_integrals<T>(m[1], m[3], m[4], m[7], Js);
  corner_integrals<T>(m[2], m[4], m[5], m[8], Jt);
  const T area_scale = T(hx * hy);
  const double idet = 1.0 / r[6];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const int i1 = (i + 1) % 3, i2 = (i + 2) % 3;
    const T li0 = T(l0[i]);
    const T lis = T((r[2 * i1 + 1] - r[2 * i2 + 1]) * idet * hx);
    const T lit = T((r[2 * i2] - r[2 * i1]) * idet * hy);
#pragma unroll
    for (int j = 0; j < 4; ++j) out[4 * i + j] = area_scale * (li0 * J1[j] + lis * Js[j] + lit * Jt[j]);
  }
  if (dual) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const T sj = out[j] + out[4 + j] + out[8 + j];
#pragma unroll
      for (int i = 0; i < 3; ++i) out[4 * i + j] = T(4) * out[4 * i + j] - sj;
    }
  }
}

// Counter-clockwise vertex order of triangle record r.
__host__ __device__ __forceinline__ void ccw_vertices(const double (&r)[kTriRec], double (&V)[3][2]) {
  V[0][0] = r[0];
  V[0][1] = r[1];
  const bool flip = r[6] < 0.0;
  V[1][0] = flip ? r[4] : r[2];
  V[1][1] = flip ? r[5] : r[3];
  V[2][0] = flip ? r[2] : r[4];
  V[2][1] = flip ? r[3] : r[5];
}

}  // namespace ibvt
