/*
 * FP64 CPU oracle for the mortar coupling in two dimensions: the Q1
 * (bilinear) auxiliary space on a staggered rectilinear grid against a P1
 * triangle mesh, the setting of the paper's 2D experiments (Section 4: the
 * Turek–Hron benchmark and the inertia test, with bilinear hats attached to
 * the fluid grid and linear triangles for the solid).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * GPU library is checked against; the product never links or calls it.
 *
 * What it computes, per candidate (triangle T, velocity component d, lattice
 * cell C) pair:
 *     ∫_{T∩C} λ_i N_j dA
 * for the three P1 hats λ_i of T (Section 2.1) and the four Q1 hats N_j of
 * the cell corners (the auxiliary Lagrangian space of Section 2.3).  Summing
 * pieces over all pairs gives the mortar integral B of Section 2.3 (solid
 * rows i, fluid columns j).
 *
 * Route (chosen to share nothing with the GPU kernels):
 *   - the triangle is clipped as a polygon by the four half-planes of the
 *     cell (Sutherland–Hodgman);
 *   - the clipped convex polygon is split into triangles from its vertex
 *     centroid;
 *   - on each sub-triangle τ the integrand λ_i N_j is a product of three
 *     affine factors (λ_i and one 1D hat per axis), integrated exactly by
 *       ∫_τ f1 f2 f3 = |τ|/60 · Σ_{v∈{0,1,2}^3} (Π_w c_w(v)!) Π_m f_m(y_{v_m}),
 *     the expansion of the product in barycentric monomials together with
 *     ∫_τ λ^α = 2|τ| α! / (|α|+2)!  (c_w(v) = multiplicity of vertex w in v).
 *   No quadrature constants are involved.
 *
 * The shape-derivative terms use the same closed form:
 *   ∂B_ij/∂X_{a,k} = Σ_{T∋a} ∫_T (λ_a λ_i ∂_k N_j + ∂_k λ_a λ_i N_j),
 * where ∂_k N_j on a cell is a constant times the other axis' hat, so every
 * integrand is again a product of three affine factors.
 *
 * Tie rules (the same as the 3D oracle's): a point with signed distance
 * s >= 0 is inside a half-plane; a cut point's coordinate on its line is set
 * to the line value.  Pieces with area <= drop_rel·|T| are reported as not
 * kept (their values are still written).  Zero-area triangles produce no
 * pieces.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MAXP 16

typedef struct { int n; double p[MAXP][2]; } Poly;

static double W27[27];
static int w_ready = 0;

static void init_weights(void) {
  if (w_ready) return;
  static const double fact[4] = {1, 1, 2, 6};
  for (int s = 0; s < 27; ++s) {
    int c[3] = {0, 0, 0};
    c[s % 3]++; c[(s / 3) % 3]++; c[s / 9]++;
    W27[s] = fact[c[0]] * fact[c[1]] * fact[c[2]];
  }
  w_ready = 1;
}

/* ∫_τ f1 f2 f3 / |τ| for affine f_m given by their values at the 3 vertices */
static double mean3(const double* f1, const double* f2, const double* f3) {
  double acc = 0.0;
  for (int s = 0; s < 27; ++s) acc += W27[s] * f1[s % 3] * f2[(s / 3) % 3] * f3[s / 9];
  return acc / 60.0;
}

static double tri_area(const double* p0, const double* p1, const double* p2) {
  return 0.5 * fabs((p1[0] - p0[0]) * (p2[1] - p0[1]) - (p1[1] - p0[1]) * (p2[0] - p0[0]));
}

/* Barycentric coefficients: λ_i(x) = coef[i][0] + coef[i][1..2]·x, from the
 * inverse of the 3x3 matrix with rows (1, x_v, y_v) (Gauss–Jordan). */
static int barycentric(const double P[3][2], double coef[3][3]) {
  double A[3][6];
  for (int r = 0; r < 3; ++r) {
    A[r][0] = 1.0; A[r][1] = P[r][0]; A[r][2] = P[r][1];
    for (int c = 0; c < 3; ++c) A[r][3 + c] = (r == c) ? 1.0 : 0.0;
  }
  for (int col = 0; col < 3; ++col) {
    int piv = col;
    for (int r = col + 1; r < 3; ++r) if (fabs(A[r][col]) > fabs(A[piv][col])) piv = r;
    if (A[piv][col] == 0.0) return -1;
    if (piv != col) for (int c = 0; c < 6; ++c) { double t = A[col][c]; A[col][c] = A[piv][c]; A[piv][c] = t; }
    double d = A[col][col];
    for (int c = 0; c < 6; ++c) A[col][c] /= d;
    for (int r = 0; r < 3; ++r) if (r != col) {
      double f = A[r][col];
      if (f != 0.0) for (int c = 0; c < 6; ++c) A[r][c] -= f * A[col][c];
    }
  }
  /* [1 x y] · inv = I  ⇒  column i of inv gives λ_i's coefficients. */
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k) coef[i][k] = A[k][3 + i];
  return 0;
}

static void push_pt(Poly* Q, const double* p) {
  if (Q->n > 0) {
    const double* q = Q->p[Q->n - 1];
    if (q[0] == p[0] && q[1] == p[1]) return;
  }
  if (Q->n < MAXP) { Q->p[Q->n][0] = p[0]; Q->p[Q->n][1] = p[1]; Q->n++; }
}

/* Keep the half-plane sgn·(x[axis] - c) >= 0 (Sutherland–Hodgman). */
static void clip_halfplane(Poly* P, int axis, double c, double sgn) {
  Poly Q;
  Q.n = 0;
  for (int k = 0; k < P->n; ++k) {
    const double* a = P->p[k];
    const double* b = P->p[(k + 1) % P->n];
    double sa = sgn * (a[axis] - c), sb = sgn * (b[axis] - c);
    if (sa >= 0) push_pt(&Q, a);
    if ((sa >= 0) != (sb >= 0)) {
      const double* pin = (sa >= 0) ? a : b;
      const double* pout = (sa >= 0) ? b : a;
      double sin_ = (sa >= 0) ? sa : sb, sout = (sa >= 0) ? sb : sa;
      double t = sin_ / (sin_ - sout);
      double I[2];
      for (int e = 0; e < 2; ++e) I[e] = pin[e] + t * (pout[e] - pin[e]);
      I[axis] = c;
      push_pt(&Q, I);
    }
  }
  if (Q.n > 1 && Q.p[Q.n - 1][0] == Q.p[0][0] && Q.p[Q.n - 1][1] == Q.p[0][1]) Q.n--;
  if (Q.n < 3) Q.n = 0;
  *P = Q;
}

/* Per-pair integration.  Inputs: triangle vertex coordinates P, barycentric
 * coefficients, cell bounds lo/hi.  Outputs: piece area, 12 values
 * val[i*4 + (a + 2b)] = ∫ λ_i N_ab.  Optional shape terms: with z (3 values:
 * z at the triangle's vertices) and u (4 values at the cell corners), adds
 * G[a*2+k] = Σ_{i,j} z_i u_j ∫ (λ_a λ_i ∂_k N_j + ∂_k λ_a λ_i N_j). */
static void piece(const double P[3][2], const double coef[3][3], const double lo[2],
                  const double hi[2], double* area_out, double* val, const double* z,
                  const double* u, double* G) {
  Poly poly;
  poly.n = 3;
  for (int v = 0; v < 3; ++v) { poly.p[v][0] = P[v][0]; poly.p[v][1] = P[v][1]; }
  for (int e = 0; e < 2 && poly.n > 0; ++e) {
    clip_halfplane(&poly, e, lo[e], +1.0);
    if (poly.n > 0) clip_halfplane(&poly, e, hi[e], -1.0);
  }
  memset(val, 0, 12 * sizeof(double));
  *area_out = 0.0;
  if (poly.n == 0) return;

  double apex[2] = {0, 0};
  for (int k = 0; k < poly.n; ++k) { apex[0] += poly.p[k][0]; apex[1] += poly.p[k][1]; }
  apex[0] /= poly.n;
  apex[1] /= poly.n;

  double h[2] = {hi[0] - lo[0], hi[1] - lo[1]};
  for (int k = 0; k < poly.n; ++k) {
    const double* Y[3] = {apex, poly.p[k], poly.p[(k + 1) % poly.n]};
    double at = tri_area(Y[0], Y[1], Y[2]);
    if (at == 0.0) continue;
    *area_out += at;
    double lam[3][3], hat[2][2][3];
    for (int v = 0; v < 3; ++v) {
      for (int i = 0; i < 3; ++i) lam[i][v] = coef[i][0] + coef[i][1] * Y[v][0] + coef[i][2] * Y[v][1];
      for (int e = 0; e < 2; ++e) {
        hat[e][0][v] = (hi[e] - Y[v][e]) / h[e];
        hat[e][1][v] = (Y[v][e] - lo[e]) / h[e];
      }
    }
    for (int i = 0; i < 3; ++i)
      for (int b = 0; b < 2; ++b)
        for (int a = 0; a < 2; ++a) val[i * 4 + a + 2 * b] += at * mean3(lam[i], hat[0][a], hat[1][b]);
    if (G) {
      double w[3];                       /* w = Σ_i z_i λ_i at the vertices */
      for (int v = 0; v < 3; ++v) {
        w[v] = 0;
        for (int i = 0; i < 3; ++i) w[v] += z[i] * lam[i][v];
      }
      for (int b = 0; b < 2; ++b)
        for (int a = 0; a < 2; ++a) {
          int j = a + 2 * b;
          int ab[2] = {a, b};
          /* ∂_k λ_a · ∫ w N_j */
          double wN = at * mean3(w, hat[0][a], hat[1][b]);
          for (int aa = 0; aa < 3; ++aa)
            for (int k = 0; k < 2; ++k) G[aa * 2 + k] += u[j] * coef[aa][1 + k] * wN;
          /* ∫ λ_a w ∂_k N_j,  ∂_k N_j = ±1/h_k · (the other axis' hat) */
          for (int k = 0; k < 2; ++k) {
            double sgnk = ab[k] ? 1.0 / h[k] : -1.0 / h[k];
            int k1 = 1 - k;
            for (int aa = 0; aa < 3; ++aa) {
              double t = at * mean3(lam[aa], w, hat[k1][ab[k1]]);
              G[aa * 2 + k] += u[j] * sgnk * t;
            }
          }
        }
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Exported entry points (called from oracle/plane.py through ctypes).       */
/* ------------------------------------------------------------------------ */

/* Lattice cells overlapped by the bounding box of each triangle, per
 * velocity component.  lat[d*2+e] holds the n = nlat[d*2+e] node
 * coordinates of component d's lattice along axis e.  For each selected
 * triangle s and component d, writes ranges[(s*2+d)*4 + {0,1}] = first cell
 * index per axis and ranges[(s*2+d)*4 + {2,3}] = number of cells per axis,
 * and counts[s*2+d] = their product.  Returns 0, or -2 if a box leaves a
 * lattice's node hull. */
int o2_pair_counts(const double* const* lat, const int64_t* nlat, const double* X,
                   const int32_t* tris, const int64_t* subset, int64_t n_sub,
                   int64_t* counts, int32_t* ranges) {
  int status = 0;
  for (int64_t s = 0; s < n_sub; ++s) {
    int64_t t = subset[s];
    double mn[2], mx[2];
    for (int e = 0; e < 2; ++e) { mn[e] = INFINITY; mx[e] = -INFINITY; }
    for (int v = 0; v < 3; ++v)
      for (int e = 0; e < 2; ++e) {
        double x = X[2 * (int64_t)tris[3 * t + v] + e];
        if (x < mn[e]) mn[e] = x;
        if (x > mx[e]) mx[e] = x;
      }
    for (int d = 0; d < 2; ++d) {
      int64_t cnt = 1;
      for (int e = 0; e < 2; ++e) {
        const double* L = lat[d * 2 + e];
        int64_t n = nlat[d * 2 + e];
        if (mn[e] < L[0] || mx[e] > L[n - 1]) { status = -2; cnt = 0; break; }
        int64_t lo = 0;                      /* largest k with L[k] <= mn */
        for (int64_t k = 0; k < n; ++k) if (L[k] <= mn[e]) lo = k;
        if (lo > n - 2) lo = n - 2;
        int64_t hi = lo;                     /* last cell whose left node < mx */
        for (int64_t k = lo; k < n - 1; ++k) if (L[k] < mx[e]) hi = k;
        ranges[(s * 2 + d) * 4 + e] = (int32_t)lo;
        ranges[(s * 2 + d) * 4 + 2 + e] = (int32_t)(hi - lo + 1);
        cnt *= (hi - lo + 1);
      }
      counts[s * 2 + d] = cnt;
    }
  }
  return status;
}

/* Integrate every candidate pair.  offsets[s*2+d] is the first pair index of
 * (selected triangle s, component d).  For pair p:
 *   vals[p*12 + i*4 + corner], areas[p] (piece area), keep[p]
 *   (area > drop_rel·|T|), cellidx[p*2 + e] (cell index per axis).
 * With z (2 x n_vert, row-major by component), u (2 fluid arrays, x fastest)
 * and G non-NULL, also G[p*6 + a*2 + k], the shape-derivative terms of the
 * pair, with w = Σ_i z_i λ_i — or, with dual set, w = Σ_i z_i ψ_i for the
 * dual multipliers ψ_i = 4λ_i − 1 of the triangle, i.e. the same terms with
 * z_i replaced by 4 z_i − Σ_k z_k.  zero_tris counts degenerate triangles.
 * Returns 0. */
int o2_pairs(const double* const* lat, const int64_t* nlat, const double* X, int64_t n_vert,
             const int32_t* tris, const int64_t* subset, int64_t n_sub, const int32_t* ranges,
             const int64_t* offsets, double drop_rel, int nthreads, double* vals, double* areas,
             uint8_t* keep, int32_t* cellidx, const double* z, const double* const* u, double* G,
             int64_t* zero_tris, int dual) {
  init_weights();
  int64_t nz = 0;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : nz)
#endif
  for (int64_t sd = 0; sd < n_sub * 2; ++sd) {
    int64_t s = sd / 2;
    int d = (int)(sd % 2);
    int64_t t = subset[s];
    double P[3][2], coef[3][3];
    for (int v = 0; v < 3; ++v)
      for (int e = 0; e < 2; ++e) P[v][e] = X[2 * (int64_t)tris[3 * t + v] + e];
    double areaT = tri_area(P[0], P[1], P[2]);
    const int32_t* r = ranges + sd * 4;
    int64_t base = offsets[sd];
    int64_t ncell = (int64_t)r[2] * r[3];
    int degenerate = (areaT == 0.0) || barycentric(P, coef) != 0;
    if (degenerate && d == 0) nz += 1;
    double zl[3] = {0, 0, 0};
    if (z) for (int v = 0; v < 3; ++v) zl[v] = z[(int64_t)d * n_vert + tris[3 * t + v]];
    if (z && dual) {
      double zsum = zl[0] + zl[1] + zl[2];
      for (int v = 0; v < 3; ++v) zl[v] = 4.0 * zl[v] - zsum;
    }
    for (int64_t q = 0; q < ncell; ++q) {
      int64_t p = base + q;
      int ci[2] = {r[0] + (int)(q % r[2]), r[1] + (int)(q / r[2])};
      for (int e = 0; e < 2; ++e) cellidx[p * 2 + e] = ci[e];
      double lo[2], hi[2];
      for (int e = 0; e < 2; ++e) {
        lo[e] = lat[d * 2 + e][ci[e]];
        hi[e] = lat[d * 2 + e][ci[e] + 1];
      }
      double ul[4];
      double* Gp = NULL;
      if (G) {
        Gp = G + p * 6;
        memset(Gp, 0, 6 * sizeof(double));
        int64_t nx = nlat[d * 2 + 0];
        for (int b = 0; b < 2; ++b)
          for (int a = 0; a < 2; ++a) ul[a + 2 * b] = u[d][(ci[0] + a) + nx * (int64_t)(ci[1] + b)];
      }
      if (degenerate) {
        memset(vals + p * 12, 0, 12 * sizeof(double));
        areas[p] = 0.0;
        keep[p] = 0;
        continue;
      }
      double area;
      piece(P, coef, lo, hi, &area, vals + p * 12, zl, ul, Gp);
      areas[p] = area;
      keep[p] = area > drop_rel * areaT;
    }
  }
  if (zero_tris) *zero_tris = nz;
  return 0;
}

/* Exposed for the closed-form tests: ∫_τ f1 f2 f3 for affine f given by
 * vertex values (3 each), τ with vertices Y (3x2). */
double o2_int3(const double* Y, const double* f1, const double* f2, const double* f3) {
  init_weights();
  return tri_area(Y, Y + 2, Y + 4) * mean3(f1, f2, f3);
}

/* Exposed for the clipping tests: area of triangle P (3x2) ∩ box [lo, hi]. */
double o2_clip_area(const double* P, const double* lo, const double* hi) {
  init_weights();
  double PP[3][2], coef[3][3], val[12], area;
  for (int v = 0; v < 3; ++v) for (int e = 0; e < 2; ++e) PP[v][e] = P[2 * v + e];
  if (barycentric(PP, coef) != 0) return 0.0;
  piece(PP, coef, lo, hi, &area, val, NULL, NULL, NULL);
  return area;
}
