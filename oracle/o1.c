/*
 * FP64 CPU oracle for the mortar coupling of the L2-projection transfer
 * (Section 2.3, "Variational Transfer: the L2-Projection Approach").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * GPU library is checked against; the product never links or calls it.
 *
 * What it computes, per candidate (tetrahedron T, velocity component d,
 * lattice cell C) pair:
 *     B_ij restricted to the piece T ∩ C:   ∫_{T∩C} λ_i N_j dV
 * for the four P1 hat functions λ_i of T (Section 2.1, Spatial
 * Discretization) and the eight Q1 hat functions N_j of the cell corners
 * (the auxiliary Lagrangian space on the finite-difference grid, Section
 * 2.3).  Summing pieces over all pairs gives the mortar integral B of
 * Section 2.3 (solid rows i, fluid columns j).
 *
 * Route (chosen to share nothing with the GPU kernels):
 *   - the tetrahedron is held as a list of polygonal faces and clipped by
 *     the six half-spaces of the cell, face by face (Sutherland–Hodgman), a
 *     cap polygon closing each cut;
 *   - the clipped convex piece is split into sub-tetrahedra from its vertex
 *     centroid;
 *   - on each sub-tetrahedron τ the integrand λ_i N_j is a product of four
 *     affine factors (λ_i and one 1D hat per axis), integrated exactly by
 *       ∫_τ f1 f2 f3 f4 = |τ|/840 · Σ_{v∈{0..3}^4} (Π_w c_w(v)!) Π_m f_m(y_{v_m}),
 *     the expansion of the product in barycentric monomials together with
 *     ∫_τ λ^α = 6|τ| α! / (|α|+3)!  (c_w(v) = multiplicity of vertex w in v).
 *   No quadrature constants are involved.
 *
 * The shape-derivative terms of the backward pass use the same closed form:
 *   ∂B_ij/∂X_{a,k} = Σ_{T∋a} ∫_T (λ_a λ_i ∂_k N_j + ∂_k λ_a λ_i N_j),
 * where ∂_k N_j on a cell is a constant times two affine hats, so every
 * integrand is again a product of four affine factors.
 *
 * Tie rules: a point with signed distance s >= 0 is inside a half-space;
 * a cut point's coordinate on its plane is set to the plane value.  Pieces
 * with volume <= drop_rel·|T| are reported as not kept (their values are
 * still written).  Zero-volume tetrahedra produce no pieces.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MAXV 40
#define MAXF 20
#define MAXCAP 96

typedef struct { int n; double p[MAXV][3]; } Face;
typedef struct { int nf; Face f[MAXF]; } Polyh;

static double W256[256];
static int w_ready = 0;

static void init_weights(void) {
  if (w_ready) return;
  static const double fact[5] = {1, 1, 2, 6, 24};
  for (int s = 0; s < 256; ++s) {
    int c[4] = {0, 0, 0, 0};
    c[s & 3]++; c[(s >> 2) & 3]++; c[(s >> 4) & 3]++; c[(s >> 6) & 3]++;
    W256[s] = fact[c[0]] * fact[c[1]] * fact[c[2]] * fact[c[3]];
  }
  w_ready = 1;
}

/* ∫_τ f1 f2 f3 f4 / |τ| for affine f_m given by their values at the 4 vertices */
static double mean4(const double* f1, const double* f2, const double* f3, const double* f4) {
  double acc = 0.0;
  for (int s = 0; s < 256; ++s)
    acc += W256[s] * f1[s & 3] * f2[(s >> 2) & 3] * f3[(s >> 4) & 3] * f4[(s >> 6) & 3];
  return acc / 840.0;
}

static double det3(const double* a, const double* b, const double* c) {
  return a[0] * (b[1] * c[2] - b[2] * c[1]) - a[1] * (b[0] * c[2] - b[2] * c[0]) +
         a[2] * (b[0] * c[1] - b[1] * c[0]);
}

static double tet_volume(const double* p0, const double* p1, const double* p2, const double* p3) {
  double a[3], b[3], c[3];
  for (int k = 0; k < 3; ++k) { a[k] = p1[k] - p0[k]; b[k] = p2[k] - p0[k]; c[k] = p3[k] - p0[k]; }
  return fabs(det3(a, b, c)) / 6.0;
}

/* Barycentric coefficients: λ_i(x) = coef[i][0] + coef[i][1..3]·x, from the
 * inverse of the 4x4 matrix with rows (1, x_v, y_v, z_v) (Gauss–Jordan). */
static int barycentric(const double P[4][3], double coef[4][4]) {
  double A[4][8];
  for (int r = 0; r < 4; ++r) {
    A[r][0] = 1.0; A[r][1] = P[r][0]; A[r][2] = P[r][1]; A[r][3] = P[r][2];
    for (int c = 0; c < 4; ++c) A[r][4 + c] = (r == c) ? 1.0 : 0.0;
  }
  for (int col = 0; col < 4; ++col) {
    int piv = col;
    for (int r = col + 1; r < 4; ++r) if (fabs(A[r][col]) > fabs(A[piv][col])) piv = r;
    if (A[piv][col] == 0.0) return -1;
    if (piv != col) for (int c = 0; c < 8; ++c) { double t = A[col][c]; A[col][c] = A[piv][c]; A[piv][c] = t; }
    double d = A[col][col];
    for (int c = 0; c < 8; ++c) A[col][c] /= d;
    for (int r = 0; r < 4; ++r) if (r != col) {
      double f = A[r][col];
      if (f != 0.0) for (int c = 0; c < 8; ++c) A[r][c] -= f * A[col][c];
    }
  }
  /* [1 x y z] · inv = I  ⇒  column i of inv gives λ_i's coefficients. */
  for (int i = 0; i < 4; ++i)
    for (int k = 0; k < 4; ++k) coef[i][k] = A[k][4 + i];
  return 0;
}

static void push_pt(Face* F, const double* p) {
  if (F->n > 0) {
    const double* q = F->p[F->n - 1];
    if (q[0] == p[0] && q[1] == p[1] && q[2] == p[2]) return;
  }
  if (F->n < MAXV) { memcpy(F->p[F->n], p, 3 * sizeof(double)); F->n++; }
}

static int cap_add(double cap[][3], int ncap, const double* p) {
  for (int k = 0; k < ncap; ++k)
    if (cap[k][0] == p[0] && cap[k][1] == p[1] && cap[k][2] == p[2]) return ncap;
  if (ncap < MAXCAP) { memcpy(cap[ncap], p, 3 * sizeof(double)); ncap++; }
  return ncap;
}

/* Keep the half-space sgn·(x[axis] - c) >= 0. */
static void clip_halfspace(Polyh* P, int axis, double c, double sgn) {
  int any_out = 0, any_in = 0;
  for (int f = 0; f < P->nf; ++f)
    for (int k = 0; k < P->f[f].n; ++k) {
      double s = sgn * (P->f[f].p[k][axis] - c);
      if (s < 0) any_out = 1; else any_in = 1;
    }
  if (!any_out) return;
  if (!any_in) { P->nf = 0; return; }

  static __thread Polyh Q;
  double cap[MAXCAP][3];
  int ncap = 0;
  Q.nf = 0;
  for (int f = 0; f < P->nf; ++f) {
    const Face* F = &P->f[f];
    Face G; G.n = 0;
    for (int k = 0; k < F->n; ++k) {
      const double* a = F->p[k];
      const double* b = F->p[(k + 1) % F->n];
      double sa = sgn * (a[axis] - c), sb = sgn * (b[axis] - c);
      if (sa >= 0) {
        push_pt(&G, a);
        if (sa == 0) ncap = cap_add(cap, ncap, a);
      }
      if ((sa >= 0) != (sb >= 0)) {
        /* interpolate from the inside end so both faces sharing the edge
         * produce the identical point */
        const double* pin = (sa >= 0) ? a : b;
        const double* pout = (sa >= 0) ? b : a;
        double sin_ = (sa >= 0) ? sa : sb, sout = (sa >= 0) ? sb : sa;
        double t = sin_ / (sin_ - sout);
        double I[3];
        for (int e = 0; e < 3; ++e) I[e] = pin[e] + t * (pout[e] - pin[e]);
        I[axis] = c;
        push_pt(&G, I);
        ncap = cap_add(cap, ncap, I);
      }
    }
    /* close the loop: drop a last point equal to the first */
    if (G.n > 1) {
      const double* q = G.p[G.n - 1];
      if (q[0] == G.p[0][0] && q[1] == G.p[0][1] && q[2] == G.p[0][2]) G.n--;
    }
    if (G.n >= 3 && Q.nf < MAXF) Q.f[Q.nf++] = G;
  }
  if (ncap >= 3 && Q.nf < MAXF) {
    /* order the cap points by angle about their centroid in the plane */
    int u = (axis + 1) % 3, v = (axis + 2) % 3;
    double cu = 0, cv = 0;
    for (int k = 0; k < ncap; ++k) { cu += cap[k][u]; cv += cap[k][v]; }
    cu /= ncap; cv /= ncap;
    double ang[MAXCAP];
    int ord[MAXCAP];
    for (int k = 0; k < ncap; ++k) { ang[k] = atan2(cap[k][v] - cv, cap[k][u] - cu); ord[k] = k; }
    for (int i = 1; i < ncap; ++i) {       /* insertion sort */
      int o = ord[i], j = i - 1;
      while (j >= 0 && ang[ord[j]] > ang[o]) { ord[j + 1] = ord[j]; --j; }
      ord[j + 1] = o;
    }
    Face G; G.n = 0;
    for (int k = 0; k < ncap; ++k) push_pt(&G, cap[ord[k]]);
    if (G.n >= 3) Q.f[Q.nf++] = G;
  }
  *P = Q;
}

/* Per-pair integration.  Inputs: tet vertex coordinates P, barycentric
 * coefficients, cell bounds lo/hi.  Outputs: piece volume, 32 values
 * val[i*8 + (a + 2b + 4c)] = ∫ λ_i N_abc.  Optional shape terms: with z (4
 * values: z at the tet's vertices) and u (8 values at the cell corners), adds
 * G[a*3+k] = Σ_{i,j} z_i u_j ∫ (λ_a λ_i ∂_k N_j + ∂_k λ_a λ_i N_j). */
static void piece(const double P[4][3], const double coef[4][4], const double lo[3],
                  const double hi[3], double* vol_out, double* val, const double* z,
                  const double* u, double* G) {
  static __thread Polyh poly;
  poly.nf = 4;
  static const int fv[4][3] = {{1, 2, 3}, {0, 3, 2}, {0, 1, 3}, {0, 2, 1}};
  for (int f = 0; f < 4; ++f) {
    poly.f[f].n = 3;
    for (int k = 0; k < 3; ++k) memcpy(poly.f[f].p[k], P[fv[f][k]], 3 * sizeof(double));
  }
  for (int e = 0; e < 3 && poly.nf > 0; ++e) {
    clip_halfspace(&poly, e, lo[e], +1.0);
    if (poly.nf > 0) clip_halfspace(&poly, e, hi[e], -1.0);
  }
  memset(val, 0, 32 * sizeof(double));
  *vol_out = 0.0;
  if (poly.nf == 0) return;

  double apex[3] = {0, 0, 0};
  int cnt = 0;
  for (int f = 0; f < poly.nf; ++f)
    for (int k = 0; k < poly.f[f].n; ++k) {
      for (int e = 0; e < 3; ++e) apex[e] += poly.f[f].p[k][e];
      cnt++;
    }
  for (int e = 0; e < 3; ++e) apex[e] /= cnt;

  double h[3];
  for (int e = 0; e < 3; ++e) h[e] = hi[e] - lo[e];

  for (int f = 0; f < poly.nf; ++f) {
    const Face* F = &poly.f[f];
    for (int k = 1; k + 1 < F->n; ++k) {
      const double* Y[4] = {apex, F->p[0], F->p[k], F->p[k + 1]};
      double vt = tet_volume(Y[0], Y[1], Y[2], Y[3]);
      if (vt == 0.0) continue;
      *vol_out += vt;
      double lam[4][4], hat[3][2][4];
      for (int v = 0; v < 4; ++v) {
        for (int i = 0; i < 4; ++i)
          lam[i][v] = coef[i][0] + coef[i][1] * Y[v][0] + coef[i][2] * Y[v][1] + coef[i][3] * Y[v][2];
        for (int e = 0; e < 3; ++e) {
          hat[e][0][v] = (hi[e] - Y[v][e]) / h[e];
          hat[e][1][v] = (Y[v][e] - lo[e]) / h[e];
        }
      }
      for (int i = 0; i < 4; ++i)
        for (int c = 0; c < 2; ++c)
          for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 2; ++a)
              val[i * 8 + a + 2 * b + 4 * c] +=
                  vt * mean4(lam[i], hat[0][a], hat[1][b], hat[2][c]);
      if (G) {
        double w[4];                       /* w = Σ_i z_i λ_i at the vertices */
        for (int v = 0; v < 4; ++v) {
          w[v] = 0;
          for (int i = 0; i < 4; ++i) w[v] += z[i] * lam[i][v];
        }
        for (int c = 0; c < 2; ++c)
          for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 2; ++a) {
              int j = a + 2 * b + 4 * c;
              int ab[3] = {a, b, c};
              /* ∂_k λ_a · ∫ w N_j */
              double wN = vt * mean4(w, hat[0][a], hat[1][b], hat[2][c]);
              for (int aa = 0; aa < 4; ++aa)
                for (int k = 0; k < 3; ++k) G[aa * 3 + k] += u[j] * coef[aa][1 + k] * wN;
              /* ∫ λ_a w ∂_k N_j,  ∂_k N_j = ±1/h_k · (the other two hats) */
              for (int k = 0; k < 3; ++k) {
                double sgnk = ab[k] ? 1.0 / h[k] : -1.0 / h[k];
                int k1 = (k + 1) % 3, k2 = (k + 2) % 3;
                for (int aa = 0; aa < 4; ++aa) {
                  double t = vt * mean4(lam[aa], w, hat[k1][ab[k1]], hat[k2][ab[k2]]);
                  G[aa * 3 + k] += u[j] * sgnk * t;
                }
              }
            }
      }
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Exported entry points (called from oracle/__init__.py through ctypes).   */
/* ------------------------------------------------------------------------ */

/* Lattice cells overlapped by the bounding box of each tetrahedron, per
 * velocity component (the overlap search of the assembly, Section 2.3).
 * lat[d*3+e] holds the n = nlat[d*3+e] node coordinates of component d's
 * lattice along axis e.  For each selected tet s and component d, writes
 * ranges[(s*3+d)*6 + {0,1,2}] = first cell index per axis and
 * ranges[(s*3+d)*6 + {3,4,5}] = number of cells per axis, and
 * counts[s*3+d] = their product.  Returns 0, or -2 if a box leaves a
 * lattice's node hull. */
int o1_pair_counts(const double* const* lat, const int64_t* nlat, const double* X,
                   const int32_t* tets, const int64_t* subset, int64_t n_sub,
                   int64_t* counts, int32_t* ranges) {
  int status = 0;
  for (int64_t s = 0; s < n_sub; ++s) {
    int64_t t = subset[s];
    double mn[3], mx[3];
    for (int e = 0; e < 3; ++e) { mn[e] = INFINITY; mx[e] = -INFINITY; }
    for (int v = 0; v < 4; ++v)
      for (int e = 0; e < 3; ++e) {
        double x = X[3 * (int64_t)tets[4 * t + v] + e];
        if (x < mn[e]) mn[e] = x;
        if (x > mx[e]) mx[e] = x;
      }
    for (int d = 0; d < 3; ++d) {
      int64_t cnt = 1;
      for (int e = 0; e < 3; ++e) {
        const double* L = lat[d * 3 + e];
        int64_t n = nlat[d * 3 + e];
        if (mn[e] < L[0] || mx[e] > L[n - 1]) { status = -2; cnt = 0; break; }
        int64_t lo = 0;                      /* largest k with L[k] <= mn */
        for (int64_t k = 0; k < n; ++k) if (L[k] <= mn[e]) lo = k;
        if (lo > n - 2) lo = n - 2;
        int64_t hi = lo;                     /* last cell whose left node < mx */
        for (int64_t k = lo; k < n - 1; ++k) if (L[k] < mx[e]) hi = k;
        ranges[(s * 3 + d) * 6 + e] = (int32_t)lo;
        ranges[(s * 3 + d) * 6 + 3 + e] = (int32_t)(hi - lo + 1);
        cnt *= (hi - lo + 1);
      }
      counts[s * 3 + d] = cnt;
    }
  }
  return status;
}

/* Integrate every candidate pair.  offsets[s*3+d] is the first pair index of
 * (selected tet s, component d) (exclusive prefix sum of counts).  For pair p:
 *   vals[p*32 + i*8 + corner], vols[p] (piece volume), keep[p]
 *   (volume > drop_rel·|T|), cellidx[p*3 + e] (cell index per axis).
 * With z (3 x n_vert, row-major by component), u (3 fluid arrays, x fastest,
 * lattice sizes from nlat) and G non-NULL, also G[p*12 + a*3 + k], the
 * shape-derivative terms of the pair, with w = Σ_i z_i λ_i — or, with dual
 * set, w = Σ_i z_i ψ_i for the dual multipliers ψ_i = 5λ_i − 1 of the tet
 * (Section 2.3, eq. biorth), i.e. the same terms with z_i replaced by
 * 5 z_i − Σ_k z_k.  zero_tets counts degenerate tets (they produce no
 * pieces).  Returns 0. */
int o1_pairs(const double* const* lat, const int64_t* nlat, const double* X, int64_t n_vert,
             const int32_t* tets, const int64_t* subset, int64_t n_sub, const int32_t* ranges,
             const int64_t* offsets, double drop_rel, int nthreads, double* vals, double* vols,
             uint8_t* keep, int32_t* cellidx, const double* z, const double* const* u, double* G,
             int64_t* zero_tets, int dual) {
  init_weights();
  int64_t nz = 0;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : nz)
#endif
  for (int64_t sd = 0; sd < n_sub * 3; ++sd) {
    int64_t s = sd / 3;
    int d = (int)(sd % 3);
    int64_t t = subset[s];
    double P[4][3], coef[4][4];
    for (int v = 0; v < 4; ++v)
      for (int e = 0; e < 3; ++e) P[v][e] = X[3 * (int64_t)tets[4 * t + v] + e];
    double volT = tet_volume(P[0], P[1], P[2], P[3]);
    const int32_t* r = ranges + sd * 6;
    int64_t base = offsets[sd];
    int64_t ncell = (int64_t)r[3] * r[4] * r[5];
    int degenerate = (volT == 0.0) || barycentric(P, coef) != 0;
    if (degenerate && d == 0) nz += 1;
    double zl[4] = {0, 0, 0, 0};
    if (z) for (int v = 0; v < 4; ++v) zl[v] = z[(int64_t)d * n_vert + tets[4 * t + v]];
    if (z && dual) {
      double zsum = zl[0] + zl[1] + zl[2] + zl[3];
      for (int v = 0; v < 4; ++v) zl[v] = 5.0 * zl[v] - zsum;
    }
    for (int64_t q = 0; q < ncell; ++q) {
      int64_t p = base + q;
      int ci[3] = {r[0] + (int)(q % r[3]), r[1] + (int)((q / r[3]) % r[4]),
                   r[2] + (int)(q / ((int64_t)r[3] * r[4]))};
      for (int e = 0; e < 3; ++e) cellidx[p * 3 + e] = ci[e];
      double lo[3], hi[3];
      for (int e = 0; e < 3; ++e) {
        lo[e] = lat[d * 3 + e][ci[e]];
        hi[e] = lat[d * 3 + e][ci[e] + 1];
      }
      double ul[8];
      double* Gp = NULL;
      if (G) {
        Gp = G + p * 12;
        memset(Gp, 0, 12 * sizeof(double));
        int64_t nx = nlat[d * 3 + 0], ny = nlat[d * 3 + 1];
        for (int c = 0; c < 2; ++c)
          for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 2; ++a)
              ul[a + 2 * b + 4 * c] = u[d][(ci[0] + a) + nx * ((ci[1] + b) + ny * (int64_t)(ci[2] + c))];
      }
      if (degenerate) {
        memset(vals + p * 32, 0, 32 * sizeof(double));
        vols[p] = 0.0;
        keep[p] = 0;
        continue;
      }
      double vol;
      piece(P, coef, lo, hi, &vol, vals + p * 32, zl, ul, Gp);
      vols[p] = vol;
      keep[p] = vol > drop_rel * volT;
    }
  }
  if (zero_tets) *zero_tets = nz;
  return 0;
}

/* Exposed for the closed-form tests: ∫_τ f1 f2 f3 f4 for affine f given by
 * vertex values (4 each), τ with vertices Y (4x3). */
double o1_int4(const double* Y, const double* f1, const double* f2, const double* f3,
               const double* f4) {
  init_weights();
  return tet_volume(Y, Y + 3, Y + 6, Y + 9) * mean4(f1, f2, f3, f4);
}

/* Exposed for the clipping tests: volume of tet P (4x3) ∩ box [lo, hi]. */
double o1_clip_volume(const double* P, const double* lo, const double* hi) {
  init_weights();
  double PP[4][3], coef[4][4], val[32], vol;
  for (int v = 0; v < 4; ++v) for (int e = 0; e < 3; ++e) PP[v][e] = P[3 * v + e];
  if (barycentric(PP, coef) != 0) return 0.0;
  piece(PP, coef, lo, hi, &vol, val, NULL, NULL, NULL);
  return vol;
}
