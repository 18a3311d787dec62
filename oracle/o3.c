/*
 * FP64 CPU oracle for the coupling with an unstructured background: a P1
 * tetrahedral fluid mesh (piecewise affine, the case for which the paper's
 * assembly generates quadrature points, Section 2.3) against the P1
 * tetrahedral solid mesh.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * GPU library is checked against; the product never links or calls it.
 *
 * Per candidate pair (solid tet T, fluid tet F):
 *     ∫_{T∩F} λ_i μ_j dV
 * for the four P1 hats λ_i of T and the four P1 hats μ_j of F (Section 2.3:
 * B_ij = ∫ N_f,j N_fsi,i with the fluid space now P1 on F).
 *
 * Route (chosen to share nothing with the GPU kernels):
 *   - T is held as a list of triangular faces and clipped by the four
 *     half-spaces of F (the side of each face plane that holds F's opposite
 *     vertex), face by face (Sutherland–Hodgman), a cap polygon closing each
 *     cut;
 *   - the clipped convex piece is split into sub-tetrahedra from its vertex
 *     centroid;
 *   - on each sub-tetrahedron τ the integrand is a product of two affine
 *     factors, integrated exactly by
 *       ∫_τ f g = |τ|/20 · (Σ_v f(y_v) g(y_v) + Σ_v f(y_v) · Σ_v g(y_v)),
 *     which follows from ∫_τ λ_a λ_b = |τ|(1 + δ_ab)/20.
 *
 * Tie rule: a point with signed distance s >= 0 is inside.  Pieces with
 * volume <= drop_rel·|T| are reported as not kept (their values are still
 * written).  Zero-volume solid tets produce no pieces.
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

static double det3(const double* a, const double* b, const double* c) {
  return a[0] * (b[1] * c[2] - b[2] * c[1]) - a[1] * (b[0] * c[2] - b[2] * c[0]) +
         a[2] * (b[0] * c[1] - b[1] * c[0]);
}

static double tet_volume(const double* p0, const double* p1, const double* p2, const double* p3) {
  double a[3], b[3], c[3];
  for (int k = 0; k < 3; ++k) { a[k] = p1[k] - p0[k]; b[k] = p2[k] - p0[k]; c[k] = p3[k] - p0[k]; }
  return fabs(det3(a, b, c)) / 6.0;
}

/* Barycentric coefficients λ_i(x) = coef[i][0] + coef[i][1..3]·x from the
 * inverse of the matrix with rows (1, x_v) (Gauss–Jordan, partial pivoting). */
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

/* Keep the half-space nrm·x - c >= 0. */
static void clip_plane(Polyh* P, const double nrm[3], double c) {
  int any_out = 0, any_in = 0;
  for (int f = 0; f < P->nf; ++f)
    for (int k = 0; k < P->f[f].n; ++k) {
      const double* x = P->f[f].p[k];
      double s = nrm[0] * x[0] + nrm[1] * x[1] + nrm[2] * x[2] - c;
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
      double sa = nrm[0] * a[0] + nrm[1] * a[1] + nrm[2] * a[2] - c;
      double sb = nrm[0] * b[0] + nrm[1] * b[1] + nrm[2] * b[2] - c;
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
        push_pt(&G, I);
        ncap = cap_add(cap, ncap, I);
      }
    }
    if (G.n > 1) {
      const double* q = G.p[G.n - 1];
      if (q[0] == G.p[0][0] && q[1] == G.p[0][1] && q[2] == G.p[0][2]) G.n--;
    }
    if (G.n >= 3 && Q.nf < MAXF) Q.f[Q.nf++] = G;
  }
  if (ncap >= 3 && Q.nf < MAXF) {
    /* order the cap points by angle about their centroid, in a basis of
     * the plane */
    double e1[3], e2[3];
    int m = (fabs(nrm[0]) < fabs(nrm[1])) ? ((fabs(nrm[0]) < fabs(nrm[2])) ? 0 : 2)
                                         : ((fabs(nrm[1]) < fabs(nrm[2])) ? 1 : 2);
    double ax[3] = {0, 0, 0};
    ax[m] = 1.0;
    e1[0] = nrm[1] * ax[2] - nrm[2] * ax[1];
    e1[1] = nrm[2] * ax[0] - nrm[0] * ax[2];
    e1[2] = nrm[0] * ax[1] - nrm[1] * ax[0];
    e2[0] = nrm[1] * e1[2] - nrm[2] * e1[1];
    e2[1] = nrm[2] * e1[0] - nrm[0] * e1[2];
    e2[2] = nrm[0] * e1[1] - nrm[1] * e1[0];
    double cen[3] = {0, 0, 0};
    for (int k = 0; k < ncap; ++k) for (int e = 0; e < 3; ++e) cen[e] += cap[k][e];
    for (int e = 0; e < 3; ++e) cen[e] /= ncap;
    double ang[MAXCAP];
    int ord[MAXCAP];
    for (int k = 0; k < ncap; ++k) {
      double d[3] = {cap[k][0] - cen[0], cap[k][1] - cen[1], cap[k][2] - cen[2]};
      ang[k] = atan2(d[0] * e2[0] + d[1] * e2[1] + d[2] * e2[2],
                     d[0] * e1[0] + d[1] * e1[1] + d[2] * e1[2]);
      ord[k] = k;
    }
    for (int i = 1; i < ncap; ++i) {
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

/* ∫_τ f g for affine f, g given at the 4 vertices of τ (volume vt). */
static double int2(double vt, const double* f, const double* g) {
  double fg = 0, sf = 0, sg = 0;
  for (int v = 0; v < 4; ++v) { fg += f[v] * g[v]; sf += f[v]; sg += g[v]; }
  return vt * (fg + sf * sg) / 20.0;
}

/* One pair: solid tet S (vertices, λ coefficients), fluid tet F (vertices,
 * μ coefficients).  val[i*4 + j] = ∫ λ_i μ_j over S ∩ F and, when lam is
 * given, lam[a*4 + i] = ∫ λ_a λ_i over it (the reverse mode's second
 * integral); returns the piece volume. */
static double piece(const double S[4][3], const double ls[4][4], const double F[4][3],
                    const double lf[4][4], double* val, double* lam) {
  static __thread Polyh poly;
  poly.nf = 4;
  static const int fv[4][3] = {{1, 2, 3}, {0, 3, 2}, {0, 1, 3}, {0, 2, 1}};
  for (int f = 0; f < 4; ++f) {
    poly.f[f].n = 3;
    for (int k = 0; k < 3; ++k) memcpy(poly.f[f].p[k], S[fv[f][k]], 3 * sizeof(double));
  }
  /* half-space of F opposite vertex k: μ_k >= 0 */
  for (int k = 0; k < 4 && poly.nf > 0; ++k) {
    double nrm[3] = {lf[k][1], lf[k][2], lf[k][3]};
    clip_plane(&poly, nrm, -lf[k][0]);
  }
  memset(val, 0, 16 * sizeof(double));
  if (lam) memset(lam, 0, 16 * sizeof(double));
  if (poly.nf == 0) return 0.0;
  double apex[3] = {0, 0, 0};
  int cnt = 0;
  for (int f = 0; f < poly.nf; ++f)
    for (int k = 0; k < poly.f[f].n; ++k) {
      for (int e = 0; e < 3; ++e) apex[e] += poly.f[f].p[k][e];
      cnt++;
    }
  for (int e = 0; e < 3; ++e) apex[e] /= cnt;
  double vol = 0.0;
  for (int f = 0; f < poly.nf; ++f) {
    const Face* G = &poly.f[f];
    for (int k = 1; k + 1 < G->n; ++k) {
      const double* Y[4] = {apex, G->p[0], G->p[k], G->p[k + 1]};
      double vt = tet_volume(Y[0], Y[1], Y[2], Y[3]);
      if (vt == 0.0) continue;
      vol += vt;
      double la[4][4], mu[4][4];
      for (int v = 0; v < 4; ++v)
        for (int i = 0; i < 4; ++i) {
          la[i][v] = ls[i][0] + ls[i][1] * Y[v][0] + ls[i][2] * Y[v][1] + ls[i][3] * Y[v][2];
          mu[i][v] = lf[i][0] + lf[i][1] * Y[v][0] + lf[i][2] * Y[v][1] + lf[i][3] * Y[v][2];
        }
      for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) val[i * 4 + j] += int2(vt, la[i], mu[j]);
      if (lam)
        for (int a = 0; a < 4; ++a)
          for (int i = 0; i < 4; ++i) lam[a * 4 + i] += int2(vt, la[a], la[i]);
    }
  }
  (void)F;
  return vol;
}

/* Integrate the listed (solid tet, fluid tet) pairs.  pairs: (n_pairs, 2)
 * int64.  Outputs vals (n_pairs, 16), lams (n_pairs, 16; nullable), vols,
 * keep (vol > drop_rel·|T|).
 * zero_tets counts solid tets of zero volume among the pairs' solid tets
 * (their pairs are written as empty).  Returns 0. */
int o3_pairs(const double* Xs, const int32_t* tets_s, const double* Xf, const int32_t* tets_f,
             const int64_t* pairs, int64_t n_pairs, double drop_rel, int nthreads, double* vals,
             double* lams, double* vols, uint8_t* keep) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 64)
#endif
  for (int64_t p = 0; p < n_pairs; ++p) {
    const int64_t ts = pairs[2 * p], tf = pairs[2 * p + 1];
    double S[4][3], F[4][3], ls[4][4], lf[4][4];
    for (int v = 0; v < 4; ++v)
      for (int e = 0; e < 3; ++e) {
        S[v][e] = Xs[3 * (int64_t)tets_s[4 * ts + v] + e];
        F[v][e] = Xf[3 * (int64_t)tets_f[4 * tf + v] + e];
      }
    double volS = tet_volume(S[0], S[1], S[2], S[3]);
    double volF = tet_volume(F[0], F[1], F[2], F[3]);
    if (volS == 0.0 || volF == 0.0 || barycentric(S, ls) != 0 || barycentric(F, lf) != 0) {
      memset(vals + 16 * p, 0, 16 * sizeof(double));
      if (lams) memset(lams + 16 * p, 0, 16 * sizeof(double));
      vols[p] = 0.0;
      keep[p] = 0;
      continue;
    }
    double vol = piece(S, ls, F, lf, vals + 16 * p, lams ? lams + 16 * p : NULL);
    vols[p] = vol;
    keep[p] = vol > drop_rel * volS;
  }
  return 0;
}

/* Exposed for the pins: volume of tet S (4x3) ∩ tet F (4x3). */
double o3_clip_volume(const double* Sp, const double* Fp) {
  double S[4][3], F[4][3], ls[4][4], lf[4][4], val[16];
  for (int v = 0; v < 4; ++v)
    for (int e = 0; e < 3; ++e) { S[v][e] = Sp[3 * v + e]; F[v][e] = Fp[3 * v + e]; }
  if (barycentric(S, ls) != 0 || barycentric(F, lf) != 0) return 0.0;
  return piece(S, ls, F, lf, val, NULL);
}

/* Exposed for the pins: ∫_τ f g for affine f, g given at τ's vertices. */
double o3_int2(const double* Y, const double* f, const double* g) {
  return int2(tet_volume(Y, Y + 3, Y + 6, Y + 9), f, g);
}
