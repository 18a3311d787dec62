// Transfer applies (Section 2.3): velocity  w_s = S^{-1} B v_f  and force
// f_f += alpha B^T f_s, plus the consistent-mass solve.
//
// SpMV: CSR with a group of G lanes per row (rows of B hold a few tens of
// entries, rows of B^T about twice as many); the group strides through the
// row, each lane issuing the loads of U entries at a time, so each wave
// reads contiguous runs of values and column indices with several gathers
// in flight, reduces with lane shuffles and writes one result per row.  The three velocity components run in one
// launch (grid.y).  B^T rows are the touched fluid nodes; their results are
// scattered to the caller's full fluid arrays through the row map (each
// fluid node appears once, so no atomics).
//
// Consistent mass: Chebyshev semi-iteration on D^-1 M (D = diag M) for all
// components at once (one pass over M serves every right-hand side).  The
// spectrum of D^-1 M is known in advance for the P1 mass: an element's
// D_e^-1 M_e = (I + 1 1^T)/2 has the eigenvalues 1/2 and (m + 1)/2 (m
// vertices per element), and a Rayleigh quotient of the assembled pair
// x^T M x / x^T D x, a ratio of sums of the elements' quotients, stays
// between the elements' extremes: [1/2, 5/2] for tetrahedra, [1/2, 2] for
// triangles.  So the iteration needs no inner products: one launch per
// iteration (q = M d, x += d, r -= q, next d from r), with scalars fixed on
// the host, no reduction and no read-back; the count that reduces the error
// by a given factor follows from the Chebyshev polynomial on those bounds.
// Each cycle of iterations ends with the true residual b - M x in double,
// which decides whether another cycle runs.  In the mixed-precision path the
// cycles solve for a float correction of a double solution (iterative
// refinement).
//
// Solid vectors are component-major (ncomp, n_vert): three components in
// three dimensions, two in the plane.
#include "internal.hpp"

#include <cmath>

namespace ibvt {

namespace {

constexpr int kThreads = 256;

template <typename T>
struct SpmvArgs {
  const int64_t* rowptr[3];
  const int32_t* col[3];
  const T* val[3];
  int64_t nrows[3];
  const T* x[3];
  T* y[3];
  const int32_t* rowmap[3];
  const T* scale;   // per-row factor (lumped inverse mass) or null
  T alpha;
  int accumulate;
};

// G lanes per row, U entries per lane per round (their loads issued
// together; the per-lane order of the sums is the entry order).
template <typename T, int G, int U>
__global__ __launch_bounds__(kThreads) void k_spmv(SpmvArgs<T> a) {
  const int d = blockIdx.y;
  const int64_t row = int64_t(blockIdx.x) * (kThreads / G) + threadIdx.x / G;
  const int g = threadIdx.x % G;
  T s = T(0);
  const bool active = row < a.nrows[d];
  if (active) {
    const int64_t b = a.rowptr[d][row], e = a.rowptr[d][row + 1];
    const int32_t* __restrict__ col = a.col[d];
    const T* __restrict__ val = a.val[d];
    const T* __restrict__ x = a.x[d];
    for (int64_t k0 = b + g; k0 < e; k0 += U * G) {
      int32_t c[U];
      T v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t k = k0 + int64_t(u) * G;
        c[u] = k < e ? col[k] : 0;
        v[u] = k < e ? val[k] : T(0);
      }
      T xv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) xv[u] = k0 + int64_t(u) * G < e ? x[c[u]] : T(0);
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (k0 + int64_t(u) * G < e) s += v[u] * xv[u];
    }
  }
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, kWave);
  if (active && g == 0) {
    T v = a.alpha * s;
    if (a.scale) v *= a.scale[row];
    const int64_t dst = a.rowmap[d] ? int64_t(a.rowmap[d][row]) : row;
    if (a.accumulate) a.y[d][dst] += v;
    else a.y[d][dst] = v;
  }
}

template <typename T, int G, int U>
int launch_spmv_g(const SpmvArgs<T>& a, int nc, hipStream_t s, const char* name) {
  int64_t mx = 0;
  for (int d = 0; d < nc; ++d) mx = std::max(mx, a.nrows[d]);
  if (mx <= 0) return IBVT_OK;
  dim3 grid(unsigned(ceil_div(mx, kThreads / G)), unsigned(nc));
  ProfScope ps(name, s);
  k_spmv<T, G, U><<<grid, kThreads, 0, s>>>(a);
  return hip_check(hipGetLastError(), "spmv launch");
}

// Rows averaging fewer than 56 entries (B: a vertex's fluid nodes) take 8
// lanes with 8 entries each per round; longer rows (B^T: a fluid node's
// vertices) 16 lanes with 4 (the faster of the shapes measured on MI355X
// for each).
template <typename T>
int launch_spmv(const SpmvArgs<T>& a, int nc, int64_t nnz, hipStream_t s, const char* name) {
  int64_t rows = 0;
  for (int d = 0; d < nc; ++d) rows += a.nrows[d];
  if (nnz < 56 * rows) return launch_spmv_g<T, 8, 8>(a, nc, s, name);
  return launch_spmv_g<T, 16, 4>(a, nc, s, name);
}

// ---------------------------------------------------------------------------
// consistent-mass solve
// ---------------------------------------------------------------------------

// q = M x for the NC components (values V, vectors T), at the start of a
// solve.  kMG lanes per row stride through it (coalesced reads of the row's
// columns and values) and reduce with lane shuffles in a fixed order.
constexpr int kMG = 4;  // the fastest of 2, 4, 8, 16 on MI355X for P1 mass rows (~15 entries)

template <typename T, typename V, int NC>
__global__ __launch_bounds__(kThreads) void k_mass_spmv(int64_t n, const int64_t* __restrict__ rp,
                                                       const int32_t* __restrict__ col,
                                                       const V* __restrict__ val,
                                                       const T* __restrict__ x, T* __restrict__ q) {
  const int g = threadIdx.x % kMG;
  for (int64_t i = int64_t(blockIdx.x) * (kThreads / kMG) + threadIdx.x / kMG;
       i - threadIdx.x / kMG < n; i += int64_t(gridDim.x) * (kThreads / kMG)) {
    T sd[3] = {0, 0, 0};
    if (i < n) {
      for (int64_t k = rp[i] + g; k < rp[i + 1]; k += kMG) {
        const int64_t j = col[k];
        const T m = T(val[k]);
#pragma unroll
        for (int d = 0; d < NC; ++d) sd[d] += m * x[d * n + j];
      }
    }
#pragma unroll
    for (int o = kMG / 2; o > 0; o >>= 1)
#pragma unroll
      for (int d = 0; d < NC; ++d) sd[d] += __shfl_xor(sd[d], o, kWave);
    if (i < n && g == 0)
#pragma unroll
      for (int d = 0; d < NC; ++d) q[d * n + i] = sd[d];
  }
}

// Start of a cycle: r = b - q (q = M x) or r = b with x = 0 when q is
// null; d = D^-1 r / θ.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_cheb_start(int nc, int64_t n, const T* __restrict__ b,
                                                        const T* __restrict__ q, T* __restrict__ x,
                                                        T* __restrict__ r, T* __restrict__ d,
                                                        const double* __restrict__ dinv,
                                                        double inv_theta) {
  const int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
  if (i >= n) return;
  const double di = dinv[i] * inv_theta;
  for (int c = 0; c < nc; ++c) {
    const int64_t k = int64_t(c) * n + i;
    T rv;
    if (q) {
      rv = b[k] - q[k];
    } else {
      rv = b[k];
      x[k] = T(0);
    }
    r[k] = rv;
    d[k] = T(di * double(rv));
  }
}

__global__ __launch_bounds__(kThreads) void k_reduce6(const double* __restrict__ part, int64_t nb,
                                                     double* __restrict__ out) {
  __shared__ double red[6][kThreads / kWave];
  double loc[6] = {0, 0, 0, 0, 0, 0};
  for (int64_t b = threadIdx.x; b < nb; b += kThreads)
    for (int d = 0; d < 6; ++d) loc[d] += part[b * 6 + d];
  for (int d = 0; d < 6; ++d) {
    const double w = wave_sum(loc[d]);
    if (lane_id() == 0) red[d][threadIdx.x / kWave] = w;
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    double t = 0;
    for (int w = 0; w < kThreads / kWave; ++w) t += red[threadIdx.x][w];
    out[threadIdx.x] = t;
  }
}

// One Chebyshev iteration, kMG lanes per row as in k_mass_spmv: q = M d_in
// (gathered), then for the row's own entries x += d_in, r -= q and
// d_out = c_keep d_in + c_new D^-1 r.  d_in and d_out are distinct buffers,
// so rows read by other blocks are never overwritten within a launch.
template <typename T, typename V, int NC>
__global__ __launch_bounds__(kThreads) void k_cheb(int64_t n, const int64_t* __restrict__ rp,
                                                  const int32_t* __restrict__ col,
                                                  const V* __restrict__ val,
                                                  const double* __restrict__ dinv,
                                                  const T* __restrict__ din, T* __restrict__ dout,
                                                  T* __restrict__ x, T* __restrict__ r, T c_keep,
                                                  T c_new) {
  const int g = threadIdx.x % kMG;
  for (int64_t i = int64_t(blockIdx.x) * (kThreads / kMG) + threadIdx.x / kMG;
       i - threadIdx.x / kMG < n; i += int64_t(gridDim.x) * (kThreads / kMG)) {
    T sd[3] = {0, 0, 0};
    if (i < n) {
      const int64_t e = rp[i + 1];
      // two entries per lane per round, their loads issued together (same
      // per-lane order of the sums)
      for (int64_t k0 = rp[i] + g; k0 < e; k0 += 2 * kMG) {
        const int64_t k1 = k0 + kMG;
        const int64_t j0 = col[k0];
        const int64_t j1 = k1 < e ? col[k1] : j0;
        const T m0 = T(val[k0]);
        const T m1 = k1 < e ? T(val[k1]) : T(0);
        T p0[NC], p1[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          p0[c] = din[c * n + j0];
          p1[c] = din[c * n + j1];
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          sd[c] += m0 * p0[c];
          if (k1 < e) sd[c] += m1 * p1[c];
        }
      }
    }
#pragma unroll
    for (int o = kMG / 2; o > 0; o >>= 1)
#pragma unroll
      for (int c = 0; c < NC; ++c) sd[c] += __shfl_xor(sd[c], o, kWave);
    if (i < n && g == 0) {
      const T di = T(dinv[i]);
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const int64_t k = c * n + i;
        const T dv = din[k];
        const T rv = r[k] - sd[c];
        x[k] += dv;
        r[k] = rv;
        dout[k] = c_keep * dv + c_new * di * rv;
      }
    }
  }
}


// residual in double: res = b - M x  (b, x of type T; M double), kMG
// lanes per row as in k_mass_spmv.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_residual64(int nc, int64_t n, const int64_t* __restrict__ rp,
                                                        const int32_t* __restrict__ col,
                                                        const double* __restrict__ val,
                                                        const T* __restrict__ b,
                                                        const double* __restrict__ x,
                                                        double* __restrict__ res,
                                                        double* __restrict__ part) {
  __shared__ double red[6][kThreads / kWave];
  const int g = threadIdx.x % kMG;
  double loc[6] = {0, 0, 0, 0, 0, 0};
  for (int64_t i = int64_t(blockIdx.x) * (kThreads / kMG) + threadIdx.x / kMG;
       i - threadIdx.x / kMG < n; i += int64_t(gridDim.x) * (kThreads / kMG)) {
    double s[3] = {0, 0, 0};
    if (i < n) {
      for (int64_t k = rp[i] + g; k < rp[i + 1]; k += kMG) {
        const int64_t j = col[k];
        for (int d = 0; d < nc; ++d) s[d] += val[k] * x[int64_t(d) * n + j];
      }
    }
#pragma unroll
    for (int o = kMG / 2; o > 0; o >>= 1)
      for (int d = 0; d < 3; ++d) s[d] += __shfl_xor(s[d], o, kWave);
    if (i < n && g == 0) {
      for (int d = 0; d < nc; ++d) {
        const double bv = double(b[int64_t(d) * n + i]);
        const double rv = bv - s[d];
        res[int64_t(d) * n + i] = rv;
        loc[d] += rv * rv;
        loc[3 + d] += bv * bv;
      }
    }
  }
  for (int d = 0; d < 6; ++d) {
    const double w = wave_sum(loc[d]);
    if (lane_id() == 0) red[d][threadIdx.x / kWave] = w;
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    double t = 0;
    for (int w = 0; w < kThreads / kWave; ++w) t += red[threadIdx.x][w];
    part[int64_t(blockIdx.x) * 6 + threadIdx.x] = t;
  }
}

template <typename Tin, typename Tout>
__global__ void k_convert(int64_t n, const Tin* __restrict__ a, Tout* __restrict__ b) {
  const int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
  if (i < n) b[i] = Tout(a[i]);
}

template <typename T>
__global__ void k_lumped_apply(int nc, int64_t n, const T* __restrict__ rhs,
                               const T* __restrict__ minv, T* __restrict__ x) {
  const int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
  if (i < n)
    for (int d = 0; d < nc; ++d) x[int64_t(d) * n + i] = rhs[int64_t(d) * n + i] * minv[i];
}

template <typename T>
__global__ void k_axpy(int64_t n, T alpha, const T* __restrict__ x, T* __restrict__ y) {
  const int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
  if (i < n) y[i] += alpha * x[i];
}

__global__ void k_add_correction(int64_t n3, const float* __restrict__ e, double* __restrict__ x) {
  const int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
  if (i < n3) x[i] += double(e[i]);
}

inline unsigned nblk(int64_t n) { return unsigned(ceil_div(n > 0 ? n : 1, kThreads)); }

// blocks of the row-group kernels (grid-stride over groups of kThreads / kMG
// rows; capped so that their per-block partials stay few)
inline unsigned nblk_rows(int64_t n) {
  return unsigned(std::min<int64_t>(ceil_div(n > 0 ? n : 1, kThreads / kMG), 2048));
}

// Workspace layout of the mass solve (bytes): partials, 6 vectors of T
// (q, r, d and d' of the iteration and two refinement vectors; b is read in
// place), plus double x/res for the residuals and the refinement.
struct MassWork {
  double* part;
  double* tmp;
  void* vec;
  double* x64;
  double* res64;
};

// Layout of the mass-solve workspace for n vertices and value size tsize:
// residual partials, reduction results, six (3, n) vectors of T, the double
// solution and residual.  Returns the bytes it spans; with base non-null
// also sets w's pointers into [base, base + bytes).
size_t mass_workspace_layout(int64_t n, size_t tsize, char* base, MassWork* w) {
  // per-block partials of the residual kernel fit
  const int64_t nb = std::max<int64_t>(nblk(n), nblk_rows(n));
  const size_t off_part = 256;
  const size_t off_tmp = off_part + size_t(nb) * 6 * sizeof(double);
  const size_t off_vec = (off_tmp + 16 * sizeof(double) + 255) & ~size_t(255);
  const size_t off_x64 = (off_vec + size_t(6 * 3 * n) * tsize + 255) & ~size_t(255);
  const size_t off_res = (off_x64 + size_t(3 * n) * sizeof(double) + 255) & ~size_t(255);
  const size_t total = off_res + size_t(3 * n) * sizeof(double) + 256;
  if (base && w) {
    w->part = reinterpret_cast<double*>(base + off_part);
    w->tmp = reinterpret_cast<double*>(base + off_tmp);
    w->vec = base + off_vec;
    w->x64 = reinterpret_cast<double*>(base + off_x64);
    w->res64 = reinterpret_cast<double*>(base + off_res);
  }
  return total;
}

// The workspace in the coupling's own buffer (grown as needed), or at ext
// (the caller's memory of at least mass_workspace_layout bytes).
int mass_workspace(ibvt_coupling* c, size_t tsize, MassWork& w, char* ext) {
  const int64_t n = c->n_vert;
  if (ext) {
    mass_workspace_layout(n, tsize, ext, &w);
    return IBVT_OK;
  }
  const size_t total = mass_workspace_layout(n, tsize, nullptr, nullptr);
  int st = ensure(c, c->work, total);
  if (st) return st;
  mass_workspace_layout(n, tsize, c->work.as<char>(), &w);
  return IBVT_OK;
}

// Bounds of the spectrum of D^-1 M for the coupling's P1 mass (elements of
// dim + 1 vertices): [1/2, (dim + 2)/2].
struct ChebBounds {
  double theta, delta, sigma1;
};

ChebBounds cheb_bounds(const ibvt_coupling* c) {
  const double lo = 0.5, hi = 0.5 * double(c->dim + 2);
  ChebBounds k;
  k.theta = 0.5 * (hi + lo);
  k.delta = 0.5 * (hi - lo);
  k.sigma1 = k.theta / k.delta;
  return k;
}

// Iterations after which the Chebyshev polynomial on the bounds is at most
// eps in magnitude there (T_k(σ1) >= 1/eps): the error's energy norm is then
// reduced by eps at least.
int cheb_iterations(const ChebBounds& k, double eps) {
  if (!(eps < 1.0)) return 1;  // a loose tolerance: one iteration, then the residual test
  const double it = std::acosh(1.0 / eps) / std::acosh(k.sigma1);
  return std::max(1, int(std::ceil(it)));
}

// `iters` Chebyshev iterations on M (values V) for the right-hand sides b
// (type T), x in/out (x_zero: start from x = 0, which the first launch
// writes).  The scalars follow the three-term recurrence of the scaled
// Chebyshev polynomials: ρ_0 = 1/σ1, ρ_{k+1} = 1/(2σ1 − ρ_k), d_{k+1} =
// ρ_{k+1}ρ_k d_k + (2ρ_{k+1}/δ) D^-1 r_{k+1}, d_0 = D^-1 r_0 / θ.
template <typename T, typename V>
int cheb_cycle(ibvt_coupling* c, const V* mval, const T* b, T* x, bool x_zero, int iters,
               const MassWork& w, hipStream_t s) {
  const int64_t n = c->n_vert;
  const int nc = c->ncomp;
  const unsigned nb = nblk(n);
  const unsigned nbm = nblk_rows(n);
  T* q = static_cast<T*>(w.vec);
  T* r = q + 3 * n;
  T* dbuf[2] = {r + 3 * n, r + 6 * n};
  const int64_t* rp = c->M.rowptr.as<int64_t>();
  const int32_t* col = c->M.col.as<int32_t>();
  const double* dinv = c->Mdiag_inv.as<double>();
  const ChebBounds k = cheb_bounds(c);
  if (!x_zero) {
    if (nc == 3) k_mass_spmv<T, V, 3><<<nbm, kThreads, 0, s>>>(n, rp, col, mval, x, q);
    else k_mass_spmv<T, V, 2><<<nbm, kThreads, 0, s>>>(n, rp, col, mval, x, q);
  }
  k_cheb_start<T><<<nb, kThreads, 0, s>>>(nc, n, b, x_zero ? nullptr : q, x, r, dbuf[0], dinv,
                                          1.0 / k.theta);
  int st = hip_check(hipGetLastError(), "mass solve start launch");
  if (st) return st;
  double rho = 1.0 / k.sigma1;
  for (int it = 0; it < iters; ++it) {
    ProfScope ps("mass_iteration", s);
    const double rho1 = 1.0 / (2.0 * k.sigma1 - rho);
    const T c_keep = T(rho1 * rho), c_new = T(2.0 * rho1 / k.delta);
    const T* din = dbuf[it & 1];
    T* dout = dbuf[(it + 1) & 1];
    if (nc == 3)
      k_cheb<T, V, 3><<<nbm, kThreads, 0, s>>>(n, rp, col, mval, dinv, din, dout, x, r, c_keep,
                                               c_new);
    else
      k_cheb<T, V, 2><<<nbm, kThreads, 0, s>>>(n, rp, col, mval, dinv, din, dout, x, r, c_keep,
                                               c_new);
    rho = rho1;
  }
  return hip_check(hipGetLastError(), "mass solve launch");
}

// True residual norms ||b - M x|| / ||b|| in double (x as double).
template <typename T>
int true_residual(ibvt_coupling* c, const T* b, const double* x, const MassWork& w, hipStream_t s,
                  double rel[3]) {
  const int64_t n = c->n_vert;
  const unsigned nb = nblk_rows(n);
  k_residual64<T><<<nb, kThreads, 0, s>>>(c->ncomp, n, c->M.rowptr.as<int64_t>(),
                                          c->M.col.as<int32_t>(),
                                          c->M.val.as<double>(), b, x, w.res64, w.part);
  k_reduce6<<<1, kThreads, 0, s>>>(w.part, nb, w.tmp);
  double h[6];
  int st = hip_check(hipMemcpyAsync(h, w.tmp, sizeof(h), hipMemcpyDeviceToHost, s), "res read");
  if (st) return st;
  if ((st = hip_check(hipStreamSynchronize(s), "res sync"))) return st;
  for (int d = 0; d < 3; ++d) rel[d] = (h[3 + d] > 0) ? std::sqrt(h[d] / h[3 + d]) : 0.0;
  return IBVT_OK;
}

}  // namespace

int apply_B(ibvt_coupling* c, const void* const x[3], void* y, bool lumped_scale, hipStream_t s) {
  if (c->matrix_free) return apply_B_matfree(c, x, y, lumped_scale, s);
  const int64_t n = c->n_vert;
  int64_t nnz = 0;
  for (int d = 0; d < c->ncomp; ++d) nnz += c->B[d].nnz;
  if (c->precision == IBVT_FP32_MIXED) {
    SpmvArgs<float> a{};
    for (int d = 0; d < 3; ++d) {
      a.rowptr[d] = c->B[d].rowptr.as<int64_t>();
      a.col[d] = c->B[d].col.as<int32_t>();
      a.val[d] = c->B[d].val.as<float>();
      a.nrows[d] = n;
      a.x[d] = static_cast<const float*>(x[d]);
      a.y[d] = static_cast<float*>(y) + d * n;
    }
    a.scale = lumped_scale ? c->minv.as<float>() : nullptr;
    a.alpha = 1.0f;
    return launch_spmv<float>(a, c->ncomp, nnz, s, "spmv_B");
  }
  SpmvArgs<double> a{};
  for (int d = 0; d < 3; ++d) {
    a.rowptr[d] = c->B[d].rowptr.as<int64_t>();
    a.col[d] = c->B[d].col.as<int32_t>();
    a.val[d] = c->B[d].val.as<double>();
    a.nrows[d] = n;
    a.x[d] = static_cast<const double*>(x[d]);
    a.y[d] = static_cast<double*>(y) + d * n;
  }
  a.scale = lumped_scale ? c->minv.as<double>() : nullptr;
  a.alpha = 1.0;
  return launch_spmv<double>(a, c->ncomp, nnz, s, "spmv_B");
}

// out[d][rowmap[r]] += alpha * (B^dT ys_d)[r]
int apply_Bt(ibvt_coupling* c, const void* ys, void* const out[3], double alpha, hipStream_t s) {
  if (c->matrix_free) return apply_Bt_matfree(c, ys, out, alpha, s);
  const int64_t n = c->n_vert;
  int64_t nnz = 0;
  for (int d = 0; d < c->ncomp; ++d) nnz += c->Bt[d].nnz;
  if (c->precision == IBVT_FP32_MIXED) {
    SpmvArgs<float> a{};
    for (int d = 0; d < 3; ++d) {
      a.rowptr[d] = c->Bt[d].rowptr.as<int64_t>();
      a.col[d] = c->Bt[d].col.as<int32_t>();
      a.val[d] = c->Bt[d].val.as<float>();
      a.nrows[d] = c->Bt[d].nrows;
      a.x[d] = static_cast<const float*>(ys) + d * n;
      a.y[d] = static_cast<float*>(out[d]);
      a.rowmap[d] = c->Bt[d].rowmap.as<int32_t>();
    }
    a.alpha = float(alpha);
    a.accumulate = 1;
    return launch_spmv<float>(a, c->ncomp, nnz, s, "spmv_Bt");
  }
  SpmvArgs<double> a{};
  for (int d = 0; d < 3; ++d) {
    a.rowptr[d] = c->Bt[d].rowptr.as<int64_t>();
    a.col[d] = c->Bt[d].col.as<int32_t>();
    a.val[d] = c->Bt[d].val.as<double>();
    a.nrows[d] = c->Bt[d].nrows;
    a.x[d] = static_cast<const double*>(ys) + d * n;
    a.y[d] = static_cast<double*>(out[d]);
    a.rowmap[d] = c->Bt[d].rowmap.as<int32_t>();
  }
  a.alpha = alpha;
  a.accumulate = 1;
  return launch_spmv<double>(a, c->ncomp, nnz, s, "spmv_Bt");
}

int lumped_solve(ibvt_coupling* c, const void* rhs, void* x, hipStream_t s) {
  const int64_t n = c->n_vert;
  if (c->precision == IBVT_FP32_MIXED)
    k_lumped_apply<float><<<nblk(n), kThreads, 0, s>>>(c->ncomp, n, static_cast<const float*>(rhs),
                                                       c->minv.as<float>(), static_cast<float*>(x));
  else
    k_lumped_apply<double><<<nblk(n), kThreads, 0, s>>>(c->ncomp, n, static_cast<const double*>(rhs),
                                                        c->minv.as<double>(),
                                                        static_cast<double*>(x));
  return hip_check(hipGetLastError(), "lumped launch");
}

int axpy_solid(ibvt_coupling* c, double alpha, const void* x, void* y, hipStream_t s) {
  const int64_t n3 = int64_t(c->ncomp) * c->n_vert;
  if (c->precision == IBVT_FP32_MIXED)
    k_axpy<float><<<nblk(n3), kThreads, 0, s>>>(n3, float(alpha), static_cast<const float*>(x),
                                                static_cast<float*>(y));
  else
    k_axpy<double><<<nblk(n3), kThreads, 0, s>>>(n3, alpha, static_cast<const double*>(x),
                                                 static_cast<double*>(y));
  return hip_check(hipGetLastError(), "axpy launch");
}

// x = M^{-1} rhs (every component).  x holds the start (lumped solution)
// when x_has_guess.
size_t mass_solve_workspace_bytes(const ibvt_coupling* c) {
  const size_t tsize = c->precision == IBVT_FP32_MIXED ? sizeof(float) : sizeof(double);
  return mass_workspace_layout(c->n_vert, tsize, nullptr, nullptr);
}

int mass_solve(ibvt_coupling* c, const void* rhs, void* x, double rtol, int maxit, hipStream_t s,
               ibvt_solve_info* info, bool x_has_guess, char* ws) {
  if (!c->has_M) return set_error(IBVT_E_INVALID, "consistent mass was not built (flags)");
  const int64_t n = c->n_vert;
  const int64_t nn = int64_t(c->ncomp) * n;
  int st;
  if (!x_has_guess && (st = lumped_solve(c, rhs, x, s))) return st;
  int done = 0;
  bool conv = false;
  double rel[3] = {0, 0, 0};
  const ChebBounds kb = cheb_bounds(c);
  auto converged = [&]() {
    for (int d = 0; d < c->ncomp; ++d)
      if (!(rel[d] <= rtol)) return false;
    return true;
  };
  // Each cycle aims a tenth below its target, so that the norm in which the
  // bound holds (energy of the error) and the residual's 2-norm tested here
  // rarely differ by enough to need another cycle.
  if (c->precision == IBVT_FP64) {
    MassWork w;
    if ((st = mass_workspace(c, sizeof(double), w, ws))) return st;
    double* xd = static_cast<double*>(x);
    const double* b = static_cast<const double*>(rhs);
    const int per_cycle = cheb_iterations(kb, 0.1 * rtol);
    do {
      const int it = std::min(per_cycle, maxit - done);
      if ((st = cheb_cycle<double, double>(c, c->M.val.as<double>(), b, xd, false, it, w, s)))
        return st;
      done += it;
      if ((st = true_residual<double>(c, b, xd, w, s, rel))) return st;
    } while (!(conv = converged()) && done < maxit);
  } else {
    // iterative refinement: double residual, float correction cycles
    MassWork w;
    if ((st = mass_workspace(c, sizeof(float), w, ws))) return st;
    const float* b = static_cast<const float*>(rhs);
    float* xf = static_cast<float*>(x);
    k_convert<float, double><<<nblk(nn), kThreads, 0, s>>>(nn, xf, w.x64);
    float* e = static_cast<float*>(w.vec) + 4 * 3 * n;   // vectors 4 and 5 of the workspace
    float* rf = e + 3 * n;
    for (;;) {
      if ((st = true_residual<float>(c, b, w.x64, w, s, rel))) return st;
      if ((conv = converged()) || done >= maxit) break;
      k_convert<double, float><<<nblk(nn), kThreads, 0, s>>>(nn, w.res64, rf);
      // the reduction still needed (rtol over the largest relative
      // residual), at most what float iterations can give
      double worst = 0.0;
      for (int d = 0; d < c->ncomp; ++d) worst = std::max(worst, rel[d]);
      const double want = std::min(0.1, std::max(1e-5, rtol / worst));
      const int it = std::min(cheb_iterations(kb, 0.1 * want), maxit - done);
      if ((st = cheb_cycle<float, float>(c, c->Mval32.as<float>(), rf, e, true, it, w, s)))
        return st;
      k_add_correction<<<nblk(nn), kThreads, 0, s>>>(nn, e, w.x64);
      done += it;
    }
    k_convert<double, float><<<nblk(nn), kThreads, 0, s>>>(nn, w.x64, xf);
    if ((st = hip_check(hipGetLastError(), "refinement launch"))) return st;
  }
  int iters[3] = {0, 0, 0};
  for (int d = 0; d < c->ncomp; ++d) iters[d] = done;
  if (info) {
    for (int d = 0; d < 3; ++d) {
      info->iterations[d] = iters[d];
      info->rel_residual[d] = rel[d];
    }
  }
  if (!conv) return set_error(IBVT_E_NOT_CONVERGED, "consistent-mass solve reached maxit");
  return IBVT_OK;
}

}  // namespace ibvt
