// Fixed-point (Picard) fluid-structure coupling of Section 3 (Steps 1-6) on
// top of the transfers (3D and planar grid couplings, and the unstructured
// coupling), and the fluid lattice's Q1 lumped volume.
//
// The driver runs the transfers, the Step-2 update and the Step-6 residual
// on the device; the solid and fluid solves are the caller's callbacks.
// Each iteration reads back two numbers (the infinity norms of Step 6).
#include <hipcub/hipcub.hpp>

#include <cmath>
#include <vector>

#include "internal.hpp"

namespace ibvt {

namespace {

constexpr int kThreads = 256;

inline unsigned nblk(int64_t n) { return unsigned(ceil_div(n > 0 ? n : 1, kThreads)); }

// X[i][e] = X_ref[i][e] + u0[e][i]  (current configuration from the
// displacement at the start of the step; dim coordinates per vertex)
template <typename T>
__global__ void k_configuration(int64_t n, int dim, const double* __restrict__ Xref,
                                const T* __restrict__ u0, double* __restrict__ X) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= dim * n) return;
  const int64_t i = k / dim;
  const int e = int(k - dim * i);
  X[k] = Xref[k] + double(u0[int64_t(e) * n + i]);
}

// Step 2: u = u0 + dt w
template <typename T>
__global__ void k_displacement(int64_t n3, const T* __restrict__ u0, const T* __restrict__ w,
                               T dt, T* __restrict__ u) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k < n3) u[k] = u0[k] + dt * w[k];
}

// Step 6 partials: per block max |f − f_prev| and max |f|; f_prev = f.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_inf_norms(int64_t n3, const T* __restrict__ f,
                                                         T* __restrict__ fprev,
                                                         double* __restrict__ part) {
  __shared__ double red[2][kThreads / kWave];
  double dmax = 0.0, amax = 0.0;
  for (int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < n3;
       k += int64_t(gridDim.x) * blockDim.x) {
    const double a = double(f[k]);
    dmax = fmax(dmax, fabs(a - double(fprev[k])));
    amax = fmax(amax, fabs(a));
    fprev[k] = f[k];
  }
  dmax = wave_max(dmax);
  amax = wave_max(amax);
  if (lane_id() == 0) {
    red[0][threadIdx.x / kWave] = dmax;
    red[1][threadIdx.x / kWave] = amax;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    double m = 0.0;
    for (int w = 0; w < kThreads / kWave; ++w) m = fmax(m, red[threadIdx.x][w]);
    part[2 * blockIdx.x + threadIdx.x] = m;
  }
}

__global__ void k_inf_final(const double* __restrict__ part, int nb, double* __restrict__ out) {
  if (threadIdx.x < 2) {
    double m = 0.0;
    for (int b = 0; b < nb; ++b) m = fmax(m, part[2 * b + threadIdx.x]);
    out[threadIdx.x] = m;
  }
}

// f[j] /= wx[ix] wy[iy] wz[iz] over an (n_z, n_y, n_x) lattice
template <typename T>
__global__ void k_density(int64_t nf, int nx, int ny, const double* __restrict__ wx,
                          const double* __restrict__ wy, const double* __restrict__ wz,
                          T* __restrict__ f) {
  const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= nf) return;
  const int64_t ix = j % nx, r = j / nx;
  const int64_t iy = r % ny, iz = r / ny;
  const double w = wx[ix] * wy[iy] * wz[iz];  // > 0 on lattices of two or more cells per axis
  f[j] = w > 0.0 ? T(double(f[j]) / w) : T(0);
}

// f[j] /= wx[ix] wy[iy] over an (n_y, n_x) planar lattice
template <typename T>
__global__ void k_density2(int64_t nf, int nx, const double* __restrict__ wx,
                           const double* __restrict__ wy, T* __restrict__ f) {
  const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= nf) return;
  const int64_t ix = j % nx, iy = j / nx;
  const double w = wx[ix] * wy[iy];
  f[j] = w > 0.0 ? T(double(f[j]) / w) : T(0);
}

__global__ void k_volume(int64_t nf, int nx, int ny, const double* __restrict__ wx,
                         const double* __restrict__ wy, const double* __restrict__ wz,
                         double* __restrict__ out) {
  const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= nf) return;
  const int64_t ix = j % nx, r = j / nx;
  out[j] = wx[ix] * wy[r % ny] * wz[r / ny];
}

// f[j] /= vol[j] for nodal fluid values (unstructured background)
template <typename T>
__global__ void k_density_nodal(int64_t nf, const double* __restrict__ vol, T* __restrict__ f) {
  const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  // a node no tet touches has no volume and no load: its density is zero
  if (j < nf) f[j] = vol[j] > 0.0 ? T(double(f[j]) / vol[j]) : T(0);
}

// One item per (fluid tet, corner), in tet-major order: key = the corner's
// vertex, value = |T| / 4.
__global__ void k_fvol_items(int64_t n_ft, const int32_t* __restrict__ tets,
                             const double* __restrict__ X, int32_t* __restrict__ keys,
                             double* __restrict__ vals) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= 4 * n_ft) return;
  const int64_t t = k >> 2;
  const int32_t* v = tets + 4 * t;
  const double* a = X + 3 * int64_t(v[0]);
  double e[3][3];
  for (int m = 0; m < 3; ++m) {
    const double* b = X + 3 * int64_t(v[m + 1]);
    for (int c = 0; c < 3; ++c) e[m][c] = b[c] - a[c];
  }
  const double det = e[0][0] * (e[1][1] * e[2][2] - e[1][2] * e[2][1]) -
                     e[0][1] * (e[1][0] * e[2][2] - e[1][2] * e[2][0]) +
                     e[0][2] * (e[1][0] * e[2][1] - e[1][1] * e[2][0]);
  keys[k] = v[k & 3];
  vals[k] = fabs(det) / 24.0;
}

// vol[j] = Σ of vertex j's items, in tet order (the items were sorted by a
// stable sort of the tet-major order): one thread per vertex, its run found
// by binary search.
__global__ void k_fvol_sum(int64_t n_v, int64_t n_items, const int32_t* __restrict__ skeys,
                           const double* __restrict__ svals, double* __restrict__ vol) {
  const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= n_v) return;
  int64_t lo = 0, hi = n_items;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (skeys[mid] < j) lo = mid + 1;
    else hi = mid;
  }
  double sum = 0.0;
  for (int64_t k = lo; k < n_items && skeys[k] == j; ++k) sum += svals[k];
  vol[j] = sum;
}

// Lumped volume ∫ μ_j = Σ_{T∋j} |T| / 4 of every fluid node of an
// unstructured background, into c->fvol (deterministic: no value atomics).
int fluid_nodal_volumes(ibvt_coupling* c, hipStream_t s) {
  const int64_t n_ft = c->n_ftet, n_fv = c->n_fvert, n_items = 4 * n_ft;
  int st;
  if ((st = ensure(c, c->fvol, size_t(n_fv + 1) * sizeof(double)))) return st;
  int end_bit = 1;
  while ((int64_t(1) << end_bit) < n_fv + 1) ++end_bit;
  size_t temp_bytes = 0;
  if ((st = hip_check(hipcub::DeviceRadixSort::SortPairs(
                          nullptr, temp_bytes, static_cast<const int32_t*>(nullptr),
                          static_cast<int32_t*>(nullptr), static_cast<const double*>(nullptr),
                          static_cast<double*>(nullptr), int(n_items), 0, end_bit, s),
                      "sort size")))
    return st;
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  const size_t n4 = al(size_t(n_items) * sizeof(int32_t)), n8 = al(size_t(n_items) * sizeof(double));
  if ((st = ensure(c, c->tbuf, 2 * n4 + 2 * n8 + temp_bytes + 256))) return st;
  char* base = c->tbuf.as<char>();
  int32_t* keys = reinterpret_cast<int32_t*>(base);
  int32_t* skeys = reinterpret_cast<int32_t*>(base + n4);
  double* vals = reinterpret_cast<double*>(base + 2 * n4);
  double* svals = reinterpret_cast<double*>(base + 2 * n4 + n8);
  void* temp = base + 2 * n4 + 2 * n8;
  if (n_items > 0) {
    k_fvol_items<<<nblk(n_items), kThreads, 0, s>>>(n_ft, c->ftets.as<int32_t>(),
                                                    c->fX.as<double>(), keys, vals);
    if ((st = hip_check(hipcub::DeviceRadixSort::SortPairs(temp, temp_bytes, keys, skeys, vals,
                                                           svals, int(n_items), 0, end_bit, s),
                        "radix sort")))
      return st;
  }
  k_fvol_sum<<<nblk(n_fv), kThreads, 0, s>>>(n_fv, n_items, skeys, svals, c->fvol.as<double>());
  if ((st = hip_check(hipGetLastError(), "fluid volume launch"))) return st;
  return hip_check(hipStreamSynchronize(s), "sync");
}

// ∫ of the 1D hats of a lattice over its hull [L_0, L_{n-1}]
std::vector<double> hat_weights(const std::vector<double>& L) {
  const size_t n = L.size();
  std::vector<double> w(n, 0.0);
  for (size_t k = 0; k + 1 < n; ++k) {
    const double h = L[k + 1] - L[k];
    w[k] += 0.5 * h;
    w[k + 1] += 0.5 * h;
  }
  return w;
}

// 1D hat weights of the lattices (offsets as the lattice coordinates; the
// planar coupling's unused axes are empty) uploaded once per coupling.
int fluid_weights(ibvt_coupling* c, hipStream_t s) {
  if (c->fvol_ready) return IBVT_OK;
  if (c->unstructured) {
    const int st = fluid_nodal_volumes(c, s);
    if (st) return st;
    c->fvol_ready = true;
    return IBVT_OK;
  }
  std::vector<double> all;
  for (int k = 0; k < 9; ++k) {
    const std::vector<double> w = hat_weights(c->lat_host[k]);
    all.insert(all.end(), w.begin(), w.end());
  }
  int st = ensure(c, c->fvol, all.size() * sizeof(double));
  if (st) return st;
  if ((st = hip_check(hipMemcpyAsync(c->fvol.p, all.data(), all.size() * sizeof(double),
                                     hipMemcpyHostToDevice, s),
                      "copy fluid weights")) ||
      (st = hip_check(hipStreamSynchronize(s), "sync")))
    return st;
  c->fvol_ready = true;
  return IBVT_OK;
}

template <typename T>
int fsi_typed(ibvt_coupling* c, const ibvt_fsi_config* cfg, const ibvt_fsi_buffers* buf,
              ibvt_solid_fn solid, void* sctx, ibvt_fluid_fn fluid, void* fctx, hipStream_t s,
              ibvt_fsi_report* rep) {
  const int nc = c->ncomp;  // = dim
  const int64_t n = c->n_vert, n3 = int64_t(nc) * n;
  int st;
  // current configuration and T there
  if ((st = ensure(c, c->fsiX, size_t(n3) * sizeof(double)))) return st;
  k_configuration<T><<<nblk(n3), kThreads, 0, s>>>(n, c->dim, buf->X_ref,
                                                   static_cast<const T*>(buf->u_hat0),
                                                   c->fsiX.as<double>());
  if ((st = hip_check(hipGetLastError(), "configuration launch"))) return st;
  if ((st = reassemble_coupling(c, c->fsiX.as<double>(), s))) return st;
  if (cfg->force_density && (st = fluid_weights(c, s))) return st;
  const unsigned nb = std::min<unsigned>(nblk(n3), 1024u);
  if ((st = ensure(c, c->fsinorm, size_t(2 * nb + 2) * sizeof(double)))) return st;
  if ((st = ensure(c, c->work2, size_t(n3) * sizeof(T)))) return st;
  const bool lumped_T = c->dual || cfg->mass == IBVT_LUMPED;
  const void* vf_in[3] = {buf->v_f[0], buf->v_f[1], buf->v_f[2]};
  void* ft[3] = {buf->f_tilde[0], buf->f_tilde[1], buf->f_tilde[2]};
  void* vf[3] = {buf->v_f[0], buf->v_f[1], buf->v_f[2]};
  double f1 = 0.0, res = 0.0;
  int it = 0;
  bool conv = false;
  while (it < cfg->max_iter) {
    ++it;
    // Step 1: w_s = T v_f
    st = transfer_velocity(c, vf_in, buf->w_s, lumped_T ? IBVT_LUMPED : IBVT_CONSISTENT,
                           cfg->cg_rtol, cfg->cg_maxit, s, nullptr);
    if (st) return st;
    // Step 2: u_hat = u_hat0 + dt w_s
    k_displacement<T><<<nblk(n3), kThreads, 0, s>>>(n3, static_cast<const T*>(buf->u_hat0),
                                                    static_cast<const T*>(buf->w_s), T(cfg->dt),
                                                    static_cast<T*>(buf->u_hat));
    if ((st = hip_check(hipGetLastError(), "displacement launch"))) return st;
    // Step 3: the solid solve
    if ((st = solid(sctx, buf->u_hat, buf->f_fsi, s))) return st;
    // Step 4: f_tilde = alpha B^T S^{-1} f_fsi (the literal T^T on the load)
    for (int d = 0; d < nc; ++d)
      if ((st = hip_check(hipMemsetAsync(ft[d], 0, size_t(c->n_fluid[d]) * sizeof(T), s),
                          "clear f_tilde")))
        return st;
    if (lumped_T) st = lumped_solve(c, buf->f_fsi, c->work2.p, s);
    else st = mass_solve(c, buf->f_fsi, c->work2.p, cfg->cg_rtol, cfg->cg_maxit, s, nullptr, false);
    if (st) return st;
    if ((st = apply_Bt(c, c->work2.p, ft, cfg->alpha, s))) return st;
    if (cfg->force_density && c->unstructured) {
      for (int d = 0; d < nc; ++d)
        k_density_nodal<T><<<nblk(c->n_fluid[d]), kThreads, 0, s>>>(
            c->n_fluid[d], c->fvol.as<double>(), static_cast<T*>(ft[d]));
      if ((st = hip_check(hipGetLastError(), "density launch"))) return st;
    } else if (cfg->force_density) {
      const double* w = c->fvol.as<double>();
      for (int d = 0; d < nc; ++d) {
        const int nx = c->ld.n[3 * d], ny = c->ld.n[3 * d + 1];
        if (c->dim == 2)
          k_density2<T><<<nblk(c->n_fluid[d]), kThreads, 0, s>>>(
              c->n_fluid[d], nx, w + c->ld.off[3 * d], w + c->ld.off[3 * d + 1],
              static_cast<T*>(ft[d]));
        else
          k_density<T><<<nblk(c->n_fluid[d]), kThreads, 0, s>>>(
              c->n_fluid[d], nx, ny, w + c->ld.off[3 * d], w + c->ld.off[3 * d + 1],
              w + c->ld.off[3 * d + 2], static_cast<T*>(ft[d]));
      }
      if ((st = hip_check(hipGetLastError(), "density launch"))) return st;
    }
    // Step 5: the fluid solve
    if ((st = fluid(fctx, ft, vf, s))) return st;
    // Step 6: infinity norms of f_l − f_{l−1} and of f_l; f_prev = f_l
    k_inf_norms<T><<<nb, kThreads, 0, s>>>(n3, static_cast<const T*>(buf->f_fsi),
                                           static_cast<T*>(buf->f_prev), c->fsinorm.as<double>());
    k_inf_final<<<1, 64, 0, s>>>(c->fsinorm.as<double>(), int(nb),
                                 c->fsinorm.as<double>() + 2 * nb);
    if ((st = hip_check(hipGetLastError(), "norm launch"))) return st;
    double h[2];
    if ((st = hip_check(hipMemcpyAsync(h, c->fsinorm.as<double>() + 2 * nb, sizeof(h),
                                       hipMemcpyDeviceToHost, s),
                        "read norms")) ||
        (st = hip_check(hipStreamSynchronize(s), "sync")))
      return st;
    res = h[0];
    if (it == 1) f1 = h[1];
    const double rel = f1 > 0.0 ? res / f1 : (res > 0.0 ? INFINITY : 0.0);
    if ((cfg->eps_abs > 0.0 && res < cfg->eps_abs) || (cfg->eps_rel > 0.0 && rel < cfg->eps_rel)) {
      conv = true;
      break;
    }
  }
  if (rep) {
    rep->iterations = it;
    rep->converged = conv ? 1 : 0;
    rep->res_abs = res;
    rep->res_rel = f1 > 0.0 ? res / f1 : 0.0;
    rep->f1_norm = f1;
  }
  return conv ? IBVT_OK : set_error(IBVT_E_NOT_CONVERGED, "Picard iteration reached max_iter");
}

}  // namespace

}  // namespace ibvt

using namespace ibvt;

extern "C" {

int fsi_step(ibvt_coupling* c, const ibvt_fsi_config* cfg, const ibvt_fsi_buffers* buf,
             ibvt_solid_fn solid, void* solid_ctx, ibvt_fluid_fn fluid, void* fluid_ctx,
             hipStream_t stream, ibvt_fsi_report* report) {
  if (report) *report = ibvt_fsi_report{};
  if (!c || !cfg || !buf || !solid || !fluid) return set_error(IBVT_E_INVALID, "NULL argument");
  c->stream = stream;
  if (!buf->X_ref || !buf->u_hat0 || !buf->u_hat || !buf->w_s || !buf->f_fsi || !buf->f_prev)
    return set_error(IBVT_E_INVALID, "NULL solid buffer");
  for (int d = 0; d < c->ncomp; ++d)
    if (!buf->v_f[d] || !buf->f_tilde[d]) return set_error(IBVT_E_INVALID, "NULL fluid buffer");
  if (cfg->max_iter < 1 || !std::isfinite(cfg->dt) || !std::isfinite(cfg->alpha))
    return set_error(IBVT_E_INVALID, "max_iter >= 1, finite dt and alpha required");
  if (cfg->mass != IBVT_LUMPED && cfg->mass != IBVT_CONSISTENT)
    return set_error(IBVT_E_INVALID, "mass must be IBVT_LUMPED or IBVT_CONSISTENT");
  if (c->dual && cfg->mass != IBVT_LUMPED)
    return set_error(IBVT_E_INVALID, "the dual basis has a diagonal S: use IBVT_LUMPED");
  if (!c->dual && cfg->mass == IBVT_CONSISTENT) {
    if (!c->has_M) return set_error(IBVT_E_INVALID, "consistent mass was not built");
    if (!(cfg->cg_rtol > 0.0) || cfg->cg_maxit < 1)
      return set_error(IBVT_E_INVALID, "bad mass-solve rtol/maxit");
  }
  if (c->precision == IBVT_FP32_MIXED)
    return fsi_typed<float>(c, cfg, buf, solid, solid_ctx, fluid, fluid_ctx, stream, report);
  return fsi_typed<double>(c, cfg, buf, solid, solid_ctx, fluid, fluid_ctx, stream, report);
}

int ibvt_fluid_lumped_volume_2d(const ibvt_grid2d* grid, int comp, double* out,
                                hipStream_t stream) {
  if (!grid || !out || comp < 0 || comp > 1) return set_error(IBVT_E_INVALID, "bad argument");
  std::vector<double> w[2];
  for (int e = 0; e < 2; ++e) {
    int64_t n = 0;
    int st = ibvt_lattice_coords_2d(grid, comp, e, nullptr, &n);
    if (st) return st;
    std::vector<double> L(static_cast<size_t>(n));
    if ((st = ibvt_lattice_coords_2d(grid, comp, e, L.data(), &n))) return st;
    w[e] = hat_weights(L);
  }
  const size_t total = w[0].size() + w[1].size() + 1;
  double* dw = nullptr;
  int st = hip_check(hipMallocAsync(reinterpret_cast<void**>(&dw), total * sizeof(double), stream),
                     "weights alloc");
  if (st) return st;
  std::vector<double> all(w[0]);
  all.insert(all.end(), w[1].begin(), w[1].end());
  all.push_back(1.0);  // the unit third axis of k_volume
  st = hip_check(hipMemcpyAsync(dw, all.data(), total * sizeof(double), hipMemcpyHostToDevice,
                                stream),
                 "weights copy");
  const int64_t nx = int64_t(w[0].size()), ny = int64_t(w[1].size());
  if (!st) {
    k_volume<<<nblk(nx * ny), kThreads, 0, stream>>>(nx * ny, int(nx), int(ny), dw, dw + nx,
                                                     dw + nx + ny, out);
    st = hip_check(hipGetLastError(), "area launch");
  }
  const int st2 = hip_check(hipStreamSynchronize(stream), "sync");
  (void)hipFreeAsync(dw, stream);
  return st ? st : st2;
}

int ibvt_fluid_lumped_volume(const ibvt_grid* grid, int comp, double* out, hipStream_t stream) {
  if (!grid || !out || comp < 0 || comp > 2) return set_error(IBVT_E_INVALID, "bad argument");
  std::vector<double> w[3];
  for (int e = 0; e < 3; ++e) {
    int64_t n = 0;
    int st = ibvt_lattice_coords(grid, comp, e, nullptr, &n);
    if (st) return st;
    std::vector<double> L(static_cast<size_t>(n));
    if ((st = ibvt_lattice_coords(grid, comp, e, L.data(), &n))) return st;
    w[e] = hat_weights(L);
  }
  const size_t total = w[0].size() + w[1].size() + w[2].size();
  double* dw = nullptr;
  int st = hip_check(hipMallocAsync(reinterpret_cast<void**>(&dw), total * sizeof(double), stream),
                     "weights alloc");
  if (st) return st;
  std::vector<double> all;
  for (int e = 0; e < 3; ++e) all.insert(all.end(), w[e].begin(), w[e].end());
  st = hip_check(hipMemcpyAsync(dw, all.data(), total * sizeof(double), hipMemcpyHostToDevice,
                                stream),
                 "weights copy");
  const int64_t nx = int64_t(w[0].size()), ny = int64_t(w[1].size()), nz = int64_t(w[2].size());
  if (!st) {
    k_volume<<<nblk(nx * ny * nz), kThreads, 0, stream>>>(nx * ny * nz, int(nx), int(ny), dw,
                                                          dw + nx, dw + nx + ny, out);
    st = hip_check(hipGetLastError(), "volume launch");
  }
  const int st2 = hip_check(hipStreamSynchronize(stream), "sync");
  (void)hipFreeAsync(dw, stream);
  return st ? st : st2;
}

}  // extern "C"
