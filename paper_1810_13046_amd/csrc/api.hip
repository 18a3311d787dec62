// C-ABI entry points of libibvt (declared in include/ibvt.h).
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "internal.hpp"

#include <algorithm>
#include <map>
#include <mutex>

namespace ibvt {

namespace {
thread_local std::string g_last_error;

struct ProfRec {
  const char* name;
  hipEvent_t a, b;
};
struct ProfState {
  std::mutex mu;
  bool on = false;
  std::vector<ProfRec> recs;
};
ProfState& prof() {
  static ProfState p;
  return p;
}
}  // namespace

ProfScope::ProfScope(const char* name, hipStream_t stream) : s(stream) {
  ProfState& P = prof();
  if (!P.on) return;
  ProfRec r{name, nullptr, nullptr};
  if (hipEventCreate(&r.a) != hipSuccess || hipEventCreate(&r.b) != hipSuccess) return;
  (void)hipEventRecord(r.a, stream);
  std::lock_guard<std::mutex> g(P.mu);
  slot = int(P.recs.size());
  P.recs.push_back(r);
}

ProfScope::~ProfScope() {
  if (slot < 0) return;
  ProfState& P = prof();
  std::lock_guard<std::mutex> g(P.mu);
  if (slot < int(P.recs.size())) (void)hipEventRecord(P.recs[slot].b, s);
}

int set_error(int status, const std::string& msg) {
  g_last_error = msg;
  return status;
}

int hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return IBVT_OK;
  if (e == hipErrorOutOfMemory)
    return set_error(IBVT_E_NOMEM, std::string(what) + ": " + hipGetErrorString(e));
  return set_error(IBVT_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

namespace {
std::mutex g_alloc_mu;
ibvt_alloc g_alloc{};  // allocator of new handles (null members: hipMallocAsync)

// Stream-ordered release of one buffer through the handle's allocator.
hipError_t free_buffer(ibvt_coupling* c, void* p) {
  if (c->alloc.free) {
    c->alloc.free(p, c->stream, c->alloc.ctx);
    return hipSuccess;
  }
  return hipFreeAsync(p, c->stream);
}

ibvt_alloc current_allocator() {
  std::lock_guard<std::mutex> g(g_alloc_mu);
  return g_alloc;
}
}  // namespace

int ensure(ibvt_coupling* c, DevBuf& b, size_t bytes) {
  if (bytes == 0) bytes = 1;
  if (b.p && b.cap >= bytes) return IBVT_OK;
  // stream-ordered: the old buffer is released after the work queued on
  // the call's stream, and growing does not synchronize the device
  if (b.p) {
    hipError_t e = free_buffer(c, b.p);
    c->device_bytes -= int64_t(b.cap);
    b.p = nullptr;
    b.cap = 0;
    if (e != hipSuccess) return hip_check(e, "hipFreeAsync");
  }
  // grow with headroom so a moving mesh does not reallocate every step
  // (1/8 of the size, 1/32 above 1 GiB)
  const size_t want = bytes + (bytes > (size_t(1) << 30) ? bytes / 32 : bytes / 8) + 256;
  if (c->alloc.alloc) {
    b.p = c->alloc.alloc(want, c->stream, c->alloc.ctx);
    if (!b.p) return set_error(IBVT_E_NOMEM, "the coupling's allocator returned NULL");
  } else {
    hipError_t e = hipMallocAsync(&b.p, want, c->stream);
    if (e != hipSuccess) {
      b.p = nullptr;
      (void)hipGetLastError();
      return hip_check(e, "hipMallocAsync");
    }
  }
  b.cap = want;
  c->device_bytes += int64_t(want);
  return IBVT_OK;
}

void release(ibvt_coupling* c, DevBuf& b) {
  if (b.p) {
    (void)free_buffer(c, b.p);
    c->device_bytes -= int64_t(b.cap);
  }
  b.p = nullptr;
  b.cap = 0;
}

namespace {

// Per-body sums, one block per body: tets, zero-volume tets and volume over
// the body's tet range, candidate pairs and kept pieces over its pair range
// in each of the `groups` pair groups (pair_off over groups x n_t).  Output
// cnt[b][4] = (tets, zero tets, pairs, pieces), vol[b].
constexpr int kBodyThreads = 256;
__global__ __launch_bounds__(kBodyThreads) void k_body_info(
    const int64_t* __restrict__ off, int64_t n_t, int groups, const double* __restrict__ tetvol,
    const int64_t* __restrict__ pair_off, const uint8_t* __restrict__ keep,
    int64_t* __restrict__ cnt, double* __restrict__ vol) {
  __shared__ unsigned long long s_zero[kBodyThreads / kWave], s_kept[kBodyThreads / kWave];
  __shared__ double s_vol[kBodyThreads / kWave];
  const int b = blockIdx.x;
  const int64_t t0 = off[b], t1 = off[b + 1];
  unsigned long long zero = 0, kept = 0;
  double v = 0.0;
  for (int64_t t = t0 + threadIdx.x; t < t1; t += kBodyThreads) {
    const double x = tetvol[t];
    v += x;
    zero += (x == 0.0) ? 1u : 0u;
  }
  int64_t pairs = 0;
  for (int g = 0; g < groups; ++g) {
    const int64_t p0 = pair_off[int64_t(g) * n_t + t0], p1 = pair_off[int64_t(g) * n_t + t1];
    pairs += p1 - p0;
    if (keep)
      for (int64_t p = p0 + threadIdx.x; p < p1; p += kBodyThreads) kept += keep[p] ? 1u : 0u;
  }
  zero = wave_sum(zero);
  kept = wave_sum(kept);
  v = wave_sum(v);
  const int w = threadIdx.x / kWave;
  if (lane_id() == 0) {
    s_zero[w] = zero;
    s_kept[w] = kept;
    s_vol[w] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < kBodyThreads / kWave; ++k) {
      zero += s_zero[k];
      kept += s_kept[k];
      v += s_vol[k];
    }
    cnt[4 * b + 0] = t1 - t0;
    cnt[4 * b + 1] = int64_t(zero);
    cnt[4 * b + 2] = pairs;
    cnt[4 * b + 3] = keep ? int64_t(kept) : -1;
    vol[b] = v;
  }
}

void release_csr(ibvt_coupling* c, Csr& m) {
  release(c, m.rowptr);
  release(c, m.col);
  release(c, m.val);
  release(c, m.rowmap);
}

void release_all(ibvt_coupling* c) {
  DevBuf* bufs[] = {&c->lat,      &c->X,         &c->tets,      &c->vt_ptr,    &c->vt_tet,
                    &c->tetvol,   &c->tetrec,    &c->rng,       &c->pmom,      &c->cnt,
                    &c->pair_off, &c->owner,     &c->pval,      &c->keep,      &c->rownnz,
                    &c->mark,     &c->cidx,      &c->tbuf,      &c->mlump,     &c->minv,
                    &c->Mval32,   &c->Mdiag_inv, &c->flags_dev, &c->counters,  &c->scan_tmp,
                    &c->work,     &c->work2,     &c->zbuf,      &c->pool,      &c->pinfo,
                    &c->order,    &c->pscan,     &c->rowbox,    &c->rowcap,    &c->rowtmpoff,
                    &c->rowtmpcol, &c->rowtmpval, &c->tetgrad, &c->mcoef,
                    &c->fsiX,     &c->fsinorm,   &c->fvol,      &c->fX,        &c->ftets,
                    &c->frec,     &c->fbox,      &c->forder,    &c->ftree,     &c->ucoo,
                    &c->rb,       &c->bodyinfo,  &c->tcorder,   &c->rowspilloff,
                    &c->rowspill};
  for (DevBuf* b : bufs) release(c, *b);
  if (c->host_rb) {
    (void)hipHostFree(c->host_rb);
    c->host_rb = nullptr;
  }
  // an unstructured coupling's components share B[0] and Bt[0]
  const int own = c->unstructured ? 1 : 3;
  for (int d = 0; d < own; ++d) {
    release_csr(c, c->B[d]);
    release_csr(c, c->Bt[d]);
  }
  for (int d = own; d < 3; ++d) c->B[d] = c->Bt[d] = Csr{};
  release_csr(c, c->M);
}

int validate_grid(const ibvt_grid* g) {
  if (!g) return set_error(IBVT_E_INVALID, "grid is NULL");
  for (int e = 0; e < 3; ++e) {
    if (g->n_cells[e] < 2)
      return set_error(IBVT_E_INVALID, "each axis needs at least 2 cells (cell-centre lattices)");
    if (!g->faces[e]) return set_error(IBVT_E_INVALID, "grid faces pointer is NULL");
    for (int k = 0; k <= g->n_cells[e]; ++k)
      if (!std::isfinite(g->faces[e][k]))
        return set_error(IBVT_E_INVALID, "non-finite face coordinate");
    for (int k = 0; k < g->n_cells[e]; ++k)
      if (!(g->faces[e][k + 1] > g->faces[e][k]))
        return set_error(IBVT_E_INVALID, "face coordinates must be strictly increasing");
  }
  int64_t n = 1;
  for (int e = 0; e < 3; ++e) n *= int64_t(g->n_cells[e]) + 1;
  if (n >= (int64_t(1) << 31))
    return set_error(IBVT_E_CAPACITY, "lattice has 2^31 nodes or more (int32 column indices)");
  return IBVT_OK;
}

// Lattice of component d along axis e: faces along d, midpoints elsewhere.
std::vector<double> lattice_axis(const ibvt_grid* g, int d, int e) {
  std::vector<double> out;
  const int n = g->n_cells[e];
  if (e == d) {
    out.assign(g->faces[e], g->faces[e] + n + 1);
  } else {
    out.resize(n);
    for (int k = 0; k < n; ++k) out[k] = 0.5 * (g->faces[e][k] + g->faces[e][k + 1]);
  }
  return out;
}

int setup_lattices(ibvt_coupling* c, const ibvt_grid* g, hipStream_t s) {
  int32_t off = 0;
  for (int d = 0; d < 3; ++d) {
    int64_t nf = 1;
    for (int e = 0; e < 3; ++e) {
      c->lat_host[3 * d + e] = lattice_axis(g, d, e);
      c->ld.off[3 * d + e] = off;
      c->ld.n[3 * d + e] = int32_t(c->lat_host[3 * d + e].size());
      off += c->ld.n[3 * d + e];
      nf *= c->ld.n[3 * d + e];
    }
    c->n_fluid[d] = nf;
  }
  int st = ensure(c, c->lat, size_t(off) * sizeof(double));
  if (st) return st;
  std::vector<double> flat;
  flat.reserve(off);
  for (int k = 0; k < 9; ++k) flat.insert(flat.end(), c->lat_host[k].begin(), c->lat_host[k].end());
  st = hip_check(hipMemcpyAsync(c->lat.p, flat.data(), flat.size() * sizeof(double),
                                hipMemcpyHostToDevice, s),
                 "lattice copy");
  if (st) return st;
  return hip_check(hipStreamSynchronize(s), "lattice sync");
}

bool bad_ptr(const void* p) { return p == nullptr; }

// A handle whose last assembly failed holds matrices and per-pair data of
// different assemblies: every call that reads them is refused.
int require_ready(const ibvt_coupling* c) {
  if (!c->ready)
    return set_error(IBVT_E_INVALID,
                     "the coupling's last assembly failed: reassemble it successfully first");
  return IBVT_OK;
}

// Planar grids: the same checks and lattices over two axes.  The lattice
// table keeps the 3 x 3 layout (entries of axis or component 2 stay empty).
int validate_grid2d(const ibvt_grid2d* g) {
  if (!g) return set_error(IBVT_E_INVALID, "grid is NULL");
  for (int e = 0; e < 2; ++e) {
    if (g->n_cells[e] < 2)
      return set_error(IBVT_E_INVALID, "each axis needs at least 2 cells (cell-centre lattices)");
    if (!g->faces[e]) return set_error(IBVT_E_INVALID, "grid faces pointer is NULL");
    for (int k = 0; k <= g->n_cells[e]; ++k)
      if (!std::isfinite(g->faces[e][k]))
        return set_error(IBVT_E_INVALID, "non-finite face coordinate");
    for (int k = 0; k < g->n_cells[e]; ++k)
      if (!(g->faces[e][k + 1] > g->faces[e][k]))
        return set_error(IBVT_E_INVALID, "face coordinates must be strictly increasing");
  }
  if ((int64_t(g->n_cells[0]) + 1) * (int64_t(g->n_cells[1]) + 1) >= (int64_t(1) << 31))
    return set_error(IBVT_E_CAPACITY, "lattice has 2^31 nodes or more (int32 column indices)");
  return IBVT_OK;
}

std::vector<double> lattice_axis2d(const ibvt_grid2d* g, int d, int e) {
  ibvt_grid g3{};
  for (int k = 0; k < 2; ++k) {
    g3.n_cells[k] = g->n_cells[k];
    g3.faces[k] = g->faces[k];
  }
  return lattice_axis(&g3, d, e);
}

int setup_lattices2d(ibvt_coupling* c, const ibvt_grid2d* g, hipStream_t s) {
  int32_t off = 0;
  for (int k = 0; k < 9; ++k) {
    c->lat_host[k].clear();
    c->ld.off[k] = 0;
    c->ld.n[k] = 0;
  }
  for (int d = 0; d < 2; ++d) {
    int64_t nf = 1;
    for (int e = 0; e < 2; ++e) {
      c->lat_host[3 * d + e] = lattice_axis2d(g, d, e);
      c->ld.off[3 * d + e] = off;
      c->ld.n[3 * d + e] = int32_t(c->lat_host[3 * d + e].size());
      off += c->ld.n[3 * d + e];
      nf *= c->ld.n[3 * d + e];
    }
    c->n_fluid[d] = nf;
  }
  c->n_fluid[2] = 0;
  int st = ensure(c, c->lat, size_t(off) * sizeof(double));
  if (st) return st;
  std::vector<double> flat;
  flat.reserve(off);
  for (int k = 0; k < 9; ++k) flat.insert(flat.end(), c->lat_host[k].begin(), c->lat_host[k].end());
  st = hip_check(hipMemcpyAsync(c->lat.p, flat.data(), flat.size() * sizeof(double),
                                hipMemcpyHostToDevice, s),
                 "lattice copy");
  if (st) return st;
  return hip_check(hipStreamSynchronize(s), "lattice sync");
}

// Copies the mesh, builds the topology and assembles; frees the handle on
// failure.
int finish_assembly(ibvt_coupling* c, const double* X, const int32_t* elems, hipStream_t stream,
                    ibvt_coupling** out) {
  const int K = c->dim + 1;
  int st = ensure(c, c->X, size_t(c->dim * c->n_vert) * sizeof(double));
  if (!st) st = ensure(c, c->tets, size_t(K * c->n_tet + 4) * sizeof(int32_t));
  if (!st)
    st = hip_check(hipMemcpyAsync(c->X.p, X, size_t(c->dim * c->n_vert) * sizeof(double),
                                  hipMemcpyDeviceToDevice, stream),
                   "copy X");
  if (!st && c->n_tet > 0)
    st = hip_check(hipMemcpyAsync(c->tets.p, elems, size_t(K * c->n_tet) * sizeof(int32_t),
                                  hipMemcpyDeviceToDevice, stream),
                   "copy elements");
  if (!st) st = build_topology(c, stream);
  if (!st) st = assemble_all(c, stream);
  if (st) {
    std::string keep_msg = g_last_error;
    (void)hipStreamSynchronize(stream);
    release_all(c);
    delete c;
    g_last_error = keep_msg;
    return st;
  }
  *out = c;
  return IBVT_OK;
}

// Argument checks of transfer_velocity_vjp (no work done).
int check_velocity_vjp(ibvt_coupling* c, const void* g_us, const void* const u_f[3],
                       const void* u_s, int mass, double cg_rtol, int cg_maxit,
                       void* const g_uf[3], double* g_X) {
  if (!c || !g_us) return set_error(IBVT_E_INVALID, "NULL argument");
  if (int st0 = require_ready(c)) return st0;
  if (mass != IBVT_LUMPED && mass != IBVT_CONSISTENT)
    return set_error(IBVT_E_INVALID, "mass must be IBVT_LUMPED or IBVT_CONSISTENT");
  if (c->dual && mass != IBVT_LUMPED)
    return set_error(IBVT_E_INVALID, "the dual basis has a diagonal S: use IBVT_LUMPED");
  if (g_X && (!u_f || !u_s)) return set_error(IBVT_E_INVALID, "g_X needs u_f and u_s");
  if (g_X)
    for (int d = 0; d < c->ncomp; ++d)
      if (!u_f[d]) return set_error(IBVT_E_INVALID, "NULL fluid component");
  if (g_uf)
    for (int d = 0; d < c->ncomp; ++d)
      if (!g_uf[d]) return set_error(IBVT_E_INVALID, "NULL g_uf component");
  if (mass == IBVT_CONSISTENT) {
    if (!c->has_M) return set_error(IBVT_E_INVALID, "consistent mass was not built");
    if (!(cg_rtol > 0.0) || cg_maxit < 1) return set_error(IBVT_E_INVALID, "bad mass-solve rtol/maxit");
  }
  return IBVT_OK;
}

// Argument checks of transfer_force_vjp (no work done).
int check_force_vjp(ibvt_coupling* c, const void* const g_ff[3], const void* f_s, double alpha,
                    double* g_X) {
  if (!c || !g_ff) return set_error(IBVT_E_INVALID, "NULL argument");
  if (int st0 = require_ready(c)) return st0;
  for (int d = 0; d < c->ncomp; ++d)
    if (!g_ff[d]) return set_error(IBVT_E_INVALID, "NULL g_ff component");
  if (g_X && !f_s) return set_error(IBVT_E_INVALID, "g_X needs f_s");
  if (!std::isfinite(alpha)) return set_error(IBVT_E_INVALID, "alpha must be finite");
  return IBVT_OK;
}

// z = S^{-1} g_us into c->zbuf, and g_uf += B^T z.
int velocity_adjoint(ibvt_coupling* c, const void* g_us, int mass, double cg_rtol, int cg_maxit,
                     void* const g_uf[3], hipStream_t stream, void** z_out) {
  const size_t tsize = c->precision == IBVT_FP32_MIXED ? sizeof(float) : sizeof(double);
  // z lives in its own buffer (the shape kernels reuse work2)
  int st = ensure(c, c->zbuf, size_t(3 * c->n_vert) * tsize);
  if (st) return st;
  void* z = c->zbuf.p;
  if (mass == IBVT_LUMPED) {
    if ((st = lumped_solve(c, g_us, z, stream))) return st;
  } else if ((st = mass_solve(c, g_us, z, cg_rtol, cg_maxit, stream, nullptr, false))) {
    return st;
  }
  if (g_uf && (st = apply_Bt(c, z, g_uf, 1.0, stream))) return st;
  *z_out = z;
  return IBVT_OK;
}

// g_fs += alpha B g_ff (B into scratch, then accumulate).
int force_adjoint(ibvt_coupling* c, const void* const g_ff[3], double alpha, void* g_fs,
                  hipStream_t stream) {
  if (!g_fs) return IBVT_OK;
  const size_t tsize = c->precision == IBVT_FP32_MIXED ? sizeof(float) : sizeof(double);
  int st = ensure(c, c->zbuf, size_t(3 * c->n_vert) * tsize);
  if (st) return st;
  if ((st = apply_B(c, g_ff, c->zbuf.p, false, stream))) return st;
  return axpy_solid(c, alpha, c->zbuf.p, g_fs, stream);
}

}  // namespace
}  // namespace ibvt

using namespace ibvt;

extern "C" {

const char* ibvt_status_string(int status) {
  switch (status) {
    case IBVT_OK: return "ok";
    case IBVT_E_INVALID: return "invalid argument";
    case IBVT_E_OUT_OF_GRID: return "solid outside the fluid lattice";
    case IBVT_E_HIP: return "HIP runtime error";
    case IBVT_E_NOMEM: return "out of device memory";
    case IBVT_E_NOT_CONVERGED: return "iteration limit reached before convergence";
    case IBVT_E_CAPACITY: return "internal capacity exceeded";
    case IBVT_E_UNSUPPORTED: return "unsupported combination";
    default: return "unknown status";
  }
}

const char* ibvt_last_error(void) { return g_last_error.c_str(); }

int ibvt_lattice_coords(const ibvt_grid* grid, int comp, int axis, double* out, int64_t* n) {
  int st = validate_grid(grid);
  if (st) return st;
  if (comp < 0 || comp > 2 || axis < 0 || axis > 2 || !n)
    return set_error(IBVT_E_INVALID, "bad comp/axis or NULL n");
  std::vector<double> v = lattice_axis(grid, comp, axis);
  *n = int64_t(v.size());
  if (out) std::memcpy(out, v.data(), v.size() * sizeof(double));
  return IBVT_OK;
}

int ibvt_lattice_coords_2d(const ibvt_grid2d* grid, int comp, int axis, double* out, int64_t* n) {
  int st = validate_grid2d(grid);
  if (st) return st;
  if (comp < 0 || comp > 1 || axis < 0 || axis > 1 || !n)
    return set_error(IBVT_E_INVALID, "bad comp/axis or NULL n");
  std::vector<double> v = lattice_axis2d(grid, comp, axis);
  *n = int64_t(v.size());
  if (out) std::memcpy(out, v.data(), v.size() * sizeof(double));
  return IBVT_OK;
}

int assemble_coupling(const ibvt_grid* grid, const ibvt_mesh* mesh, int precision,
                      uint32_t flags, hipStream_t stream, ibvt_coupling** out) {
  if (!out) return set_error(IBVT_E_INVALID, "out is NULL");
  *out = nullptr;
  int st = validate_grid(grid);
  if (st) return st;
  if (!mesh) return set_error(IBVT_E_INVALID, "mesh is NULL");
  if (mesh->n_vert < 1 || mesh->n_tet < 0)
    return set_error(IBVT_E_INVALID, "mesh needs n_vert >= 1 and n_tet >= 0");
  if (mesh->n_vert >= (int64_t(1) << 31) || mesh->n_tet >= (int64_t(1) << 31) / 3)
    return set_error(IBVT_E_CAPACITY, "mesh too large for int32 indices");
  if (bad_ptr(mesh->X) || (mesh->n_tet > 0 && bad_ptr(mesh->tets)))
    return set_error(IBVT_E_INVALID, "mesh X or tets is NULL");
  if (precision != IBVT_FP64 && precision != IBVT_FP32_MIXED)
    return set_error(IBVT_E_INVALID, "precision must be IBVT_FP64 or IBVT_FP32_MIXED");
  if (flags & ~(IBVT_BUILD_CONSISTENT_M | IBVT_NO_PIECE_STORE | IBVT_DUAL_BASIS | IBVT_NO_STORE_B))
    return set_error(IBVT_E_INVALID, "unknown flags");
  ibvt_coupling* c = new (std::nothrow) ibvt_coupling();
  if (!c) return set_error(IBVT_E_NOMEM, "host allocation failed");
  c->alloc = current_allocator();
  c->stream = stream;
  c->precision = precision;
  c->flags = flags;
  c->n_vert = mesh->n_vert;
  c->n_tet = mesh->n_tet;
  c->has_M = (flags & IBVT_BUILD_CONSISTENT_M) != 0;
  c->matrix_free = (flags & IBVT_NO_STORE_B) != 0;
  c->store_pieces = (flags & IBVT_NO_PIECE_STORE) == 0 && !c->matrix_free;
  c->dual = (flags & IBVT_DUAL_BASIS) != 0;
  for (int e = 0; e < 3; ++e) c->n_cells[e] = grid->n_cells[e];
  st = setup_lattices(c, grid, stream);
  if (st) {
    release_all(c);
    delete c;
    return st;
  }
  return finish_assembly(c, mesh->X, mesh->tets, stream, out);
}

int assemble_coupling_unstructured(const ibvt_mesh* fluid, const ibvt_mesh* mesh, int precision,
                                   uint32_t flags, hipStream_t stream, ibvt_coupling** out) {
  if (!out) return set_error(IBVT_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!fluid || !mesh) return set_error(IBVT_E_INVALID, "mesh is NULL");
  if (fluid->n_vert < 4 || fluid->n_tet < 1 || mesh->n_vert < 1 || mesh->n_tet < 0)
    return set_error(IBVT_E_INVALID, "fluid mesh needs tets; solid mesh needs n_vert >= 1");
  if (fluid->n_vert >= (int64_t(1) << 31) || fluid->n_tet >= (int64_t(1) << 30) ||
      mesh->n_vert >= (int64_t(1) << 31) || mesh->n_tet >= (int64_t(1) << 31) / 3)
    return set_error(IBVT_E_CAPACITY, "mesh too large for int32 indices");
  if (bad_ptr(fluid->X) || bad_ptr(fluid->tets) || bad_ptr(mesh->X) ||
      (mesh->n_tet > 0 && bad_ptr(mesh->tets)))
    return set_error(IBVT_E_INVALID, "mesh X or tets is NULL");
  if (precision != IBVT_FP64 && precision != IBVT_FP32_MIXED)
    return set_error(IBVT_E_INVALID, "precision must be IBVT_FP64 or IBVT_FP32_MIXED");
  if (flags & IBVT_NO_STORE_B)
    return set_error(IBVT_E_UNSUPPORTED, "IBVT_NO_STORE_B is for grid couplings");
  if (flags & ~(IBVT_BUILD_CONSISTENT_M | IBVT_NO_PIECE_STORE | IBVT_DUAL_BASIS))
    return set_error(IBVT_E_INVALID, "unknown flags");
  ibvt_coupling* c = new (std::nothrow) ibvt_coupling();
  if (!c) return set_error(IBVT_E_NOMEM, "host allocation failed");
  c->alloc = current_allocator();
  c->unstructured = true;
  c->stream = stream;
  c->precision = precision;
  c->flags = flags;
  c->n_vert = mesh->n_vert;
  c->n_tet = mesh->n_tet;
  c->n_fvert = fluid->n_vert;
  c->n_ftet = fluid->n_tet;
  c->has_M = (flags & IBVT_BUILD_CONSISTENT_M) != 0;
  c->store_pieces = false;
  c->dual = (flags & IBVT_DUAL_BASIS) != 0;
  for (int d = 0; d < 3; ++d) c->n_fluid[d] = fluid->n_vert;
  int st = ensure(c, c->fX, size_t(3 * fluid->n_vert) * sizeof(double));
  if (!st) st = ensure(c, c->ftets, size_t(4 * fluid->n_tet) * sizeof(int32_t));
  if (!st) st = ensure(c, c->flags_dev, 64);
  if (!st) st = ensure(c, c->counters, kCntSlots * sizeof(unsigned long long));
  if (!st)
    st = hip_check(hipMemcpyAsync(c->fX.p, fluid->X, size_t(3 * fluid->n_vert) * sizeof(double),
                                  hipMemcpyDeviceToDevice, stream),
                   "copy fluid X");
  if (!st)
    st = hip_check(hipMemcpyAsync(c->ftets.p, fluid->tets,
                                  size_t(4 * fluid->n_tet) * sizeof(int32_t),
                                  hipMemcpyDeviceToDevice, stream),
                   "copy fluid tets");
  if (st) {
    std::string keep_msg = g_last_error;
    (void)hipStreamSynchronize(stream);
    release_all(c);
    delete c;
    g_last_error = keep_msg;
    return st;
  }
  return finish_assembly(c, mesh->X, mesh->tets, stream, out);
}

int assemble_coupling_2d(const ibvt_grid2d* grid, const ibvt_mesh2d* mesh, int precision,
                         uint32_t flags, hipStream_t stream, ibvt_coupling** out) {
  if (!out) return set_error(IBVT_E_INVALID, "out is NULL");
  *out = nullptr;
  int st = validate_grid2d(grid);
  if (st) return st;
  if (!mesh) return set_error(IBVT_E_INVALID, "mesh is NULL");
  if (mesh->n_vert < 1 || mesh->n_tri < 0)
    return set_error(IBVT_E_INVALID, "mesh needs n_vert >= 1 and n_tri >= 0");
  if (mesh->n_vert >= (int64_t(1) << 31) || mesh->n_tri >= (int64_t(1) << 31) / 3)
    return set_error(IBVT_E_CAPACITY, "mesh too large for int32 indices");
  if (bad_ptr(mesh->X) || (mesh->n_tri > 0 && bad_ptr(mesh->tris)))
    return set_error(IBVT_E_INVALID, "mesh X or tris is NULL");
  if (precision != IBVT_FP64 && precision != IBVT_FP32_MIXED)
    return set_error(IBVT_E_INVALID, "precision must be IBVT_FP64 or IBVT_FP32_MIXED");
  if (flags & IBVT_NO_STORE_B)
    return set_error(IBVT_E_UNSUPPORTED, "IBVT_NO_STORE_B is for grid couplings");
  if (flags & ~(IBVT_BUILD_CONSISTENT_M | IBVT_NO_PIECE_STORE | IBVT_DUAL_BASIS))
    return set_error(IBVT_E_INVALID, "unknown flags");
  ibvt_coupling* c = new (std::nothrow) ibvt_coupling();
  if (!c) return set_error(IBVT_E_NOMEM, "host allocation failed");
  c->alloc = current_allocator();
  c->dim = 2;
  c->ncomp = 2;
  c->stream = stream;
  c->precision = precision;
  c->flags = flags;
  c->n_vert = mesh->n_vert;
  c->n_tet = mesh->n_tri;
  c->has_M = (flags & IBVT_BUILD_CONSISTENT_M) != 0;
  c->store_pieces = true;
  c->dual = (flags & IBVT_DUAL_BASIS) != 0;
  for (int e = 0; e < 2; ++e) c->n_cells[e] = grid->n_cells[e];
  c->n_cells[2] = 0;
  st = setup_lattices2d(c, grid, stream);
  if (st) {
    release_all(c);
    delete c;
    return st;
  }
  return finish_assembly(c, mesh->X, mesh->tris, stream, out);
}

int reassemble_coupling(ibvt_coupling* c, const double* X, hipStream_t stream) {
  if (!c || !X) return set_error(IBVT_E_INVALID, "NULL coupling or X");
  c->stream = stream;
  int st = hip_check(hipMemcpyAsync(c->X.p, X, size_t(c->dim * c->n_vert) * sizeof(double),
                                    hipMemcpyDeviceToDevice, stream),
                     "copy X");
  if (st) return st;
  return assemble_all(c, stream);
}

int transfer_velocity(ibvt_coupling* c, const void* const u_f[3], void* u_s, int mass,
                      double cg_rtol, int cg_maxit, hipStream_t stream, ibvt_solve_info* info) {
  if (!c || !u_f || !u_s) return set_error(IBVT_E_INVALID, "NULL argument");
  if (int st0 = require_ready(c)) return st0;
  c->stream = stream;
  for (int d = 0; d < c->ncomp; ++d)
    if (!u_f[d]) return set_error(IBVT_E_INVALID, "NULL fluid component");
  if (mass != IBVT_LUMPED && mass != IBVT_CONSISTENT)
    return set_error(IBVT_E_INVALID, "mass must be IBVT_LUMPED or IBVT_CONSISTENT");
  if (c->dual && mass != IBVT_LUMPED)
    return set_error(IBVT_E_INVALID, "the dual basis has a diagonal S: use IBVT_LUMPED");
  if (info) std::memset(info, 0, sizeof(*info));
  if (mass == IBVT_LUMPED) return apply_B(c, u_f, u_s, true, stream);
  if (!c->has_M) return set_error(IBVT_E_INVALID, "consistent mass was not built");
  if (!(cg_rtol > 0.0) || cg_maxit < 1) return set_error(IBVT_E_INVALID, "bad mass-solve rtol/maxit");
  // rhs = B u_f into the scratch, start from the lumped solution in u_s
  const size_t tsize = c->precision == IBVT_FP32_MIXED ? sizeof(float) : sizeof(double);
  int st = ensure(c, c->work2, size_t(3 * c->n_vert) * tsize);
  if (st) return st;
  if ((st = apply_B(c, u_f, c->work2.p, false, stream))) return st;
  if ((st = lumped_solve(c, c->work2.p, u_s, stream))) return st;
  return mass_solve(c, c->work2.p, u_s, cg_rtol, cg_maxit, stream, info, true);
}

int transfer_force(ibvt_coupling* c, const void* f_s, void* const f_f[3], double alpha,
                   uint32_t flags, hipStream_t stream) {
  if (!c || !f_s || !f_f) return set_error(IBVT_E_INVALID, "NULL argument");
  if (int st0 = require_ready(c)) return st0;
  c->stream = stream;
  for (int d = 0; d < c->ncomp; ++d)
    if (!f_f[d]) return set_error(IBVT_E_INVALID, "NULL fluid component");
  if (flags & ~IBVT_FORCE_IS_LOAD) return set_error(IBVT_E_INVALID, "unknown flags");
  if (!std::isfinite(alpha)) return set_error(IBVT_E_INVALID, "alpha must be finite");
  if (flags & IBVT_FORCE_IS_LOAD) {
    const size_t tsize = c->precision == IBVT_FP32_MIXED ? sizeof(float) : sizeof(double);
    int st = ensure(c, c->work2, size_t(3 * c->n_vert) * tsize);
    if (st) return st;
    if (c->dual) {  // S = diag(m)
      if ((st = lumped_solve(c, f_s, c->work2.p, stream))) return st;
      return apply_Bt(c, c->work2.p, f_f, alpha, stream);
    }
    if (!c->has_M) return set_error(IBVT_E_INVALID, "consistent mass was not built");
    const double rtol = c->precision == IBVT_FP32_MIXED ? 1e-6 : 1e-12;
    if ((st = mass_solve(c, f_s, c->work2.p, rtol, 500, stream, nullptr, false))) return st;
    return apply_Bt(c, c->work2.p, f_f, alpha, stream);
  }
  return apply_Bt(c, f_s, f_f, alpha, stream);
}


int transfer_velocity_vjp(ibvt_coupling* c, const void* g_us, const void* const u_f[3],
                          const void* u_s, int mass, double cg_rtol, int cg_maxit,
                          void* const g_uf[3], double* g_X, hipStream_t stream) {
  int st = check_velocity_vjp(c, g_us, u_f, u_s, mass, cg_rtol, cg_maxit, g_uf, g_X);
  if (st) return st;
  c->stream = stream;
  void* z = nullptr;
  if ((st = velocity_adjoint(c, g_us, mass, cg_rtol, cg_maxit, g_uf, stream, &z))) return st;
  if (g_X) {
    const int m = mass == IBVT_CONSISTENT ? 1 : 0;
    st = c->unstructured ? shape_gradient_unstructured(c, z, u_f, u_s, m, 1.0, g_X, stream)
         : c->dim == 2   ? shape_gradient_2d(c, z, u_f, u_s, m, 1.0, g_X, stream)
                         : shape_gradient(c, z, u_f, u_s, m, 1.0, g_X, stream);
    if (st) return st;
  }
  return IBVT_OK;
}

int transfer_force_vjp(ibvt_coupling* c, const void* const g_ff[3], const void* f_s,
                       double alpha, void* g_fs, double* g_X, hipStream_t stream) {
  int st = check_force_vjp(c, g_ff, f_s, alpha, g_X);
  if (st) return st;
  c->stream = stream;
  if ((st = force_adjoint(c, g_ff, alpha, g_fs, stream))) return st;
  if (g_X) {
    st = c->unstructured
             ? shape_gradient_unstructured(c, f_s, g_ff, nullptr, -1, alpha, g_X, stream)
         : c->dim == 2 ? shape_gradient_2d(c, f_s, g_ff, nullptr, -1, alpha, g_X, stream)
                       : shape_gradient(c, f_s, g_ff, nullptr, -1, alpha, g_X, stream);
    if (st) return st;
  }
  return IBVT_OK;
}

int transfer_vjp(ibvt_coupling* c, const void* g_us, const void* const u_f[3], const void* u_s,
                 int mass, double cg_rtol, int cg_maxit, void* const g_uf[3],
                 const void* const g_ff[3], const void* f_s, double alpha, void* g_fs,
                 double* g_X, hipStream_t stream) {
  int st = check_velocity_vjp(c, g_us, u_f, u_s, mass, cg_rtol, cg_maxit, g_uf, g_X);
  if (st) return st;
  c->stream = stream;
  if ((st = check_force_vjp(c, g_ff, f_s, alpha, g_X))) return st;
  if (!(g_X && c->dim == 3 && (c->unstructured || c->mom_valid))) {
    // no stored moments to share: the two calls
    if ((st = transfer_force_vjp(c, g_ff, f_s, alpha, g_fs, g_X, stream))) return st;
    return transfer_velocity_vjp(c, g_us, u_f, u_s, mass, cg_rtol, cg_maxit, g_uf, g_X, stream);
  }
  // the force part first (its scratch is the buffer z then takes)
  if ((st = force_adjoint(c, g_ff, alpha, g_fs, stream))) return st;
  void* z = nullptr;
  if ((st = velocity_adjoint(c, g_us, mass, cg_rtol, cg_maxit, g_uf, stream, &z))) return st;
  const int m = mass == IBVT_CONSISTENT ? 1 : 0;
  if (c->unstructured)
    return shape_gradient_unstructured_two(c, z, u_f, u_s, m, f_s, g_ff, alpha, g_X, stream);
  return shape_gradient_two(c, z, u_f, u_s, m, f_s, g_ff, alpha, g_X, stream);
}

int coupling_info(const ibvt_coupling* c, ibvt_info* info) {
  if (!c || !info) return set_error(IBVT_E_INVALID, "NULL argument");
  std::memset(info, 0, sizeof(*info));
  info->precision = c->precision;
  info->has_consistent_mass = c->has_M ? 1 : 0;
  info->n_vert = c->n_vert;
  info->n_tet = c->n_tet;
  for (int d = 0; d < 3; ++d) {
    for (int e = 0; e < 3; ++e) info->lattice[d][e] = c->ld.n[3 * d + e];
    info->n_fluid[d] = c->n_fluid[d];
    info->nnz[d] = c->B[d].nnz;
    info->touched[d] = c->Bt[d].nrows;
  }
  info->pairs = c->stats.pairs;
  info->pieces = c->stats.pieces;
  info->dropped = c->stats.dropped;
  info->zero_tets = c->stats.zero_tets;
  info->nnz_mass = c->has_M ? c->M.nnz : 0;
  info->device_bytes = c->device_bytes;
  info->assemblies = c->stats.assemblies;
  info->subtets = c->stats.subtets;
  info->piece_store = c->mom_valid ? 1 : 0;
  info->dist_evals = c->stats.dist_evals;
  info->cut_points = c->stats.cut_points;
  info->plane_cuts = c->stats.plane_cuts;
  info->dual = c->dual ? 1 : 0;
  info->dim = c->dim;
  info->unstructured = c->unstructured ? 1 : 0;
  info->matrix_free = c->matrix_free ? 1 : 0;
  return IBVT_OK;
}

int coupling_export_csr(const ibvt_coupling* c, int comp, int transposed, int64_t* n_rows,
                        int64_t* nnz, int32_t* row_ptr, int32_t* col, double* val,
                        int32_t* row_map) {
  if (!c || comp < 0 || comp >= c->ncomp || !n_rows || !nnz)
    return set_error(IBVT_E_INVALID, "bad argument");
  if (int st0 = require_ready(c)) return st0;
  if (c->matrix_free)
    return set_error(IBVT_E_UNSUPPORTED, "the coupling keeps no matrices (IBVT_NO_STORE_B)");
  const Csr& m = transposed ? c->Bt[comp] : c->B[comp];
  *n_rows = m.nrows;
  *nnz = m.nnz;
  if (!row_ptr && !col && !val && !row_map) return IBVT_OK;
  int st = hip_check(hipDeviceSynchronize(), "sync");
  if (st) return st;
  if (row_ptr) {
    std::vector<int64_t> rp(size_t(m.nrows + 1));
    if ((st = hip_check(hipMemcpy(rp.data(), m.rowptr.p, rp.size() * sizeof(int64_t),
                                  hipMemcpyDeviceToHost),
                        "copy")))
      return st;
    if (m.nnz >= (int64_t(1) << 31)) return set_error(IBVT_E_CAPACITY, "nnz exceeds int32");
    for (size_t k = 0; k < rp.size(); ++k) row_ptr[k] = int32_t(rp[k]);
  }
  if (col && m.nnz)
    if ((st = hip_check(hipMemcpy(col, m.col.p, size_t(m.nnz) * sizeof(int32_t), hipMemcpyDeviceToHost),
                        "copy")))
      return st;
  if (val && m.nnz) {
    if (c->precision == IBVT_FP32_MIXED) {
      std::vector<float> v(size_t(m.nnz));
      if ((st = hip_check(hipMemcpy(v.data(), m.val.p, v.size() * sizeof(float), hipMemcpyDeviceToHost),
                          "copy")))
        return st;
      for (size_t k = 0; k < v.size(); ++k) val[k] = double(v[k]);
    } else if ((st = hip_check(hipMemcpy(val, m.val.p, size_t(m.nnz) * sizeof(double),
                                         hipMemcpyDeviceToHost),
                               "copy"))) {
      return st;
    }
  }
  if (row_map && transposed && m.nrows)
    if ((st = hip_check(hipMemcpy(row_map, m.rowmap.p, size_t(m.nrows) * sizeof(int32_t),
                                  hipMemcpyDeviceToHost),
                        "copy")))
      return st;
  return IBVT_OK;
}

void ibvt_profile_enable(int on) {
  ProfState& P = prof();
  std::lock_guard<std::mutex> g(P.mu);
  P.on = on != 0;
}

int ibvt_profile_read(const char** names, int64_t* launches, double* ms, int max) {
  ProfState& P = prof();
  std::lock_guard<std::mutex> g(P.mu);
  std::map<std::string, std::pair<int64_t, double>> acc;
  std::map<std::string, const char*> keep;
  int status = 0;
  for (ProfRec& r : P.recs) {
    float t = 0.f;
    if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&t, r.a, r.b) != hipSuccess)
      status = -IBVT_E_HIP;
    auto& e = acc[r.name];
    e.first += 1;
    e.second += double(t);
    keep[r.name] = r.name;
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  P.recs.clear();
  if (status) return status;
  int k = 0;
  for (auto& kv : acc) {
    if (k >= max) break;
    if (names) names[k] = keep[kv.first];
    if (launches) launches[k] = kv.second.first;
    if (ms) ms[k] = kv.second.second;
    ++k;
  }
  return k;
}

int coupling_release_scratch(ibvt_coupling* c, hipStream_t stream) {
  if (!c) return set_error(IBVT_E_INVALID, "NULL handle");
  if (c->dim != 3 || c->unstructured) return IBVT_OK;
  c->stream = stream;
  for (DevBuf* b : {&c->pool, &c->pinfo, &c->rowtmpcol, &c->rowtmpval, &c->rowbox, &c->rowcap,
                    &c->rowtmpoff, &c->tbuf, &c->pscan, &c->mark, &c->cidx, &c->rowspilloff,
                    &c->rowspill})
    release(c, *b);
  // the matrix-free products keep their per-tet buffer and item order
  if (!c->matrix_free) {
    release(c, c->pval);
    release(c, c->order);
  }
  c->pool_cap = 0;
  return IBVT_OK;
}

int coupling_body_info(ibvt_coupling* c, int32_t n_bodies, const int64_t* tet_offsets,
                       ibvt_body_info* out, hipStream_t stream) {
  if (!c || !tet_offsets || !out) return set_error(IBVT_E_INVALID, "NULL argument");
  if (n_bodies < 1) return set_error(IBVT_E_INVALID, "n_bodies must be >= 1");
  if (int st0 = require_ready(c)) return st0;
  if (tet_offsets[0] != 0 || tet_offsets[n_bodies] != c->n_tet)
    return set_error(IBVT_E_INVALID, "tet_offsets must start at 0 and end at n_tet");
  for (int32_t b = 0; b < n_bodies; ++b)
    if (tet_offsets[b + 1] < tet_offsets[b])
      return set_error(IBVT_E_INVALID, "tet_offsets must not decrease");
  c->stream = stream;
  const size_t ob = (size_t(n_bodies + 1) * sizeof(int64_t) + 255) & ~size_t(255);
  const size_t cb = (size_t(n_bodies) * 4 * sizeof(int64_t) + 255) & ~size_t(255);
  int st = ensure(c, c->bodyinfo, ob + cb + size_t(n_bodies) * sizeof(double));
  if (st) return st;
  int64_t* doff = c->bodyinfo.as<int64_t>();
  int64_t* dcnt = reinterpret_cast<int64_t*>(c->bodyinfo.as<char>() + ob);
  double* dvol = reinterpret_cast<double*>(c->bodyinfo.as<char>() + ob + cb);
  if ((st = hip_check(hipMemcpyAsync(doff, tet_offsets, size_t(n_bodies + 1) * sizeof(int64_t),
                                     hipMemcpyHostToDevice, stream),
                      "copy offsets")))
    return st;
  const int groups = c->unstructured ? 1 : c->ncomp;
  const uint8_t* keep = (c->matrix_free || c->n_pairs == 0) ? nullptr : c->keep.as<uint8_t>();
  k_body_info<<<unsigned(n_bodies), kBodyThreads, 0, stream>>>(
      doff, c->n_tet, groups, c->tetvol.as<double>(), c->pair_off.as<int64_t>(), keep, dcnt, dvol);
  if ((st = hip_check(hipGetLastError(), "body info launch"))) return st;
  std::vector<int64_t> hc(size_t(n_bodies) * 4);
  std::vector<double> hv(static_cast<size_t>(n_bodies));
  if ((st = hip_check(hipMemcpyAsync(hc.data(), dcnt, hc.size() * sizeof(int64_t),
                                     hipMemcpyDeviceToHost, stream),
                      "read counters")) ||
      (st = hip_check(hipMemcpyAsync(hv.data(), dvol, hv.size() * sizeof(double),
                                     hipMemcpyDeviceToHost, stream),
                      "read volumes")) ||
      (st = hip_check(hipStreamSynchronize(stream), "sync")))
    return st;
  for (int32_t b = 0; b < n_bodies; ++b) {
    out[b].tets = hc[4 * size_t(b) + 0];
    out[b].zero_tets = hc[4 * size_t(b) + 1];
    out[b].pairs = hc[4 * size_t(b) + 2];
    out[b].pieces = hc[4 * size_t(b) + 3];
    out[b].volume = hv[size_t(b)];
  }
  return IBVT_OK;
}

int ibvt_set_allocator(const ibvt_alloc* a) {
  if (a && (!a->alloc || !a->free))
    return set_error(IBVT_E_INVALID, "an allocator needs both alloc and free");
  std::lock_guard<std::mutex> g(g_alloc_mu);
  g_alloc = a ? *a : ibvt_alloc{};
  return IBVT_OK;
}

void coupling_free(ibvt_coupling* c) {
  if (!c) return;
  (void)hipDeviceSynchronize();
  c->stream = nullptr;  // the caller's streams may be gone: free on the null stream
  release_all(c);
  (void)hipStreamSynchronize(nullptr);
  for (hipEvent_t e : {c->ev_fork, c->ev_join, c->ev_sorted})
    if (e) (void)hipEventDestroy(e);
  if (c->side) (void)hipStreamDestroy(c->side);
  delete c;
}

}  // extern "C"
