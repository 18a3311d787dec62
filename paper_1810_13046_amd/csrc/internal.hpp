// Internal (non-ABI) declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/ibvt.h"
#include "common.hpp"

namespace ibvt {

// Grow-only device buffer.
struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
  template <typename T>
  T* as() const { return static_cast<T*>(p); }
};

struct Csr {
  int64_t nrows = 0;
  int64_t nnz = 0;
  DevBuf rowptr;  // int64 (nrows + 1)
  DevBuf col;     // int32 (nnz)
  DevBuf val;     // double or float (nnz)
  DevBuf rowmap;  // int32 (nrows), transposed matrices only
};

// Lattice description passed by value to kernels: 9 coordinate arrays
// (component d, axis e) concatenated in one device buffer.
struct LatDesc {
  int32_t off[9];
  int32_t n[9];
};

// Cell of pair p (component d, tet t, cell index ci) and its box [lo, hi].
__device__ __forceinline__ void pair_cell(int64_t p, int64_t n_t, const int32_t* owner,
                                          const int64_t* pair_off, const CellRange* rng,
                                          const double* lat, const LatDesc& ld, int& d,
                                          int64_t& t, int ci[3], double lo[3], double hi[3]) {
  const int64_t tc = owner[p];
  d = (tc >= n_t) + (tc >= 2 * n_t);
  t = tc - int64_t(d) * n_t;
  const CellRange r = rng[tc];
  // cell counts per tet are small: 32-bit index arithmetic
  const uint32_t q = uint32_t(p - pair_off[tc]);
  const uint32_t n0 = uint32_t(r.n[0]), n1 = uint32_t(r.n[1]);
  const uint32_t qy = q / n0;
  ci[0] = r.lo[0] + int(q - qy * n0);
  const uint32_t qz = qy / n1;
  ci[1] = r.lo[1] + int(qy - qz * n1);
  ci[2] = r.lo[2] + int(qz);
  for (int e = 0; e < 3; ++e) {
    const double* L = lat + ld.off[3 * d + e];
    lo[e] = L[ci[e]];
    hi[e] = L[ci[e] + 1];
  }
}

// A (tet, component, cell) pair as the clip reads it: the pair's index,
// the tet and component (t | d << 30) and the cell (three lattice indices of
// kCellBits bits).  Written next to the sort key and carried by the sort
// into clip order, so the clip reads one 16-byte word per pair.
struct PairDesc {
  int32_t p;
  uint32_t td;
  uint64_t cell;
};
constexpr int kCellBits = 21;
constexpr int64_t kMaxDescTets = int64_t(1) << 30;

__device__ __forceinline__ PairDesc pair_desc(int64_t p, int64_t n_t, const int32_t* owner,
                                              const int64_t* pair_off, const CellRange* rng) {
  const int64_t tc = owner[p];
  const int d = (tc >= n_t) + (tc >= 2 * n_t);
  const int64_t t = tc - int64_t(d) * n_t;
  const CellRange r = rng[tc];
  const uint32_t q = uint32_t(p - pair_off[tc]);
  const uint32_t n0 = uint32_t(r.n[0]), n1 = uint32_t(r.n[1]);
  const uint32_t qy = q / n0, qz = qy / n1;
  PairDesc o;
  o.p = int32_t(p);
  o.td = uint32_t(t) | (uint32_t(d) << 30);
  o.cell = uint64_t(uint32_t(r.lo[0]) + (q - qy * n0)) |
           (uint64_t(uint32_t(r.lo[1]) + (qy - qz * n1)) << kCellBits) |
           (uint64_t(uint32_t(r.lo[2]) + qz) << (2 * kCellBits));
  return o;
}

// Cell of a described pair and its box [lo, hi].
__device__ __forceinline__ void desc_cell(const PairDesc& q, const double* lat, const LatDesc& ld,
                                          int64_t& p, int& d, int64_t& t, int ci[3], double lo[3],
                                          double hi[3]) {
  constexpr uint64_t m = (uint64_t(1) << kCellBits) - 1;
  p = q.p;
  d = int(q.td >> 30);
  t = int64_t(q.td & ((1u << 30) - 1u));
  ci[0] = int(q.cell & m);
  ci[1] = int((q.cell >> kCellBits) & m);
  ci[2] = int(q.cell >> (2 * kCellBits));
  for (int e = 0; e < 3; ++e) {
    const double* L = lat + ld.off[3 * d + e];
    lo[e] = L[ci[e]];
    hi[e] = L[ci[e] + 1];
  }
}

struct AsmStats {
  int64_t pairs = 0, pieces = 0, dropped = 0, zero_tets = 0, subtets = 0;
  int64_t dist_evals = 0, cut_points = 0;  // clip work of the last assembly
  int64_t plane_cuts = 0;                  // (pair, cell plane) clips it ran
  int64_t assemblies = 0;
};

}  // namespace ibvt

struct ibvt_coupling {
  hipStream_t stream = nullptr;  // stream of the current call: buffers grow and shrink on it
  ibvt_alloc alloc{};            // allocator of the handle's buffers (null: hipMallocAsync)
  hipStream_t side = nullptr;    // the assembly's second stream (default priority), and
  hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_sorted = nullptr;  // its joins
  int precision = IBVT_FP64;
  uint32_t flags = 0;
  int dim = 3;    // 3: tetrahedra in a 3D grid; 2: triangles in a planar grid
  int ncomp = 3;  // velocity components (= dim)
  bool unstructured = false;  // P1 tetrahedral fluid mesh instead of a grid: one B,
                              // shared by the three components (B[1], B[2] alias B[0])
  int64_t n_fvert = 0, n_ftet = 0;  // fluid mesh sizes (unstructured)
  ibvt::DevBuf fX, ftets;    // fluid mesh copies (unstructured)
  ibvt::DevBuf frec, fbox;   // fluid tet records (vertex 0, ∇μ) and double boxes
  ibvt::DevBuf forder;       // fluid tets in Morton order
  ibvt::DevBuf ftree;        // float boxes of the implicit tree (8 per node)
  int64_t ftree_leaves = 0;  // leaves of the tree (power of two)
  ibvt::DevBuf ucoo;         // sort scratch of the unstructured assembly
  int64_t n_vert = 0, n_tet = 0;  // n_tet counts the elements (triangles when dim = 2)
  int32_t n_cells[3] = {0, 0, 0};
  std::vector<double> lat_host[9];
  ibvt::LatDesc ld{};
  int64_t n_fluid[3] = {0, 0, 0};
  ibvt::DevBuf lat;          // double, concatenated lattices
  ibvt::DevBuf X, tets;      // own copies
  ibvt::DevBuf vt_ptr, vt_tet;  // vertex -> incident tets (int64 ptr, int32 ids)
  ibvt::DevBuf tetvol;       // double n_tet
  ibvt::DevBuf tetrec;       // double n_tet*16: per-tet record (vertices, determinant);
                             // per triangle: 8 (vertices, determinant) when dim = 2
  ibvt::DevBuf tetgrad;      // double n_tet*12: ∇λ_i of every tet
  ibvt::DevBuf mcoef;        // double 3*n_tet: mass-term coefficients (reverse mode)
  ibvt::DevBuf fsiX;         // double 3*n_vert: configuration of the coupling step
  ibvt::DevBuf fsinorm;      // double: Step-6 norm partials
  ibvt::DevBuf fvol;         // double: 1D Q1 lumped weights of the three lattices
  bool fvol_ready = false;
  ibvt::DevBuf rng;          // CellRange 3*n_tet
  ibvt::DevBuf cnt;          // int64 3*n_tet
  ibvt::DevBuf pair_off;     // int64 3*n_tet + 1
  int64_t n_pairs = 0;
  ibvt::DevBuf owner;        // int32 n_pairs
  ibvt::DevBuf pval;         // T: one chunk's pairs x 32 (grid), n_pairs*12 (dim = 2),
                             // 3*n_tet*4 per-tet sums (matrix-free)
  ibvt::DevBuf pmom;         // T n_pairs*kMomPad: per-pair piece moments (reverse mode)
  ibvt::DevBuf keep;         // uint8 n_pairs
  bool store_pieces = true;  // keep the moments of every piece (reverse mode)
  bool matrix_free = false;  // IBVT_NO_STORE_B: no B, B^T or per-pair data; products clip again
  bool dual = false;         // B holds the dual-multiplier integrals ∫ ψ_i N_j
  ibvt::DevBuf pool;         // T records of kRecord values
  int64_t pool_cap = 0;      // records
  int64_t pool_needed = 0;   // records the last assembly asked for
  bool mom_valid = false;    // pmom holds the moments of every kept piece of the last assembly
  bool ready = false;        // the last assembly completed: B, B^T and the masses are usable
  ibvt::DevBuf pinfo;        // uint64 n_pairs: first record << 8 | records (0: dropped)
  ibvt::DevBuf order;        // int32 n_pairs: pairs sorted by cut pattern
  ibvt::DevBuf pscan;        // sort keys and scratch
  ibvt::DevBuf tcorder;      // int32 3*n_tet: (component, tet) items by pair count
  bool tcorder_valid = false;  // tcorder belongs to the last assembly
  ibvt::DevBuf rownnz;       // int64 3*n_vert
  ibvt::DevBuf rowbox;       // node box per (vertex, component)
  ibvt::DevBuf rowcap;       // int64 box size per row
  ibvt::DevBuf rowtmpoff;    // int64 offsets into the row scratch
  ibvt::DevBuf rowtmpcol;    // int32 row scratch columns
  ibvt::DevBuf rowtmpval;    // T row scratch values
  ibvt::DevBuf rowspilloff;  // int64 offsets of the rows' spill space
  ibvt::DevBuf rowspill;     // double partial node sums + uint8 touched flags of rows that
                             // take pairs of several chunks
  ibvt::Csr B[3], Bt[3];
  ibvt::DevBuf mark;         // int32 n_fluid + 1 (transposes of small operators)
  ibvt::DevBuf cidx;         // int64 n_fluid + 1 (transposes of small operators)
  ibvt::DevBuf tbuf;         // transpose scratch (bucket records and tables)
  ibvt::DevBuf mlump;        // double n_vert
  ibvt::DevBuf minv;         // T n_vert
  bool has_M = false;
  ibvt::Csr M;               // consistent mass (double values)
  ibvt::DevBuf Mval32;       // float copy of M values (mixed precision)
  ibvt::DevBuf Mdiag_inv;    // double n_vert
  ibvt::DevBuf flags_dev;    // unsigned
  ibvt::DevBuf counters;     // unsigned long long kCntSlots
  ibvt::DevBuf scan_tmp;     // scan scratch
  ibvt::DevBuf work;         // transfer scratch (mass-solve vectors etc.)
  ibvt::DevBuf work2;        // shape-gradient per-pair scratch / mass-solve right-hand side
  ibvt::DevBuf zbuf;         // solid-sized scratch of the reverse-mode calls
  int64_t* host_rb = nullptr;  // pinned host block of the packed read-backs (hipHostMalloc)
  ibvt::DevBuf rb;           // device block gathered for one read-back
  ibvt::DevBuf bodyinfo;     // coupling_body_info: offsets and per-body sums
  unsigned host_flags = 0;   // status flags of the last packed read-back
  ibvt::AsmStats stats;
  int64_t device_bytes = 0;
};

namespace ibvt {

// Kernel tracing: records an event pair around a launch when enabled.
struct ProfScope {
  int slot = -1;
  hipStream_t s = nullptr;
  ProfScope(const char* name, hipStream_t stream);
  ~ProfScope();
};

// status helpers (api.hip)
int set_error(int status, const std::string& msg);
int hip_check(hipError_t e, const char* what);
int ensure(ibvt_coupling* c, DevBuf& b, size_t bytes);
void release(ibvt_coupling* c, DevBuf& b);

// scan.hip: exclusive prefix sum; out has n+1 entries, out[n] = total.
int scan_i64(ibvt_coupling* c, const int64_t* in, int64_t* out, int64_t n, hipStream_t s);
int scan_i32_to_i64(ibvt_coupling* c, const int32_t* in, int64_t* out, int64_t n, hipStream_t s);

// assemble.hip
int build_topology(ibvt_coupling* c, hipStream_t s);  // dim + 1 vertices per element
int assemble_all(ibvt_coupling* c, hipStream_t s);    // dispatches on dim
int read_back(ibvt_coupling* c, void* host, const void* dev, size_t bytes, hipStream_t s);
int check_flags(ibvt_coupling* c, hipStream_t s);
// One stream synchronisation for several device counts: out[k] = *srcs[k]
// (n <= 24 int64 values) and the status flag word into c->host_flags.
int read_counts(ibvt_coupling* c, const int64_t* const* srcs, int n, int64_t* out, hipStream_t s);
// Status of a flag word (IBVT_OK when no flag is set).
int flags_status(unsigned f);
// lumped (and, when built, consistent) mass of the solid tets from tetvol
int solid_masses(ibvt_coupling* c, hipStream_t s);

// unstructured.hip: P1 tetrahedral fluid background (tree search + general
// tet ∩ tet clipping); the fluid tree is built once per handle
int build_fluid_tree(ibvt_coupling* c, hipStream_t s);
int assemble_all_unstructured(ibvt_coupling* c, hipStream_t s);
// unstructured.hip: g_X += alpha (shape terms of (z, u) [− mass term of
// (z, us) when mass >= 0]) from the stored per-pair integrals
int shape_gradient_unstructured(ibvt_coupling* c, const void* z, const void* const u[3],
                                const void* us, int mass, double alpha, double* gX,
                                hipStream_t s);
// both adjoints in one pass: (z, u) with the mass term of (z, us), plus
// alpha2 · (z2, v)
int shape_gradient_unstructured_two(ibvt_coupling* c, const void* z, const void* const u[3],
                                    const void* us, int mass, const void* z2,
                                    const void* const v[3], double alpha2, double* gX,
                                    hipStream_t s);

// assemble2d.hip: the planar coupling (Q1 quadrilateral lattice x P1 triangles)
int assemble_all_2d(ibvt_coupling* c, hipStream_t s);
int shape_gradient_2d(ibvt_coupling* c, const void* z, const void* const u[3], const void* us,
                      int mass, double alpha, double* gX, hipStream_t s);

// transpose.hip
template <typename T>
int transpose_one(ibvt_coupling* c, int d, hipStream_t s);

// sort.hip: stable sorts by small integer keys (n < 2^31).
// A nonzero carried through the small operators' transpose: its value and
// its row.
struct SortVal32 {
  float v;
  int32_t r;
};
struct SortVal64 {
  double v;
  int32_t r;
};
// tiles of a pass over n items carrying values of value_bytes bytes
int64_t sort_tiles(int64_t n, int value_bytes = 16);
// scratch bytes of one digit pass over n items with 2^bits digits
size_t sort_pass_bytes(int64_t n, int bits);
// after a pass with 2^bits digits over n items: the first output position
// of digit k is at [k * sort_tiles(n, value_bytes)] of this array
// (device); entry 2^bits * sort_tiles(n, value_bytes) holds n
const int64_t* sort_digit_starts(const void* scratch, int64_t n, int bits, int value_bytes = 16);
// order = the indices 0..n-1 stably sorted by their 8-bit keys
int order_by_byte_key(ibvt_coupling* c, int64_t n, const uint8_t* keys, int32_t* order,
                      void* scratch, hipStream_t s);

// apply.hip
int apply_B(ibvt_coupling* c, const void* const x[3], void* y, bool lumped_scale, hipStream_t s);
int apply_Bt(ibvt_coupling* c, const void* ys, void* const out[3], double alpha, hipStream_t s);
// ws: null (the coupling's own buffer, grown as needed) or device memory of
// at least mass_solve_workspace_bytes(c) bytes that the solve uses instead
// (then it allocates nothing)
int mass_solve(ibvt_coupling* c, const void* rhs, void* x, double rtol, int maxit,
               hipStream_t s, ibvt_solve_info* info, bool x_has_guess, char* ws = nullptr);
size_t mass_solve_workspace_bytes(const ibvt_coupling* c);
int lumped_solve(ibvt_coupling* c, const void* rhs, void* x, hipStream_t s);
int axpy_solid(ibvt_coupling* c, double alpha, const void* x, void* y, hipStream_t s);

// matfree.hip: the products and the shape gradient of a coupling built with
// IBVT_NO_STORE_B, clipping and integrating every piece again
// sort the (component, tet) items of a matrix-free coupling by slot class
// and cell count (into c->order, with the class bounds after the indices)
int matfree_order(ibvt_coupling* c, hipStream_t s);
int apply_B_matfree(ibvt_coupling* c, const void* const x[3], void* y, bool lumped_scale,
                    hipStream_t s);
int apply_Bt_matfree(ibvt_coupling* c, const void* ys, void* const out[3], double alpha,
                     hipStream_t s);
int shape_gradient_matfree(ibvt_coupling* c, const void* z, const void* const u[3],
                           const void* us, int mass, double alpha, double* gX, hipStream_t s);

// grad.hip
int shape_gradient(ibvt_coupling* c, const void* z, const void* const u[3], const void* us,
                   int mass, double alpha, double* gX, hipStream_t s);
// g_X += alpha Σ (per-(component, tet) pair terms pgt[(d, t)][12] − mass
// term of (z, us) when mass >= 0), gathered per vertex in a fixed order;
// grad: ∇λ of every tet, 12 doubles at stride gstride.
int shape_gather(ibvt_coupling* c, const double* pgt, const void* z, const void* us, int mass,
                 double alpha, double* gX, const double* grad, int gstride, hipStream_t s);
// both adjoints' shape terms in one pass over the stored piece moments:
// (z, u) with the mass term of (z, us), plus alpha2 · (z2, v)
int shape_gradient_two(ibvt_coupling* c, const void* z, const void* const u[3], const void* us,
                       int mass, const void* z2, const void* const v[3], double alpha2,
                       double* gX, hipStream_t s);

}  // namespace ibvt
