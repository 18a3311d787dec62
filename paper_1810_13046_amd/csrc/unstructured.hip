// Coupling with an unstructured fluid background: a P1 tetrahedral fluid
// mesh against the P1 tetrahedral solid mesh.  Section 2.3 builds the
// transfer between unstructured and structured meshes in four steps: (I) a
// tree search for the overlapping elements, (II)-(III) integration of the
// products of the two element bases on their intersections (piecewise
// affine meshes), (IV) assembly of the mortar matrices.  The fluid space
// is P1 on the fluid tets and collocated, so one B serves the three
// velocity components.
//
//  k_tet_rec        per tet of either mesh: double bounding box and record
//                   (vertices, ∇ of the four hats, determinant); a hat is
//                   λ_k(x) = δ_k0 + ∇λ_k·(x − V0).
//  k_box_partials / k_box_final
//                   bounding box of the fluid mesh (fixed-order reduction).
//  k_morton         30-bit Morton code of each fluid box centre; radix sort.
//  k_tree_leaves / k_tree_level
//                   an implicit binary tree over the sorted fluid tets
//                   (heap layout, a power of two of leaves): leaf boxes, then
//                   one launch per level up to the root (union of the two
//                   children; float boxes rounded outward, so every box
//                   contains its double one).  Built once per handle: the
//                   fluid mesh does not move.
//  k_search<MODE>   per solid tet: depth-first traversal with an explicit
//                   stack; leaves compared with the exact double boxes; one
//                   pass counts and keeps up to kSearchCap finds per tet,
//                   prefix sum, copy into place (traversal order); a second
//                   traversal fills in place when some tet found more.
//  k_sep_u / scan / k_list_u
//                   candidates that a face plane of either tet separates
//                   (all four vertices of one strictly outside a face of the
//                   other) get keep = 0; the others are listed for the clip.
//  k_pairs_u<T>     one lane per listed (solid tet, fluid tet) pair: the solid tet
//                   clipped by the fluid tet's four half-spaces μ_k >= 0
//                   (vertex graph in LDS, general planes), fanned into
//                   sub-tetrahedra, ∫ λ_i μ_j integrated exactly on each
//                   (the product of two affine factors:
//                   ∫_τ f g = |τ|/20 (Σ_v f_v g_v + Σ_v f_v Σ_v g_v)).
//  k_row_cap_u / k_rows_u<T> / k_rows_compact_u<T>
//                   one wavefront per solid vertex: the kept pairs of its
//                   incident tets in generation order, their entries summed
//                   per fluid vertex in an LDS hash (pair order), the row
//                   written sorted -> CSR rows of B (deterministic).
//  k_coo / sort / k_runs
//                   for rows too wide for the LDS gather: the 16 entries of
//                   every kept pair keyed by (solid vertex, fluid vertex),
//                   stable radix sort over the key's used bits, one lane per
//                   run of equal keys sums it in order (the same sums).
#include <hipcub/hipcub.hpp>

#include "internal.hpp"
#include "tetpair.hpp"

#include <cfloat>

namespace ibvt {

namespace {

// Depth-first stack of the tree search: one pending sibling per level at
// most, and the tree has at most 2^31 leaves (31 levels).
constexpr int kTreeStack = 32;
constexpr int kSearchThreads = 256;
// Finds per solid tet that the first search pass keeps (beyond it, a second
// traversal fills the pairs in place).
constexpr int kSearchCap = 64;

inline unsigned blocks_for(int64_t n, int threads) {
  return unsigned(ceil_div(n > 0 ? n : 1, threads));
}

// Per tet: box (mn, mx; 8 doubles with padding), record, volume (solid
// mesh only: vol != null); flags non-finite coordinates and bad indices.
__global__ void k_tet_rec(int64_t n_t, int64_t n_v, const double* __restrict__ X,
                          const int32_t* __restrict__ tets, double* __restrict__ box,
                          double* __restrict__ rec, double* __restrict__ vol, unsigned* flags) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= n_t) return;
  TetGeom G;
  bool ok = true, bad_index = false;
  for (int k = 0; k < 4; ++k) {
    const int64_t v = tets[4 * t + k];
    if (v < 0 || v >= n_v) {
      bad_index = true;
      ok = false;
      break;
    }
    for (int e = 0; e < 3; ++e) {
      G.V[k][e] = X[3 * v + e];
      ok &= isfinite(G.V[k][e]);
    }
  }
  if (!ok) {
    atomicOr(flags, bad_index ? kFlagValence : kFlagNonFinite);
    for (int k = 0; k < 8; ++k) box[8 * t + k] = 0.0;
    for (int k = 0; k < kURec; ++k) rec[kURec * t + k] = 0.0;
    if (vol) vol[t] = 0.0;
    return;
  }
  tet_geom(G);
  double b[8] = {G.mn[0], G.mn[1], G.mn[2], 0.0, G.mx[0], G.mx[1], G.mx[2], 0.0};
  store_row<8>(box + 8 * t, b);
  double r[kURec];
  for (int k = 0; k < 4; ++k)
    for (int e = 0; e < 3; ++e) {
      r[3 * k + e] = G.V[k][e];
      r[12 + 3 * k + e] = G.g[k][e];
    }
  r[24] = G.det;
  r[25] = r[26] = r[27] = 0.0;
  store_row<kURec>(rec + kURec * t, r);
  if (vol) vol[t] = fabs(G.det) / 6.0;
}

// Bounding box of all fluid boxes: per-block partials, then one block.
__global__ __launch_bounds__(256) void k_box_partials(int64_t n, const double* __restrict__ box,
                                                      double* __restrict__ part) {
  __shared__ double red[6][256 / kWave];
  double m[6] = {DBL_MAX, DBL_MAX, DBL_MAX, -DBL_MAX, -DBL_MAX, -DBL_MAX};
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < n;
       t += int64_t(gridDim.x) * blockDim.x)
    for (int e = 0; e < 3; ++e) {
      m[e] = fmin(m[e], box[8 * t + e]);
      m[3 + e] = fmax(m[3 + e], box[8 * t + 4 + e]);
    }
  for (int o = 32; o > 0; o >>= 1)
    for (int e = 0; e < 3; ++e) {
      m[e] = fmin(m[e], __shfl_xor(m[e], o, kWave));
      m[3 + e] = fmax(m[3 + e], __shfl_xor(m[3 + e], o, kWave));
    }
  if (lane_id() == 0)
    for (int e = 0; e < 6; ++e) red[e][threadIdx.x / kWave] = m[e];
  __syncthreads();
  if (threadIdx.x < 6) {
    double v = red[threadIdx.x][0];
    for (int w = 1; w < 256 / kWave; ++w)
      v = threadIdx.x < 3 ? fmin(v, red[threadIdx.x][w]) : fmax(v, red[threadIdx.x][w]);
    part[6 * blockIdx.x + threadIdx.x] = v;
  }
}

__global__ void k_box_final(int nb, const double* __restrict__ part, double* __restrict__ bb) {
  if (threadIdx.x >= 6) return;
  double v = part[threadIdx.x];
  for (int b = 1; b < nb; ++b)
    v = threadIdx.x < 3 ? fmin(v, part[6 * b + threadIdx.x]) : fmax(v, part[6 * b + threadIdx.x]);
  bb[threadIdx.x] = v;
}

__device__ __forceinline__ uint32_t spread10(uint32_t v) {
  v &= 0x3ffu;
  v = (v | (v << 16)) & 0x030000ffu;
  v = (v | (v << 8)) & 0x0300f00fu;
  v = (v | (v << 4)) & 0x030c30c3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

__global__ void k_morton(int64_t n, const double* __restrict__ box, const double* __restrict__ bb,
                         uint32_t* __restrict__ code, int32_t* __restrict__ idx) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= n) return;
  uint32_t q[3];
  for (int e = 0; e < 3; ++e) {
    const double c = 0.5 * (box[8 * t + e] + box[8 * t + 4 + e]);
    const double ext = bb[3 + e] - bb[e];
    const double u = ext > 0.0 ? (c - bb[e]) / ext : 0.0;
    q[e] = uint32_t(fmin(fmax(u * 1024.0, 0.0), 1023.0));
  }
  code[t] = (spread10(q[0]) << 2) | (spread10(q[1]) << 1) | spread10(q[2]);
  idx[t] = int32_t(t);
}

// Leaves of the implicit tree (node P - 1 + i): the box of the i-th fluid
// tet in Morton order, rounded outward to float; empty beyond n.
__global__ void k_tree_leaves(int64_t n, int64_t P, const int32_t* __restrict__ order,
                              const double* __restrict__ box, float* __restrict__ tree) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= P) return;
  float b[8];
  if (i < n) {
    const int64_t t = order[i];
    for (int e = 0; e < 3; ++e) {
      b[e] = __double2float_rd(box[8 * t + e]);
      b[4 + e] = __double2float_ru(box[8 * t + 4 + e]);
    }
  } else {
    for (int e = 0; e < 3; ++e) {
      b[e] = FLT_MAX;
      b[4 + e] = -FLT_MAX;
    }
  }
  b[3] = b[7] = 0.0f;
  store_row<8>(tree + 8 * (P - 1 + i), b);
}

// Nodes [first, first + count) of one level: union of the children.
__global__ void k_tree_level(int64_t first, int64_t count, float* __restrict__ tree) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= count) return;
  const int64_t node = first + k;
  float a[8], b[8];
  load_row<8>(tree + 8 * (2 * node + 1), a);
  load_row<8>(tree + 8 * (2 * node + 2), b);
  for (int e = 0; e < 3; ++e) {
    a[e] = fminf(a[e], b[e]);
    a[4 + e] = fmaxf(a[4 + e], b[4 + e]);
  }
  store_row<8>(tree + 8 * node, a);
}

__device__ __forceinline__ bool boxes_meet(const double mn[3], const double mx[3],
                                           const float* __restrict__ b) {
  return mx[0] >= double(b[0]) && mn[0] <= double(b[4]) && mx[1] >= double(b[1]) &&
         mn[1] <= double(b[5]) && mx[2] >= double(b[2]) && mn[2] <= double(b[6]);
}

// Tree search per solid tet.  FILL = false: count the fluid tets whose
// closed double box meets the solid tet's; FILL = true: write them at
// off[s] in traversal (Morton) order.
// MODE 0: count the finds of each solid tet (cnt); MODE 1: write them at
// off[s] (pf); MODE 2: count them and keep the first kSearchCap at
// tmp[s * kSearchCap] (*ovf = 1 when a tet has more).
template <int MODE>
__global__ __launch_bounds__(kSearchThreads) void k_search(int64_t n_s, const double* __restrict__ sbox,
                                                int64_t P, int64_t n_f,
                                                const float* __restrict__ tree,
                                                const int32_t* __restrict__ order,
                                                const double* __restrict__ fbox,
                                                int64_t* __restrict__ cnt,
                                                const int64_t* __restrict__ off,
                                                int32_t* __restrict__ pf, unsigned* flags,
                                                int32_t* __restrict__ tmp, unsigned* ovf) {
  constexpr bool FILL = MODE == 1;
  // the stacks live in LDS, entry k of thread j at k * kSearchThreads + j
  __shared__ uint32_t s_stack[kTreeStack * kSearchThreads];
  uint32_t* stack = s_stack + threadIdx.x;
  const int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s >= n_s) return;
  double mn[3], mx[3];
  for (int e = 0; e < 3; ++e) {
    mn[e] = sbox[8 * s + e];
    mx[e] = sbox[8 * s + 4 + e];
  }
  int top = 0;
  int64_t found = 0;
  int64_t pos = FILL ? off[s] : 0;
  if (boxes_meet(mn, mx, tree)) stack[kSearchThreads * top++] = 0u;
  while (top > 0) {
    const int64_t node = stack[kSearchThreads * --top];
    if (node >= P - 1) {
      const int64_t i = node - (P - 1);
      if (i >= n_f) continue;
      const int64_t t = order[i];
      const double* fb = fbox + 8 * t;
      if (mx[0] >= fb[0] && mn[0] <= fb[4] && mx[1] >= fb[1] && mn[1] <= fb[5] &&
          mx[2] >= fb[2] && mn[2] <= fb[6]) {
        if (FILL) pf[pos++] = int32_t(t);
        if (MODE == 2 && found < kSearchCap) tmp[s * kSearchCap + found] = int32_t(t);
        ++found;
      }
      continue;
    }
    const int64_t l = 2 * node + 1, r = 2 * node + 2;
    const bool gl = boxes_meet(mn, mx, tree + 8 * l), gr = boxes_meet(mn, mx, tree + 8 * r);
    if (top + 2 > kTreeStack) {
      atomicOr(flags, kFlagCapacity);
      return;
    }
    if (gr) stack[kSearchThreads * top++] = uint32_t(r);
    if (gl) stack[kSearchThreads * top++] = uint32_t(l);
  }
  if (!FILL) cnt[s] = found;
  if (MODE == 2 && found > kSearchCap) atomicOr(ovf, 1u);
}

// pf[off[s] + k] = tmp[s * kSearchCap + k] for the finds of each solid tet.
__global__ void k_search_copy(int64_t n_s, const int64_t* __restrict__ off,
                              const int32_t* __restrict__ tmp, int32_t* __restrict__ pf) {
  const int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s >= n_s) return;
  const int64_t o = off[s], n = off[s + 1] - o;
  for (int64_t k = 0; k < n; ++k) pf[o + k] = tmp[s * kSearchCap + k];
}

// Owner solid tet of pair p: the last s with off[s] <= p.
__device__ __forceinline__ int64_t pair_owner(int64_t p, int64_t n_s,
                                              const int64_t* __restrict__ off) {
  int64_t lo = 0, hi = n_s;
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (off[mid] <= p) lo = mid;
    else hi = mid;
  }
  return lo;
}

// True when the four vertices of tet record b lie strictly outside one
// face plane of tet record a (a's hat λ_k < 0 at all of them, evaluated as
// the clip evaluates it): the two tets are then disjoint.
__device__ __forceinline__ bool face_separates(const double* __restrict__ a,
                                               const double* __restrict__ b) {
  double v[4][3];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int e = 0; e < 3; ++e) v[q][e] = b[3 * q + e];
  const double a0[3] = {a[0], a[1], a[2]};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double* gk = a + 12 + 3 * k;
    const double d0 = (k == 0) ? 1.0 : 0.0;
    bool out = true;
#pragma unroll
    for (int q = 0; q < 4; ++q)
      out &= d0 + gk[0] * (v[q][0] - a0[0]) + gk[1] * (v[q][1] - a0[1]) +
                 gk[2] * (v[q][2] - a0[2]) < 0.0;
    if (out) return true;
  }
  return false;
}

// One lane per candidate pair: cand = 0 (and keep = 0) when a face plane of
// either tet separates them; those pairs are not clipped.
__global__ void k_sep_u(int64_t n_pairs, int64_t n_s, const int64_t* __restrict__ off,
                        const int32_t* __restrict__ pf, const double* __restrict__ srec,
                        const double* __restrict__ frec, int32_t* __restrict__ cand,
                        uint8_t* __restrict__ keep) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= n_pairs) return;
  const int64_t s = pair_owner(p, n_s, off);
  const int64_t f = pf[p];
  const double* rs = srec + kURec * s;
  const double* rf = frec + kURec * f;
  const bool sep = face_separates(rf, rs) || face_separates(rs, rf);
  cand[p] = sep ? 0 : 1;
  if (sep) keep[p] = 0;
}

// list[pos[p]] = p for the pairs left to clip.
__global__ void k_list_u(int64_t n_pairs, const int32_t* __restrict__ cand,
                         const int64_t* __restrict__ pos, int32_t* __restrict__ list) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p < n_pairs && cand[p]) list[pos[p]] = int32_t(p);
}

// One lane per pair: the solid tet clipped by the fluid tet's four
// half-spaces μ_k >= 0, fanned, and ∫ λ_i μ_j integrated exactly on each
// sub-tetrahedron; vals[pair][i*4 + j] (dual: 5 b_i − Σ_k b_k), keep =
// piece volume > drop_rel |T|.  Arithmetic in double (coordinates relative
// to the solid tet's vertex 0); values stored as T.
template <typename T>
__global__ __launch_bounds__(kWave) void k_pairs_u(
    int64_t n_list, const int32_t* __restrict__ list, int64_t n_s, const int64_t* __restrict__ off,
    const int32_t* __restrict__ pf, const double* __restrict__ srec,
    const double* __restrict__ frec, double drop_rel, int dual, uint8_t* __restrict__ keep,
    T* __restrict__ vals, T* __restrict__ lams, unsigned* flags, unsigned long long* counters) {
  __shared__ double sx[kUSlots * kWave], sy[kUSlots * kWave], sz[kUSlots * kWave];
  __shared__ uint32_t snb[kUSlots * kWave];
  const int lane = threadIdx.x;
  const PolyView P{sx + lane, sy + lane, sz + lane, snb + lane, kWave, (1u << kUSlots) - 1u};
  const int64_t q = int64_t(blockIdx.x) * kWave + lane;
  bool kept = false, dropped = false, fail = false;
  if (q < n_list) {
    const int64_t p = list[q];
    const int64_t s = pair_owner(p, n_s, off);
    const int64_t f = pf[p];
    double rs[kURec], rf[kURec];
    load_row<kURec>(srec + kURec * s, rs);
    load_row<kURec>(frec + kURec * f, rf);
    double acc[16], lam[10];
    double vol = 0.0;
    fail = !tet_pair_values(P, rs, rf, acc, vol, lam);
    kept = !fail && vol > drop_rel * fabs(rs[24]) / 6.0;
    dropped = !fail && !kept && vol > 0.0;
    if (kept && dual) {
      for (int j = 0; j < 4; ++j) {
        const double sj = acc[j] + acc[4 + j] + acc[8 + j] + acc[12 + j];
        for (int i = 0; i < 4; ++i) acc[4 * i + j] = 5.0 * acc[4 * i + j] - sj;
      }
    }
    T out[16];
    for (int k = 0; k < 16; ++k) out[k] = kept ? T(acc[k]) : T(0);
    store_row<16>(vals + 16 * p, out);
    T lo[kULam];
    for (int k = 0; k < kULam; ++k) lo[k] = (kept && k < 10) ? T(lam[k]) : T(0);
    store_row<kULam>(lams + kULam * p, lo);
    keep[p] = kept ? 1 : 0;
  }
  const uint64_t km = ballot64(kept), dm = ballot64(dropped), fm = ballot64(fail);
  if (lane == 0) {
    if (km) atomicAdd(&counters[kCntPieces], (unsigned long long)popc64(km));
    if (dm) atomicAdd(&counters[kCntDropped], (unsigned long long)popc64(dm));
    if (fm) atomicOr(flags, kFlagCapacity);
  }
}

// Keys of the 16 entries of every pair (one lane per pair): (solid vertex
// << cb) | fluid vertex for kept pairs (cb bits hold any fluid vertex),
// `none` (row n_vert: after every valid key) otherwise; idx = entry.
__global__ void k_coo(int64_t n_pairs, int64_t n_s, const int64_t* __restrict__ off,
                      const int32_t* __restrict__ pf, const int32_t* __restrict__ tets_s,
                      const int32_t* __restrict__ tets_f, const uint8_t* __restrict__ keep,
                      int cb, uint64_t none, uint64_t* __restrict__ keys,
                      uint32_t* __restrict__ idx) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= n_pairs) return;
  const bool k = keep[p];
  int32_t vs[4] = {0, 0, 0, 0}, vf[4] = {0, 0, 0, 0};
  if (k) {
    const int64_t s = pair_owner(p, n_s, off);
    const int64_t f = pf[p];
    for (int q = 0; q < 4; ++q) {
      vs[q] = tets_s[4 * s + q];
      vf[q] = tets_f[4 * f + q];
    }
  }
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      const int64_t e = 16 * p + 4 * i + j;
      keys[e] = k ? ((uint64_t(uint32_t(vs[i])) << cb) | uint64_t(uint32_t(vf[j]))) : none;
      idx[e] = uint32_t(e);
    }
}

// head[e] = 1 where a run of equal (valid) keys starts.
__global__ void k_run_heads(int64_t n, uint64_t none, const uint64_t* __restrict__ keys,
                            int32_t* __restrict__ head) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const uint64_t k = keys[e];
  head[e] = (k < none && (e == 0 || keys[e - 1] != k)) ? 1 : 0;
}

// One lane per run: the run's values summed in sorted (= generation)
// order; column and row of the entry.
template <typename T>
__global__ void k_run_sums(int64_t n, int cb, const uint64_t* __restrict__ keys,
                           const uint32_t* __restrict__ idx, const int32_t* __restrict__ head,
                           const int64_t* __restrict__ pos, const T* __restrict__ vals,
                           int32_t* __restrict__ col, int32_t* __restrict__ row,
                           T* __restrict__ val) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= n || !head[e]) return;
  const uint64_t k = keys[e];
  double acc = 0.0;
  for (int64_t q = e; q < n && keys[q] == k; ++q) acc += double(vals[idx[q]]);
  const int64_t u = pos[e];
  col[u] = int32_t(uint32_t(k & ((uint64_t(1) << cb) - 1)));
  row[u] = int32_t(k >> cb);
  val[u] = T(acc);
}

// rowptr[r] = first entry whose row is >= r (rows ascending).
__global__ void k_row_ptr(int64_t n_rows, int64_t nnz, const int32_t* __restrict__ row,
                          int64_t* __restrict__ rowptr) {
  const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r > n_rows) return;
  int64_t lo = 0, hi = nnz;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (row[mid] < r) lo = mid + 1;
    else hi = mid;
  }
  rowptr[r] = lo;
}

// Row scratch bound of each solid vertex: min(kURowMax, 4 x candidate
// pairs of its incident tets) distinct columns.
constexpr int kUHashBits = 9;
constexpr int kUHash = 1 << kUHashBits;  // LDS hash slots per row
constexpr int kURowMax = kUHash / 2;     // distinct columns a row may have here

__global__ void k_row_cap_u(int64_t n_v, const int64_t* __restrict__ vt_ptr,
                            const int32_t* __restrict__ vt_tet,
                            const int64_t* __restrict__ pair_off, int64_t* __restrict__ cap) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n_v) return;
  int64_t n = 0;
  for (int64_t k = vt_ptr[i]; k < vt_ptr[i + 1]; ++k) {
    const int64_t t = vt_tet[k];
    n += pair_off[t + 1] - pair_off[t];
  }
  cap[i] = min<int64_t>(kURowMax, 4 * n);
}

// One wavefront per solid vertex i builds row i of B in LDS.  The row's
// kept pairs are taken in generation order (incident tets ascending, then
// their pairs), 16 per step, one entry per lane (lane = 4·pair + fluid
// corner); the column (fluid vertex) finds its slot in an open-addressing
// hash, and the 16 pairs of a step are added one after another, so every
// column sums its contributions in pair order: the same order, and the
// same double sums, as the sort-based assembly.  The row is written sorted
// by column at tmp_off[i].  A row with more than kURowMax distinct columns
// is counted in counters[kCntRowOverflow] and left empty (the caller then
// assembles B by sorting instead).
template <typename T>
__global__ __launch_bounds__(256) void k_rows_u(
    int64_t n_v, const int64_t* __restrict__ vt_ptr, const int32_t* __restrict__ vt_tet,
    const int32_t* __restrict__ tets_s, const int64_t* __restrict__ pair_off,
    const uint8_t* __restrict__ keep, const int32_t* __restrict__ pf,
    const int32_t* __restrict__ tets_f, const T* __restrict__ pval,
    const int64_t* __restrict__ tmp_off, int32_t* __restrict__ tmp_col, T* __restrict__ tmp_val,
    int64_t* __restrict__ rownnz, unsigned long long* __restrict__ counters) {
  __shared__ int32_t s_key[4][kUHash];
  __shared__ double s_acc[4][kUHash];  // summed in double in both precisions
  __shared__ int32_t s_pbl[4][kWave];  // batch tet: first pair << 2 | local index of i
  __shared__ int32_t s_ex[4][kWave];   // batch tet: exclusive prefix of pair counts
  __shared__ int32_t s_kp[4][kWave];   // kept pairs of a step: pair << 2 | local index
  __shared__ int32_t s_lc[4][kURowMax];
  __shared__ double s_lv[4][kURowMax];
  const int wib = threadIdx.x / kWave;
  const int64_t i = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / kWave;
  const int lane = lane_id();
  if (i >= n_v) return;
  int32_t* key = s_key[wib];
  double* acc = s_acc[wib];
  int32_t* PBL = s_pbl[wib];
  int32_t* EX = s_ex[wib];
  int32_t* KP = s_kp[wib];
  for (int k = lane; k < kUHash; k += kWave) {
    key[k] = -1;
    acc[k] = 0.0;
  }
  int nuniq = 0;
  bool over = false;
  const int64_t beg = vt_ptr[i], end = vt_ptr[i + 1];
  const int u = lane >> 2, j = lane & 3;
  for (int64_t kb = beg; kb < end && !over; kb += kWave) {
    const int nk = int(min<int64_t>(kWave, end - kb));
    int cnt = 0, pbl = 0;
    if (lane < nk) {
      const int64_t t = vt_tet[kb + lane];
      const int4 tv = *reinterpret_cast<const int4*>(tets_s + 4 * t);
      const int li =
          (tv.y == int32_t(i)) ? 1 : (tv.z == int32_t(i)) ? 2 : (tv.w == int32_t(i)) ? 3 : 0;
      const int64_t pb = pair_off[t];
      cnt = int(pair_off[t + 1] - pb);
      pbl = int32_t(pb << 2) | li;
    }
    int incl = cnt;
    for (int o = 1; o < kWave; o <<= 1) {
      const int y = __shfl_up(incl, o, kWave);
      if (lane >= o) incl += y;
    }
    const int tot = __shfl(incl, kWave - 1, kWave);
    wave_lds_sync();
    PBL[lane] = pbl;
    EX[lane] = incl - cnt;
    wave_lds_sync();
    for (int q0 = 0; q0 < tot && !over; q0 += kWave) {
      const int q = q0 + lane;
      bool kept = false;
      int32_t code = 0;
      if (q < tot) {
        // the last batch tet whose pairs start at or before q
        int lo = 0, hi = nk - 1;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (EX[mid] <= q) lo = mid;
          else hi = mid - 1;
        }
        const int32_t m = PBL[lo];
        const int32_t p = (m >> 2) + (q - EX[lo]);
        kept = keep[p] != 0;
        code = (p << 2) | (m & 3);
      }
      const uint64_t km = ballot64(kept);
      const int nkept = popc64(km);
      wave_lds_sync();
      if (kept) KP[rank_below(km)] = code;
      wave_lds_sync();
      for (int s0 = 0; s0 < nkept; s0 += 16) {
        const bool have = s0 + u < nkept;
        int slot = 0;
        bool inserted = false;
        double val = 0.0;
        if (have) {
          const int32_t cd = KP[s0 + u];
          const int64_t p = cd >> 2;
          const int64_t f = pf[p];
          const int32_t cv = tets_f[4 * f + j];
          val = double(pval[16 * p + 4 * (cd & 3) + j]);
          // open addressing; the table is never more than 5/8 full
          uint32_t h = (uint32_t(cv) * 2654435769u) >> (32 - kUHashBits);
          while (true) {
            const int32_t prev = atomicCAS(&key[h], -1, cv);
            if (prev == -1 || prev == cv) {
              slot = int(h);
              inserted = prev == -1;
              break;
            }
            h = (h + 1) & (kUHash - 1);
          }
        }
        nuniq += popc64(ballot64(inserted));
        const int nstep = min(16, nkept - s0);
        for (int uu = 0; uu < nstep; ++uu) {
          wave_lds_sync();
          if (have && u == uu)
            __hip_atomic_fetch_add(&acc[slot], val, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
        }
        if (nuniq > kURowMax) {
          over = true;
          break;
        }
      }
    }
  }
  if (over) {
    if (lane == 0) {
      rownnz[i] = 0;
      atomicAdd(&counters[kCntRowOverflow], 1ull);
    }
    return;
  }
  wave_lds_sync();
  int32_t* LC = s_lc[wib];
  double* LV = s_lv[wib];
  int n = 0;
  for (int k0 = 0; k0 < kUHash; k0 += kWave) {
    const int32_t cv = key[k0 + lane];
    const bool used = cv != -1;
    const uint64_t m = ballot64(used);
    if (used) {
      LC[n + rank_below(m)] = cv;
      LV[n + rank_below(m)] = acc[k0 + lane];
    }
    n += popc64(m);
  }
  wave_lds_sync();
  const int64_t o = tmp_off[i];
  for (int e = lane; e < n; e += kWave) {
    const int32_t cv = LC[e];
    int r = 0;
    for (int x = 0; x < n; ++x) r += LC[x] < cv ? 1 : 0;
    tmp_col[o + r] = cv;
    tmp_val[o + r] = T(LV[e]);
  }
  if (lane == 0) rownnz[i] = n;
}

// Copies each row from the row scratch into the CSR arrays.
template <typename T>
__global__ __launch_bounds__(256) void k_rows_compact_u(
    int64_t n_v, const int64_t* __restrict__ tmp_off, const int32_t* __restrict__ tmp_col,
    const T* __restrict__ tmp_val, const int64_t* __restrict__ rp, int32_t* __restrict__ col,
    T* __restrict__ val) {
  const int64_t i = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / kWave;
  const int lane = lane_id();
  if (i >= n_v) return;
  const int64_t src = tmp_off[i], dst = rp[i], n = rp[i + 1] - rp[i];
  for (int64_t k = lane; k < n; k += kWave) {
    col[dst + k] = tmp_col[src + k];
    val[dst + k] = tmp_val[src + k];
  }
}

// Rows of B by the LDS row gather; returns -1 (nothing written to B) when
// some row has more than kURowMax distinct columns.
template <typename T>
int rows_by_lds(ibvt_coupling* c, int64_t n_pairs, hipStream_t s) {
  const int64_t n_v = c->n_vert;
  int st;
  if ((st = ensure(c, c->rowcap, size_t(n_v + 1) * sizeof(int64_t)))) return st;
  if ((st = ensure(c, c->rowtmpoff, size_t(n_v + 1) * sizeof(int64_t)))) return st;
  if ((st = ensure(c, c->rownnz, size_t(n_v + 1) * sizeof(int64_t)))) return st;
  {
    ProfScope ps("rows_box", s);
    if (n_v > 0)
      k_row_cap_u<<<blocks_for(n_v, 256), 256, 0, s>>>(n_v, c->vt_ptr.as<int64_t>(),
                                                       c->vt_tet.as<int32_t>(),
                                                       c->pair_off.as<int64_t>(),
                                                       c->rowcap.as<int64_t>());
    if ((st = scan_i64(c, c->rowcap.as<int64_t>(), c->rowtmpoff.as<int64_t>(), n_v, s)))
      return st;
  }
  int64_t n_tmp = 0;
  if ((st = read_back(c, &n_tmp, c->rowtmpoff.as<int64_t>() + n_v, sizeof(int64_t), s)))
    return st;
  if ((st = ensure(c, c->rowtmpcol, size_t(n_tmp + 1) * sizeof(int32_t)))) return st;
  if ((st = ensure(c, c->rowtmpval, size_t(n_tmp + 1) * sizeof(T)))) return st;
  auto* counters = c->counters.as<unsigned long long>();
  Csr& B = c->B[0];
  B.nrows = n_v;
  if ((st = ensure(c, B.rowptr, size_t(n_v + 1) * sizeof(int64_t)))) return st;
  {
    ProfScope ps("rows_gather", s);
    if (n_v > 0)
      k_rows_u<T><<<blocks_for(n_v * kWave, 256), 256, 0, s>>>(
          n_v, c->vt_ptr.as<int64_t>(), c->vt_tet.as<int32_t>(), c->tets.as<int32_t>(),
          c->pair_off.as<int64_t>(), c->keep.as<uint8_t>(), c->owner.as<int32_t>(),
          c->ftets.as<int32_t>(), c->pval.as<T>(), c->rowtmpoff.as<int64_t>(),
          c->rowtmpcol.as<int32_t>(), c->rowtmpval.as<T>(), c->rownnz.as<int64_t>(), counters);
    if ((st = hip_check(hipGetLastError(), "row gather launch"))) return st;
    if ((st = scan_i64(c, c->rownnz.as<int64_t>(), B.rowptr.as<int64_t>(), n_v, s))) return st;
  }
  unsigned long long over = 0;
  if ((st = read_back(c, &over, counters + kCntRowOverflow, sizeof(over), s))) return st;
  if (over) return -1;
  int64_t nnz = 0;
  if ((st = read_back(c, &nnz, B.rowptr.as<int64_t>() + n_v, sizeof(int64_t), s))) return st;
  B.nnz = nnz;
  if ((st = ensure(c, B.col, size_t(nnz + 1) * sizeof(int32_t)))) return st;
  if ((st = ensure(c, B.val, size_t(nnz + 1) * sizeof(T)))) return st;
  {
    ProfScope ps("rows_compact", s);
    if (n_v > 0)
      k_rows_compact_u<T><<<blocks_for(n_v * kWave, 256), 256, 0, s>>>(
          n_v, c->rowtmpoff.as<int64_t>(), c->rowtmpcol.as<int32_t>(), c->rowtmpval.as<T>(),
          B.rowptr.as<int64_t>(), B.col.as<int32_t>(), B.val.as<T>());
  }
  return hip_check(hipGetLastError(), "rows launch");
}

// Rows of B by sorting: the 16 entries of every pair keyed by (solid vertex,
// fluid vertex), a stable radix sort, one lane per run of equal keys.
template <typename T>
int rows_by_sort(ibvt_coupling* c, int64_t n_pairs, hipStream_t s) {
  const int64_t n_s = c->n_tet, n_v = c->n_vert;
  int st;
  const int64_t n_e = 16 * n_pairs;
  // key bits: cb for the fluid vertex, then enough for rows 0..n_vert
  auto bits = [](uint64_t x) { return x ? 64 - __builtin_clzll(x) : 0; };
  const int cb = bits(uint64_t(c->n_fvert > 1 ? c->n_fvert - 1 : 0));
  const int end_bit = cb + bits(uint64_t(n_v));
  const uint64_t none = uint64_t(n_v) << cb;
  size_t temp_bytes = 0;
  if (n_e > 0 &&
      (st = hip_check(hipcub::DeviceRadixSort::SortPairs(
                          nullptr, temp_bytes, static_cast<const uint64_t*>(nullptr),
                          static_cast<uint64_t*>(nullptr), static_cast<const uint32_t*>(nullptr),
                          static_cast<uint32_t*>(nullptr), int(n_e), 0, end_bit, s),
                      "sort size")))
    return st;
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  const size_t kb = al(size_t(n_e + 1) * 8), ib = al(size_t(n_e + 1) * 4);
  const size_t hb = al(size_t(n_e + 1) * 4), pb = al(size_t(n_e + 2) * 8);
  if ((st = ensure(c, c->ucoo, 2 * kb + 2 * ib + hb + pb + ib + al(temp_bytes) + 256))) return st;
  char* base = c->ucoo.as<char>();
  uint64_t* keys = reinterpret_cast<uint64_t*>(base);
  uint64_t* skeys = reinterpret_cast<uint64_t*>(base + kb);
  uint32_t* idx = reinterpret_cast<uint32_t*>(base + 2 * kb);
  uint32_t* sidx = reinterpret_cast<uint32_t*>(base + 2 * kb + ib);
  int32_t* head = reinterpret_cast<int32_t*>(base + 2 * kb + 2 * ib);
  int64_t* pos = reinterpret_cast<int64_t*>(base + 2 * kb + 2 * ib + hb);
  int32_t* rowid = reinterpret_cast<int32_t*>(base + 2 * kb + 2 * ib + hb + pb);
  void* temp = base + 2 * kb + 3 * ib + hb + pb;
  int64_t nnz = 0;
  {
    ProfScope ps("rows_sort", s);
    if (n_e > 0) {
      k_coo<<<blocks_for(n_pairs, 256), 256, 0, s>>>(
          n_pairs, n_s, c->pair_off.as<int64_t>(), c->owner.as<int32_t>(), c->tets.as<int32_t>(),
          c->ftets.as<int32_t>(), c->keep.as<uint8_t>(), cb, none, keys, idx);
      if ((st = hip_check(hipcub::DeviceRadixSort::SortPairs(temp, temp_bytes, keys, skeys, idx,
                                                             sidx, int(n_e), 0, end_bit, s),
                          "entry sort")))
        return st;
      k_run_heads<<<blocks_for(n_e, 256), 256, 0, s>>>(n_e, none, skeys, head);
      if ((st = scan_i32_to_i64(c, head, pos, n_e, s))) return st;
      if ((st = read_back(c, &nnz, pos + n_e, sizeof(int64_t), s))) return st;
    }
  }
  Csr& B = c->B[0];
  B.nrows = n_v;
  B.nnz = nnz;
  if ((st = ensure(c, B.rowptr, size_t(n_v + 1) * sizeof(int64_t)))) return st;
  if ((st = ensure(c, B.col, size_t(nnz + 1) * sizeof(int32_t)))) return st;
  if ((st = ensure(c, B.val, size_t(nnz + 1) * sizeof(T)))) return st;
  {
    ProfScope ps("rows_gather", s);
    if (n_e > 0)
      k_run_sums<T><<<blocks_for(n_e, 256), 256, 0, s>>>(n_e, cb, skeys, sidx, head, pos,
                                                         c->pval.as<T>(), B.col.as<int32_t>(),
                                                         rowid, B.val.as<T>());
    k_row_ptr<<<blocks_for(n_v + 1, 256), 256, 0, s>>>(n_v, nnz, rowid, B.rowptr.as<int64_t>());
  }
  return hip_check(hipGetLastError(), "rows launch");
}

template <typename T>
int assemble_u_typed(ibvt_coupling* c, hipStream_t s) {
  const int64_t n_s = c->n_tet, n_v = c->n_vert;
  unsigned* flags = c->flags_dev.as<unsigned>();
  auto* counters = c->counters.as<unsigned long long>();
  int st;
  if ((st = hip_check(hipMemsetAsync(flags, 0, sizeof(unsigned), s), "memset"))) return st;
  if ((st = hip_check(hipMemsetAsync(counters, 0, kCntSlots * sizeof(unsigned long long), s),
                      "memset")))
    return st;
  // (I) solid records and the tree search
  {
    ProfScope ps("tet_prep", s);
    if (n_s > 0)
      k_tet_rec<<<blocks_for(n_s, 256), 256, 0, s>>>(n_s, n_v, c->X.as<double>(),
                                                     c->tets.as<int32_t>(), c->rowbox.as<double>(),
                                                     c->tetrec.as<double>(), c->tetvol.as<double>(),
                                                     flags);
  }
  // first pass: counts, and the finds of each tet up to kSearchCap
  const size_t tmp_bytes = (size_t(n_s + 1) * kSearchCap * sizeof(int32_t) + 255) & ~size_t(255);
  if ((st = ensure(c, c->ucoo, tmp_bytes + 256))) return st;
  int32_t* stmp = c->ucoo.as<int32_t>();
  unsigned* ovf = reinterpret_cast<unsigned*>(c->ucoo.as<char>() + tmp_bytes);
  if ((st = hip_check(hipMemsetAsync(ovf, 0, sizeof(unsigned), s), "memset"))) return st;
  {
    ProfScope ps("tree_search", s);
    if (n_s > 0)
      k_search<2><<<blocks_for(n_s, kSearchThreads), kSearchThreads, 0, s>>>(
          n_s, c->rowbox.as<double>(), c->ftree_leaves, c->n_ftet, c->ftree.as<float>(),
          c->forder.as<int32_t>(), c->fbox.as<double>(), c->cnt.as<int64_t>(), nullptr, nullptr,
          flags, stmp, ovf);
  }
  if ((st = hip_check(hipGetLastError(), "search launch"))) return st;
  if ((st = scan_i64(c, c->cnt.as<int64_t>(), c->pair_off.as<int64_t>(), n_s, s))) return st;
  if ((st = check_flags(c, s))) return st;
  int64_t n_pairs = 0;
  if ((st = read_back(c, &n_pairs, c->pair_off.as<int64_t>() + n_s, sizeof(int64_t), s)))
    return st;
  if (n_pairs >= (int64_t(1) << 31) / 16)
    return set_error(IBVT_E_CAPACITY, "too many (solid tet, fluid tet) pairs");
  c->n_pairs = n_pairs;
  if ((st = ensure(c, c->owner, size_t(n_pairs + 1) * sizeof(int32_t)))) return st;
  if ((st = ensure(c, c->keep, size_t(n_pairs + 1)))) return st;
  if ((st = ensure(c, c->pval, size_t(n_pairs + 1) * 16 * sizeof(T)))) return st;
  if ((st = ensure(c, c->pmom, size_t(n_pairs + 1) * kULam * sizeof(T)))) return st;
  unsigned over = 0;
  if ((st = read_back(c, &over, ovf, sizeof(over), s))) return st;
  {
    ProfScope ps("tree_search", s);
    if (n_s > 0 && over)  // some tet found more than kSearchCap: traverse again
      k_search<1><<<blocks_for(n_s, kSearchThreads), kSearchThreads, 0, s>>>(
          n_s, c->rowbox.as<double>(), c->ftree_leaves, c->n_ftet, c->ftree.as<float>(),
          c->forder.as<int32_t>(), c->fbox.as<double>(), nullptr, c->pair_off.as<int64_t>(),
          c->owner.as<int32_t>(), flags, nullptr, nullptr);
    else if (n_s > 0)
      k_search_copy<<<blocks_for(n_s, 256), 256, 0, s>>>(n_s, c->pair_off.as<int64_t>(), stmp,
                                                        c->owner.as<int32_t>());
  }
  // (II)-(III) clip and integrate every pair that no face plane separates
  if (n_pairs > 0) {
    auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
    const size_t cb = al(size_t(n_pairs + 1) * sizeof(int32_t));
    const size_t pb = al(size_t(n_pairs + 2) * sizeof(int64_t));
    if ((st = ensure(c, c->ucoo, 2 * cb + pb + 256))) return st;
    int32_t* cand = c->ucoo.as<int32_t>();
    int64_t* pos = reinterpret_cast<int64_t*>(c->ucoo.as<char>() + cb);
    int32_t* list = reinterpret_cast<int32_t*>(c->ucoo.as<char>() + cb + pb);
    int64_t n_list = 0;
    {
      ProfScope ps("pairs_filter", s);
      k_sep_u<<<blocks_for(n_pairs, 256), 256, 0, s>>>(
          n_pairs, n_s, c->pair_off.as<int64_t>(), c->owner.as<int32_t>(), c->tetrec.as<double>(),
          c->frec.as<double>(), cand, c->keep.as<uint8_t>());
      if ((st = scan_i32_to_i64(c, cand, pos, n_pairs, s))) return st;
      k_list_u<<<blocks_for(n_pairs, 256), 256, 0, s>>>(n_pairs, cand, pos, list);
      if ((st = hip_check(hipGetLastError(), "filter launch"))) return st;
    }
    if ((st = read_back(c, &n_list, pos + n_pairs, sizeof(int64_t), s))) return st;
    ProfScope ps("pairs_tet", s);
    if (n_list > 0)
      k_pairs_u<T><<<unsigned(ceil_div(n_list, kWave)), kWave, 0, s>>>(
          n_list, list, n_s, c->pair_off.as<int64_t>(), c->owner.as<int32_t>(),
          c->tetrec.as<double>(), c->frec.as<double>(), 1e-14, c->dual ? 1 : 0,
          c->keep.as<uint8_t>(), c->pval.as<T>(), c->pmom.as<T>(), flags, counters);
  }
  if ((st = hip_check(hipGetLastError(), "pairs launch"))) return st;
  // (IV) B: rows gathered in LDS, or by sorting the entries when a row is
  // too wide for that
  if ((st = rows_by_lds<T>(c, n_pairs, s)) > 0) return st;
  if (st < 0 && (st = rows_by_sort<T>(c, n_pairs, s))) return st;
  {
    ProfScope ps("transpose", s);
    if ((st = transpose_one<T>(c, 0, s))) return st;
  }
  // the three velocity components share the fluid nodes: one B
  c->B[1] = c->B[2] = c->B[0];
  c->Bt[1] = c->Bt[2] = c->Bt[0];
  if ((st = solid_masses(c, s))) return st;
  unsigned long long cnt[kCntSlots];
  if ((st = read_back(c, cnt, counters, sizeof(cnt), s))) return st;
  c->stats.pairs = n_pairs;
  c->stats.pieces = int64_t(cnt[kCntPieces]);
  c->stats.dropped = int64_t(cnt[kCntDropped]);
  c->stats.zero_tets = 0;
  c->stats.subtets = 0;
  c->stats.dist_evals = 0;
  c->stats.cut_points = 0;
  c->mom_valid = false;
  c->stats.assemblies += 1;
  return check_flags(c, s);
}

// Reverse mode, one lane per (component d, solid tet s) walking the tet's
// kept pairs.  Moving vertex a of the solid tet moves its points by λ_a e_k
// while the fluid hats stay fixed, so with w = Σ_i z'_i λ_i (z' the dual
// weights 5 z_i − Σ_k z_k with dual multipliers, else z) and U = Σ_j u_j μ_j
// (constant gradient on the pair's fluid tet) a pair adds
//   ∂_k U · Σ_i z'_i ∫ λ_a λ_i  +  ∂_k λ_a · Σ_ij z_i u_j vals_ij
// (vals holds ∫ ψ_i μ_j with dual multipliers, which carries the weights).
// Sums in double to pgt[(d, s)][12] (vertex a, axis k at a*3 + k).  With
// TWO a second contraction (weights z2, fluid field v, factor alpha2) is
// added from the same pair data: both adjoints in one pass.
template <typename T, bool TWO>
__global__ __launch_bounds__(256) void k_shape_u(
    int64_t n_s, int64_t n_v, const int64_t* __restrict__ off, const int32_t* __restrict__ pf,
    const uint8_t* __restrict__ keep, const T* __restrict__ vals, const T* __restrict__ lams,
    const double* __restrict__ srec, const double* __restrict__ frec,
    const int32_t* __restrict__ tets_s, const int32_t* __restrict__ tets_f,
    const T* __restrict__ z, const T* u0, const T* u1, const T* u2, const T* __restrict__ z2,
    const T* v0, const T* v1, const T* v2, double alpha2, int dual, double* __restrict__ pgt) {
  const int64_t w = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (w >= 3 * n_s) return;
  const int d = int(w / n_s);
  const int64_t s = w - int64_t(d) * n_s;
  double acc[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = 0.0;
  const int64_t p0 = off[s], p1 = off[s + 1];
  if (p1 > p0) {
    const int4 tv = *reinterpret_cast<const int4*>(tets_s + 4 * s);
    const T* zd = z + int64_t(d) * n_v;
    const double zl[4] = {double(zd[tv.x]), double(zd[tv.y]), double(zd[tv.z]),
                          double(zd[tv.w])};
    double zw[4] = {zl[0], zl[1], zl[2], zl[3]};
    if (dual) {
      const double sum = zl[0] + zl[1] + zl[2] + zl[3];
      for (int i = 0; i < 4; ++i) zw[i] = 5.0 * zl[i] - sum;
    }
    double zl2[4] = {0.0, 0.0, 0.0, 0.0}, zw2[4] = {0.0, 0.0, 0.0, 0.0};
    if (TWO) {
      const T* z2d = z2 + int64_t(d) * n_v;
      zl2[0] = double(z2d[tv.x]);
      zl2[1] = double(z2d[tv.y]);
      zl2[2] = double(z2d[tv.z]);
      zl2[3] = double(z2d[tv.w]);
      const double sum = zl2[0] + zl2[1] + zl2[2] + zl2[3];
      for (int i = 0; i < 4; ++i) zw2[i] = dual ? 5.0 * zl2[i] - sum : zl2[i];
    }
    const T* v = (d == 0) ? v0 : (d == 1 ? v1 : v2);
    const double* gl = srec + kURec * s + 12;  // ∇λ_a at gl[3a + k]
    const T* u = (d == 0) ? u0 : (d == 1 ? u1 : u2);
    for (int64_t p = p0; p < p1; ++p) {
      if (!keep[p]) continue;
      const int64_t f = pf[p];
      const int4 fv = *reinterpret_cast<const int4*>(tets_f + 4 * f);
      const double ul[4] = {double(u[fv.x]), double(u[fv.y]), double(u[fv.z]), double(u[fv.w])};
      const double* gm = frec + kURec * f + 12;  // ∇μ_j at gm[3j + k]
      double gu[3];
#pragma unroll
      for (int k = 0; k < 3; ++k)
        gu[k] = ul[0] * gm[k] + ul[1] * gm[3 + k] + ul[2] * gm[6 + k] + ul[3] * gm[9 + k];
      T V[16], L[kULam];
      load_row<16>(vals + 16 * p, V);
      load_row<kULam>(lams + kULam * p, L);
      double zvu = 0.0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        double r = 0.0;
#pragma unroll
        for (int j = 0; j < 4; ++j) r += double(V[4 * i + j]) * ul[j];
        zvu += zl[i] * r;
      }
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        double zla = 0.0;
#pragma unroll
        for (int i = 0; i < 4; ++i) zla += zw[i] * double(L[lam_index(a, i)]);
#pragma unroll
        for (int k = 0; k < 3; ++k) acc[a * 3 + k] += gu[k] * zla + gl[3 * a + k] * zvu;
      }
      if (TWO) {
        const double vl[4] = {double(v[fv.x]), double(v[fv.y]), double(v[fv.z]),
                              double(v[fv.w])};
        double gv[3];
#pragma unroll
        for (int k = 0; k < 3; ++k)
          gv[k] = vl[0] * gm[k] + vl[1] * gm[3 + k] + vl[2] * gm[6 + k] + vl[3] * gm[9 + k];
        double zvv = 0.0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          double r = 0.0;
#pragma unroll
          for (int j = 0; j < 4; ++j) r += double(V[4 * i + j]) * vl[j];
          zvv += zl2[i] * r;
        }
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          double zla = 0.0;
#pragma unroll
          for (int i = 0; i < 4; ++i) zla += zw2[i] * double(L[lam_index(a, i)]);
#pragma unroll
          for (int k = 0; k < 3; ++k)
            acc[a * 3 + k] += alpha2 * (gv[k] * zla + gl[3 * a + k] * zvv);
        }
      }
    }
  }
  store_row<12>(pgt + w * 12, acc);
}

template <typename T>
int shape_u_typed(ibvt_coupling* c, const void* z, const void* const u[3], const void* us,
                  int mass, double alpha, double* gX, hipStream_t s, const void* z2 = nullptr,
                  const void* const* v = nullptr, double alpha2 = 0.0) {
  if (c->n_pairs > 0 && !c->pmom.p)
    return set_error(IBVT_E_INVALID, "the per-pair integrals are not stored");
  const size_t tc_bytes = (size_t(3 * c->n_tet + 1) * 12 * sizeof(double) + 255) & ~size_t(255);
  int st = ensure(c, c->work2, tc_bytes);
  if (st) return st;
  double* pgt = c->work2.as<double>();
  {
    ProfScope ps("shape_terms", s);
    const unsigned nb = blocks_for(3 * c->n_tet, 256);
    const T* zz = static_cast<const T*>(z);
    const T* u0 = static_cast<const T*>(u[0]);
    const T* u1 = static_cast<const T*>(u[1]);
    const T* u2 = static_cast<const T*>(u[2]);
    if (c->n_tet > 0 && z2)
      k_shape_u<T, true><<<nb, 256, 0, s>>>(
          c->n_tet, c->n_vert, c->pair_off.as<int64_t>(), c->owner.as<int32_t>(),
          c->keep.as<uint8_t>(), c->pval.as<T>(), c->pmom.as<T>(), c->tetrec.as<double>(),
          c->frec.as<double>(), c->tets.as<int32_t>(), c->ftets.as<int32_t>(), zz, u0, u1, u2,
          static_cast<const T*>(z2), static_cast<const T*>(v[0]), static_cast<const T*>(v[1]),
          static_cast<const T*>(v[2]), alpha2 / alpha, c->dual ? 1 : 0, pgt);
    else if (c->n_tet > 0)
      k_shape_u<T, false><<<nb, 256, 0, s>>>(
          c->n_tet, c->n_vert, c->pair_off.as<int64_t>(), c->owner.as<int32_t>(),
          c->keep.as<uint8_t>(), c->pval.as<T>(), c->pmom.as<T>(), c->tetrec.as<double>(),
          c->frec.as<double>(), c->tets.as<int32_t>(), c->ftets.as<int32_t>(), zz, u0, u1, u2,
          nullptr, nullptr, nullptr, nullptr, 0.0, c->dual ? 1 : 0, pgt);
  }
  if ((st = hip_check(hipGetLastError(), "shape launch"))) return st;
  return shape_gather(c, pgt, z, us, mass, alpha, gX, c->tetrec.as<double>() + 12, kURec, s);
}

}  // namespace

int build_fluid_tree(ibvt_coupling* c, hipStream_t s) {
  const int64_t n_f = c->n_ftet;
  int st;
  if ((st = ensure(c, c->frec, size_t(n_f + 1) * kURec * sizeof(double)))) return st;
  if ((st = ensure(c, c->fbox, size_t(n_f + 1) * 8 * sizeof(double)))) return st;
  unsigned* flags = c->flags_dev.as<unsigned>();
  if ((st = hip_check(hipMemsetAsync(flags, 0, sizeof(unsigned), s), "memset"))) return st;
  ProfScope ps("fluid_tree", s);
  k_tet_rec<<<blocks_for(n_f, 256), 256, 0, s>>>(n_f, c->n_fvert, c->fX.as<double>(),
                                                 c->ftets.as<int32_t>(), c->fbox.as<double>(),
                                                 c->frec.as<double>(), nullptr, flags);
  if ((st = hip_check(hipGetLastError(), "fluid record launch"))) return st;
  if ((st = check_flags(c, s))) return st;
  // bounding box of the fluid mesh
  const int nbb = int(std::min<int64_t>(blocks_for(n_f, 256), 1024));
  if ((st = ensure(c, c->ucoo, size_t(nbb + 2) * 6 * sizeof(double)))) return st;
  double* part = c->ucoo.as<double>();
  double* bb = part + 6 * nbb;
  k_box_partials<<<nbb, 256, 0, s>>>(n_f, c->fbox.as<double>(), part);
  k_box_final<<<1, 64, 0, s>>>(nbb, part, bb);
  // Morton order
  size_t temp_bytes = 0;
  if ((st = hip_check(hipcub::DeviceRadixSort::SortPairs(
                          nullptr, temp_bytes, static_cast<const uint32_t*>(nullptr),
                          static_cast<uint32_t*>(nullptr), static_cast<const int32_t*>(nullptr),
                          static_cast<int32_t*>(nullptr), int(n_f), 0, 30, s),
                      "sort size")))
    return st;
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  const size_t cb = al(size_t(n_f + 1) * 4);
  if ((st = ensure(c, c->pscan, 3 * cb + al(temp_bytes) + 256))) return st;
  char* base = c->pscan.as<char>();
  uint32_t* code = reinterpret_cast<uint32_t*>(base);
  uint32_t* scode = reinterpret_cast<uint32_t*>(base + cb);
  int32_t* idx = reinterpret_cast<int32_t*>(base + 2 * cb);
  void* temp = base + 3 * cb;
  if ((st = ensure(c, c->forder, size_t(n_f + 1) * sizeof(int32_t)))) return st;
  k_morton<<<blocks_for(n_f, 256), 256, 0, s>>>(n_f, c->fbox.as<double>(), bb, code, idx);
  if ((st = hip_check(hipcub::DeviceRadixSort::SortPairs(temp, temp_bytes, code, scode, idx,
                                                         c->forder.as<int32_t>(), int(n_f), 0, 30,
                                                         s),
                      "Morton sort")))
    return st;
  // implicit tree: P leaves (power of two), 2P - 1 nodes, levels bottom-up
  int64_t P = 1;
  while (P < n_f) P <<= 1;
  if ((st = ensure(c, c->ftree, size_t(2 * P) * 8 * sizeof(float)))) return st;
  k_tree_leaves<<<blocks_for(P, 256), 256, 0, s>>>(n_f, P, c->forder.as<int32_t>(),
                                                   c->fbox.as<double>(), c->ftree.as<float>());
  for (int64_t cnt = P / 2; cnt >= 1; cnt /= 2)
    k_tree_level<<<blocks_for(cnt, 256), 256, 0, s>>>(cnt - 1, cnt, c->ftree.as<float>());
  c->ftree_leaves = P;
  return hip_check(hipGetLastError(), "tree launch");
}

int assemble_all_unstructured(ibvt_coupling* c, hipStream_t s) {
  const int64_t n_s = c->n_tet, n_v = c->n_vert;
  int st;
  if (c->ftree_leaves == 0 && (st = build_fluid_tree(c, s))) return st;
  if ((st = ensure(c, c->tetvol, size_t(n_s + 1) * sizeof(double)))) return st;
  if ((st = ensure(c, c->tetrec, size_t(n_s + 1) * kURec * sizeof(double)))) return st;
  if ((st = ensure(c, c->rowbox, size_t(n_s + 1) * 8 * sizeof(double)))) return st;
  if ((st = ensure(c, c->cnt, size_t(n_s + 1) * sizeof(int64_t)))) return st;
  if ((st = ensure(c, c->pair_off, size_t(n_s + 1) * sizeof(int64_t)))) return st;
  if ((st = ensure(c, c->mlump, size_t(n_v + 1) * sizeof(double)))) return st;
  if (c->precision == IBVT_FP32_MIXED) {
    if ((st = ensure(c, c->minv, size_t(n_v + 1) * sizeof(float)))) return st;
    return assemble_u_typed<float>(c, s);
  }
  if ((st = ensure(c, c->minv, size_t(n_v + 1) * sizeof(double)))) return st;
  return assemble_u_typed<double>(c, s);
}

}  // namespace ibvt

namespace ibvt {

int shape_gradient_unstructured(ibvt_coupling* c, const void* z, const void* const u[3],
                                const void* us, int mass, double alpha, double* gX,
                                hipStream_t s) {
  if (c->precision == IBVT_FP32_MIXED) return shape_u_typed<float>(c, z, u, us, mass, alpha, gX, s);
  return shape_u_typed<double>(c, z, u, us, mass, alpha, gX, s);
}

int shape_gradient_unstructured_two(ibvt_coupling* c, const void* z, const void* const u[3],
                                    const void* us, int mass, const void* z2,
                                    const void* const v[3], double alpha2, double* gX,
                                    hipStream_t s) {
  if (c->precision == IBVT_FP32_MIXED)
    return shape_u_typed<float>(c, z, u, us, mass, 1.0, gX, s, z2, v, alpha2);
  return shape_u_typed<double>(c, z, u, us, mass, 1.0, gX, s, z2, v, alpha2);
}

}  // namespace ibvt
