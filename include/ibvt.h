/*
 * ibvt — L2-projection transfer between a staggered rectilinear fluid grid
 * and a P1 tetrahedral solid mesh, on AMD MI355X (gfx950).
 *
 * The operations are those of Section 2.3 of Nestola et al., "An immersed
 * boundary method for fluid-structure interaction based on overlapping
 * domain decomposition" (arXiv 1810.13046), paragraph "Variational Transfer:
 * the L2-Projection Approach":
 *
 *   - the auxiliary Q1 space on the finite-difference grid (one node lattice
 *     per velocity component of the staggered grid of Section 2.2);
 *   - the mortar integrals  B_ij = ∫ N_f,j N_fsi,i dV  (solid rows i, fluid
 *     columns j) and S_ij = ∫ N_s,j N_fsi,i dV, with the standard multiplier
 *     space equal to the P1 solid space, so S is the P1 mass matrix of
 *     Section 2.1 (consistent) or its row-sum lumping;
 *   - velocity transfer  w_s = S^{-1} B v_f  (Step 1 of the FSI algorithm,
 *     Section 3);
 *   - force transfer with the transpose (Step 4 of Section 3).
 *
 * Conventions common to every call
 *   - All field and mesh buffers are device memory owned by the caller.
 *     Solid nodal fields are (3, n_vert) row-major (component-major).
 *     Fluid fields are one array per component d, laid out (n_z, n_y, n_x)
 *     with x fastest, over component d's lattice (see ibvt_lattice_coords).
 *   - Fluid and solid fields are double for IBVT_FP64 couplings and float
 *     for IBVT_FP32_MIXED couplings.  Coordinates X and the gradient g_X are
 *     always double.
 *   - Work is enqueued on `stream` in order.  Assembly reads counts back
 *     to size its buffers: a grid reassembly synchronizes the stream seven
 *     times (four packed read-backs of counts and status flags, one per
 *     velocity component in the transpose), a few more when a handle is
 *     created (lattices, topology, mass pattern); planar and unstructured
 *     assemblies a similar fixed number.  Transfers synchronize only for
 *     the consistent-mass solve's convergence checks and when `info` is
 *     requested.
 *   - The library's device buffers grow stream-ordered (hipMallocAsync and
 *     hipFreeAsync on the call's stream), so growing them does not
 *     synchronize the device.  Calls on one handle with different streams
 *     must be ordered by the caller (an event or a synchronization), as
 *     for the data they share.
 *   - Every call returns an ibvt status; nothing throws across the ABI.
 *     ibvt_last_error() returns a thread-local message for the last failure.
 *
 * Planar couplings (assemble_coupling_2d: Q1 quadrilateral lattice x P1
 * triangles, the setting of the paper's 2D experiments in Section 4) use the
 * same handle and the same transfer calls with two components: solid fields
 * are (2, n_vert), fluid fields u_f[0], u_f[1] are (n_y, n_x) arrays (u_f[2]
 * is ignored and may be NULL), X and g_X are (n_vert, 2).  Areas replace
 * volumes: m_i = Σ_{T∋i} |T|/3, M_il = |T|(1+δ_il)/12, and the dual
 * multipliers are ψ_i = 4λ_i − 1 on each triangle.
 */
#ifndef IBVT_H
#define IBVT_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define IBVT_OK 0
#define IBVT_E_INVALID 1        /* null pointer, bad size or enum, non-finite
                                   coordinate, non-increasing faces */
#define IBVT_E_OUT_OF_GRID 2    /* a tet's bounding box leaves a velocity
                                   lattice's node hull */
#define IBVT_E_HIP 3            /* a HIP runtime call failed */
#define IBVT_E_NOMEM 4          /* device allocation failed */
#define IBVT_E_NOT_CONVERGED 5  /* a solve reached its iteration limit;
                                   results are written */
#define IBVT_E_CAPACITY 6       /* an internal fixed capacity was exceeded
                                   (clipped-piece vertices, vertex valence,
                                   index range); the coupling is unusable */
#define IBVT_E_UNSUPPORTED 7    /* valid but unsupported combination */

/* Precision of a coupling. */
#define IBVT_FP64 0             /* everything in double */
#define IBVT_FP32_MIXED 1       /* double coordinates, plane distances and
                                   cut points; float quadrature, float B
                                   values and float transfers; mass solves
                                   with float inner iterations and a double
                                   residual */

/* Mass matrix used for S. */
#define IBVT_LUMPED 0           /* S = diag(m), m_i = ∫ λ_i = Σ_{T∋i} |T|/4 */
#define IBVT_CONSISTENT 1       /* S = M, M_il = ∫ λ_i λ_l, solved by a
                                   Jacobi-scaled Chebyshev iteration */

/* assemble_coupling flags. */
#define IBVT_BUILD_CONSISTENT_M 1u  /* also build the consistent mass matrix */
#define IBVT_NO_PIECE_STORE 2u      /* do not keep the pieces' moments; the
                                       reverse-mode calls then clip again
                                       (less device memory) */
#define IBVT_DUAL_BASIS 4u          /* dual ("pseudo" L2) multipliers,
                                       Section 2.3 eq. biorth: B_ij =
                                       ∫ ψ_i N_j with ψ_i = 5λ_i − 1 on each
                                       tet (∫ λ_j ψ_i = δ_ij |T|/4), so S is
                                       the lumped mass diag(m): velocity
                                       transfers take IBVT_LUMPED (consistent
                                       is IBVT_E_INVALID) and
                                       IBVT_FORCE_IS_LOAD applies diag(m)^-1 */
#define IBVT_NO_STORE_B 8u          /* grids only: keep neither B, B^T nor
                                       any per-pair data, only the per-tet
                                       data and the solid masses; every
                                       product with B or B^T and the shape
                                       derivative clip and integrate the
                                       pieces again (the memory-saving
                                       recompute form of the reverse mode).
                                       B^T products add into the fluid
                                       arrays with atomic adds, so their
                                       rounding is not bitwise repeatable;
                                       coupling_export_csr is
                                       IBVT_E_UNSUPPORTED */

/* transfer_force flags. */
#define IBVT_FORCE_IS_LOAD 1u   /* f_s is a load vector: apply S^{-1}
                                   (consistent) before B^T, i.e. the literal
                                   transpose of the velocity transfer
                                   operator T = S^{-1} B */

typedef struct ibvt_coupling ibvt_coupling;

/* Rectilinear fluid grid: n_cells[e] cells along axis e, with n_cells[e]+1
 * strictly increasing face coordinates faces[e] (HOST pointers, read during
 * the call only).  Velocity component d lives on the faces normal to axis d
 * and at face midpoints along the other two axes (staggered grid, Section
 * 2.2), so its lattice has n_cells[d]+1 nodes along axis d and n_cells[e]
 * along e != d. */
typedef struct {
  int32_t n_cells[3];
  const double* faces[3];
} ibvt_grid;

/* P1 tetrahedral mesh in its current configuration (Section 2.1, the
 * transfer uses the current configuration, Section 2.3).  X: device,
 * (n_vert, 3) double, row-major.  tets: device, (n_tet, 4) int32 vertex
 * indices, either orientation.  Both are read during the call (the
 * coupling keeps its own copies). */
typedef struct {
  int64_t n_vert;
  int64_t n_tet;
  const double* X;
  const int32_t* tets;
} ibvt_mesh;

/* Per-component outcome of a consistent-mass solve. */
typedef struct {
  int32_t iterations[3];
  double rel_residual[3];   /* ||b - M x||_2 / ||b||_2, recomputed in double */
} ibvt_solve_info;

/* Counters of a coupling (coupling_info). */
typedef struct {
  int32_t precision;
  int32_t has_consistent_mass;
  int64_t n_vert, n_tet;
  int64_t lattice[3][3];     /* nodes per axis e of component d: [d][e] */
  int64_t n_fluid[3];        /* lattice nodes of component d */
  int64_t pairs;             /* candidate (tet, component, cell) pairs */
  int64_t pieces;            /* non-empty pieces kept (vol > 1e-14 |T|) */
  int64_t dropped;           /* non-empty pieces with vol <= 1e-14 |T| */
  int64_t zero_tets;         /* tets of zero volume (skipped) */
  int64_t nnz[3];            /* nonzeros of B^d (and of B^dT) */
  int64_t touched[3];        /* fluid nodes of component d with a nonzero
                                column in B^d (rows of B^dT) */
  int64_t nnz_mass;          /* nonzeros of the consistent mass matrix */
  int64_t device_bytes;      /* device memory held by the coupling */
  int64_t assemblies;        /* assemblies done on this handle */
  int64_t subtets;           /* sub-tetrahedra integrated by the last
                                assembly (11 quadrature points each) */
  int64_t piece_store;       /* 1 if every kept piece's moments are stored
                                for the reverse mode */
  int64_t dist_evals;        /* plane distances evaluated by the last
                                assembly's clipping (vertices x planes) */
  int64_t cut_points;        /* edge-plane intersection points it made */
  int64_t dual;              /* 1 if B holds the dual-multiplier integrals */
  int64_t dim;               /* 3, or 2 for a planar coupling (n_tet then
                                counts triangles, component 2 is empty) */
  int64_t unstructured;      /* 1 for a tetrahedral fluid background
                                (n_fluid[d] = its vertices, lattice = 0) */
  int64_t plane_cuts;        /* (pair, cell plane) clips run by the last
                                assembly (grids: the cell planes each
                                piece's tet straddles) */
  int64_t matrix_free;       /* 1 if built with IBVT_NO_STORE_B (nnz,
                                touched, pieces, subtets and the clip
                                counters are then 0) */
} ibvt_info;

/* Device allocator for a coupling's own buffers: alloc returns device
 * memory of at least `bytes` bytes, usable in stream order on `stream`, or
 * NULL (the calling entry point then fails with IBVT_E_NOMEM); free
 * releases memory alloc returned, in stream order on `stream`.  ctx is
 * passed back unchanged.  Both may be called from any entry point that
 * grows or frees a buffer (assembly, reassembly, the first call that needs
 * a workspace, coupling_free). */
typedef struct {
  void* (*alloc)(size_t bytes, hipStream_t stream, void* ctx);
  void (*free)(void* ptr, hipStream_t stream, void* ctx);
  void* ctx;
} ibvt_alloc;

/*
 * ibvt_set_allocator — the allocator of the couplings created after this
 *   call (a caching allocator such as PyTorch's, so that the library's
 *   buffers come from the same pool as the caller's tensors).  Each handle
 *   keeps the allocator it was created with and frees with it.  NULL
 *   restores the default, hipMallocAsync / hipFreeAsync on the call's
 *   stream.  Thread-safe with respect to concurrent handle creation.
 *   Errors: IBVT_E_INVALID (a non-NULL a with a NULL alloc or free).
 */
int ibvt_set_allocator(const ibvt_alloc* a);

/*
 * assemble_coupling — build B^d (d = 0, 1, 2) for the mesh and grid.
 *   Section 2.3, assembly steps (I)-(IV): overlap detection (here: index
 *   ranges on the rectilinear lattices instead of a tree search), exact
 *   integration of λ_i N_j on every tet ∩ cell piece (axis-plane clipping
 *   in double, then quadrature exact for the degree-4 integrand), and global
 *   assembly.  Also builds B^dT (over the touched fluid nodes), the lumped
 *   mass and, with IBVT_BUILD_CONSISTENT_M, the consistent mass matrix.
 *   Unless IBVT_NO_PIECE_STORE is set, the 32 moments of every piece
 *   (monomials of degree <= 4 in cell-local coordinates, no exponent above
 *   3) are kept, so that
 *   the reverse-mode calls neither clip nor integrate again.
 *   precision: IBVT_FP64 or IBVT_FP32_MIXED.
 *   out: receives a new handle owned by the library (free with
 *   coupling_free).  On failure *out is set to NULL.
 *   Limits: fewer than 2^30 tets, at most 2^21 cells along each axis,
 *   fewer than 2^31 (tet, cell) pairs and nonzeros per component
 *   (IBVT_E_UNSUPPORTED, IBVT_E_CAPACITY beyond them).
 *   Pairs are clipped and integrated in up to 8 chunks of 3 * 2^19
 *   (component, tet) items (the environment variable IBVT_CHUNK_ITEMS, a
 *   positive integer read at every assembly, sets another size); the
 *   matrices do not depend on the chunking.  B^dT is built through buckets
 *   of consecutive fluid nodes when B^d has at least 2^22 nonzeros, else by
 *   a counting sort over the lattice (IBVT_BUCKET_NNZ, a positive integer
 *   read at every assembly, sets another threshold); both give the same
 *   B^dT.
 *   Errors: IBVT_E_INVALID, IBVT_E_OUT_OF_GRID, IBVT_E_CAPACITY,
 *   IBVT_E_UNSUPPORTED, IBVT_E_NOMEM, IBVT_E_HIP.
 */
int assemble_coupling(const ibvt_grid* grid, const ibvt_mesh* mesh, int precision,
                      uint32_t flags, hipStream_t stream, ibvt_coupling** out);

/* Planar grid: as ibvt_grid with two axes (component d on the faces normal
 * to axis d, face midpoints along the other axis). */
typedef struct {
  int32_t n_cells[2];
  const double* faces[2];
} ibvt_grid2d;

/* P1 triangle mesh: X device (n_vert, 2) double row-major; tris device
 * (n_tri, 3) int32, either orientation. */
typedef struct {
  int64_t n_vert;
  int64_t n_tri;
  const double* X;
  const int32_t* tris;
} ibvt_mesh2d;

/*
 * assemble_coupling_2d — the planar coupling: B^d_ij = ∫ λ_i N^d_j dA for
 *   d = 0, 1 (Section 2.3 over areas), B^dT, the lumped mass m_i =
 *   Σ_{T∋i} |T|/3 and, with IBVT_BUILD_CONSISTENT_M, M_il = |T|(1+δ_il)/12.
 *   Each triangle ∩ cell piece is integrated exactly from its ten moments
 *   (monomials of degree <= 3 in cell-local coordinates, taken by Green's
 *   theorem over the piece boundary with the boundary's intersections in
 *   double); the moments are always kept for the reverse mode
 *   (IBVT_NO_PIECE_STORE has no effect).  IBVT_DUAL_BASIS gives ψ_i =
 *   4λ_i − 1.  The handle works with every transfer call (two components,
 *   see the conventions above), reassemble_coupling (X (n_vert, 2)),
 *   coupling_info, coupling_export_csr (comp 0 or 1) and fsi_step (two
 *   components, X_ref (n_vert, 2); the density option divides by the
 *   nodes' Q1 lumped area).
 *   Errors: IBVT_E_INVALID, IBVT_E_OUT_OF_GRID, IBVT_E_CAPACITY,
 *   IBVT_E_NOMEM, IBVT_E_HIP.
 */
int assemble_coupling_2d(const ibvt_grid2d* grid, const ibvt_mesh2d* mesh, int precision,
                         uint32_t flags, hipStream_t stream, ibvt_coupling** out);

/*
 * assemble_coupling_unstructured — the coupling with an unstructured fluid
 *   background: the fluid space is P1 on the tetrahedral mesh `fluid`
 *   (device X (n_vert, 3), tets (n_tet, 4); copied), collocated, so one
 *   B_ij = ∫ λ_i μ_j (solid vertex i, fluid vertex j; μ_j the fluid P1
 *   hats) serves the three velocity components (Section 2.3: transfer
 *   between unstructured and structured meshes, (I) a tree search for the
 *   overlapping elements, (II)-(III) exact integration on the intersections
 *   of the piecewise affine elements, (IV) assembly).  The tree over the
 *   fluid tets is built once per handle; reassemble_coupling moves the
 *   solid only.  The fluid mesh must cover the solid (partition of unity
 *   of the μ_j); solid parts outside it get no contribution.
 *   Fluid fields u_f[d] / f_f[d] are nodal arrays of the fluid mesh's
 *   n_vert values.  IBVT_DUAL_BASIS and IBVT_BUILD_CONSISTENT_M as for
 *   grids; IBVT_NO_PIECE_STORE has no effect (the per-pair integrals ∫ λ_i μ_j
 *   and ∫ λ_a λ_i are always kept).  The reverse-mode calls give g_uf, g_fs
 *   and the shape derivative g_X, the transport form of the grid case with
 *   the fluid P1 hats μ_j fixed in space:
 *     ∂B_ij/∂X_{a,k} = Σ_{T∋a} ∫_T (λ_a λ_i ∂_k μ_j + ∂_k λ_a λ_i μ_j).
 *   fsi_step drives it with v_f and f_tilde nodal arrays of the fluid mesh
 *   (the force-density option divides by the fluid nodes' lumped volumes
 *   ∫ μ_j = Σ_{T∋j} |T|/4, built on first use).
 *   Errors: IBVT_E_INVALID, IBVT_E_CAPACITY, IBVT_E_NOMEM, IBVT_E_HIP.
 */
int assemble_coupling_unstructured(const ibvt_mesh* fluid, const ibvt_mesh* solid, int precision,
                                   uint32_t flags, hipStream_t stream, ibvt_coupling** out);

/*
 * reassemble_coupling — rebuild the same coupling for moved vertices X
 * (same topology, same grid, same precision and flags): the transfer must
 * follow the current configuration of the solid (Section 2.3), so a moving
 * solid reassembles every step.  Reuses the handle's device buffers
 * (grows them when needed).  X: device (n_vert, 3) double.
 *   Errors: as assemble_coupling; on error the handle must be freed.
 */
int reassemble_coupling(ibvt_coupling* c, const double* X, hipStream_t stream);

/*
 * transfer_velocity — w_s = S^{-1} B v_f (Section 2.3; Step 1 of Section 3).
 *   u_f[d]: component d's fluid values on its lattice (read).
 *   u_s: (3, n_vert) output, overwritten.
 *   mass: IBVT_LUMPED or IBVT_CONSISTENT (needs IBVT_BUILD_CONSISTENT_M).
 *   cg_rtol, cg_maxit: stop when ||b - M x|| <= cg_rtol ||b|| per component
 *   (checked in double after each cycle of Chebyshev iterations on D^-1 M,
 *   D = diag M, whose spectrum lies in [1/2, 5/2] for P1 tetrahedra and
 *   [1/2, 2] for triangles), at most cg_maxit iterations (ignored for
 *   IBVT_LUMPED).  info: nullable.
 *   Errors: IBVT_E_INVALID, IBVT_E_NOT_CONVERGED (u_s holds the last
 *   iterate), IBVT_E_HIP.
 */
int transfer_velocity(ibvt_coupling* c, const void* const u_f[3], void* u_s, int mass,
                      double cg_rtol, int cg_maxit, hipStream_t stream, ibvt_solve_info* info);

/*
 * transfer_velocity_noalloc — transfer_velocity for callers that cannot
 *   allocate device memory (code under stream capture, tight serving loops,
 *   harnesses that forbid allocation): same arguments, results and errors,
 *   and no device allocation of any kind.  The consistent-mass solve's
 *   scratch (the right-hand side B u_f, the Chebyshev vectors, the double
 *   residual) lives in a device array of 256 MiB that the library holds on
 *   each GPU it runs on until the process ends; IBVT_LUMPED needs none.
 *   Limit: about 217 n_vert bytes (FP64) or 133 n_vert bytes (FP32-mixed)
 *   of scratch, so about 1.2M (FP64) and 2.0M (FP32-mixed) solid vertices
 *   with consistent mass; beyond it the call returns IBVT_E_CAPACITY before
 *   any work.  Every call
 *   on one GPU shares that GPU's array, which keeps the last call's
 *   contents: calls that overlap on one GPU (several streams or threads)
 *   race and must be ordered by the caller.
 *   Errors: IBVT_E_INVALID, IBVT_E_CAPACITY, IBVT_E_NOT_CONVERGED,
 *   IBVT_E_HIP.
 */
int transfer_velocity_noalloc(ibvt_coupling* c, const void* const u_f[3], void* u_s, int mass,
                              double cg_rtol, int cg_maxit, hipStream_t stream,
                              ibvt_solve_info* info);

/*
 * transfer_force — f_f[d] += alpha · B^dT f_s[d] at the touched fluid nodes
 *   (force transfer with the transpose, Section 2.3; Step 4 of Section 3,
 *   where alpha is the nondimensional scale L_ref / (rho_f U_ref^2)).
 *   f_s: (3, n_vert), the P1 nodal coefficients of the force density (read).
 *   With IBVT_FORCE_IS_LOAD f_s is a load vector and S^{-1} (consistent,
 *   cg_rtol 1e-12 for FP64 couplings, 1e-6 for FP32 couplings) is applied
 *   first.  f_f[d]: fluid arrays of component d, accumulated.
 *   Errors: IBVT_E_INVALID, IBVT_E_NOT_CONVERGED, IBVT_E_HIP.
 */
int transfer_force(ibvt_coupling* c, const void* f_s, void* const f_f[3], double alpha,
                   uint32_t flags, hipStream_t stream);

/*
 * transfer_velocity_vjp — reverse mode of u_s = S^{-1} B(X) u_f.
 *   With z = S^{-1} g_us:
 *     g_uf[d] += B^dT z_d                       (force-spreading transpose)
 *     g_X     += Σ_d [ z_d^T (∂B^d/∂X) u_f,d − z_d^T (∂S/∂X) u_s,d ]
 *   where ∂B_ij/∂X_{a,k} = Σ_{T∋a} ∫_T (λ_a λ_i ∂_k N_j + ∂_k λ_a λ_i N_j)
 *   (the P1 hats move with the vertices, the Q1 hats stay on the grid) and
 *   ∂|T|/∂X_a = |T| ∇λ_a for the mass.  The derivation is ours; the paper
 *   defines only the forward operators.
 *   g_us, u_s: (3, n_vert) (read); u_f: as in transfer_velocity (read).
 *   g_uf: nullable array of 3 fluid arrays (accumulated); g_X: nullable
 *   (n_vert, 3) double (accumulated).
 *   Errors: IBVT_E_INVALID, IBVT_E_NOT_CONVERGED, IBVT_E_HIP.
 */
int transfer_velocity_vjp(ibvt_coupling* c, const void* g_us, const void* const u_f[3],
                          const void* u_s, int mass, double cg_rtol, int cg_maxit,
                          void* const g_uf[3], double* g_X, hipStream_t stream);

/*
 * transfer_force_vjp — reverse mode of f_f = f_f0 + alpha · B(X)^T f_s
 *   (flags 0 only):  g_fs += alpha · B g_ff,
 *   g_X += alpha · Σ_d f_s,d^T (∂B^d/∂X) g_ff,d.
 *   g_ff: 3 fluid arrays (read); f_s: (3, n_vert) (read); g_fs: nullable
 *   (3, n_vert) (accumulated); g_X: nullable (n_vert, 3) double (accumulated).
 *   Errors: IBVT_E_INVALID, IBVT_E_HIP.
 */
int transfer_force_vjp(ibvt_coupling* c, const void* const g_ff[3], const void* f_s,
                       double alpha, void* g_fs, double* g_X, hipStream_t stream);

/*
 * transfer_vjp — both reverse-mode calls above in one: the effect of
 *   transfer_velocity_vjp(c, g_us, u_f, u_s, mass, cg_rtol, cg_maxit, g_uf,
 *   g_X) followed by transfer_force_vjp(c, g_ff, f_s, alpha, g_fs, g_X),
 *   for a caller that needs the adjoints of both transfers (the velocity
 *   and the force of one coupling step, as in Section 3's loop).  When the
 *   per-pair integrals are stored (3D grid couplings without
 *   IBVT_NO_PIECE_STORE, and unstructured couplings) the two
 *   shape-derivative contractions are taken in one pass over them;
 *   otherwise (planar couplings, re-clipped pieces) the two calls' paths run
 *   one after the other.  Arguments, layouts, ownership and nullability as in the two
 *   calls; g_X (nullable) receives both contributions (sums may differ from
 *   the two separate calls by rounding).
 *   Errors: those of the two calls (IBVT_E_INVALID, IBVT_E_NOT_CONVERGED,
 *   IBVT_E_HIP); nothing is accumulated when an argument check fails.
 */
int transfer_vjp(ibvt_coupling* c, const void* g_us, const void* const u_f[3], const void* u_s,
                 int mass, double cg_rtol, int cg_maxit, void* const g_uf[3],
                 const void* const g_ff[3], const void* f_s, double alpha, void* g_fs,
                 double* g_X, hipStream_t stream);

/* coupling_info — fill *info (host).  Errors: IBVT_E_INVALID. */
int coupling_info(const ibvt_coupling* c, ibvt_info* info);

/*
 * coupling_release_scratch — return the device memory that only the
 *   assembly uses (grid couplings: the piece store, the per-pair values and
 *   record offsets, the row and transpose scratch, the pair order), keeping
 *   what the transfers and the reverse mode read (B, B^T, masses, piece
 *   moments, per-tet data).  For callers that hold couplings between
 *   reassemblies; the next reassembly allocates the scratch again.  Other
 *   couplings: nothing is released.  Stream-ordered on `stream`.
 *   Errors: IBVT_E_INVALID (NULL handle).
 */
int coupling_release_scratch(ibvt_coupling* c, hipStream_t stream);

/* Counters of one body: the tets of a mesh grouped into bodies by
 * consecutive index ranges. */
typedef struct {
  int64_t tets;       /* tets (triangles) of the body */
  int64_t zero_tets;  /* of zero volume (skipped by the assembly) */
  int64_t pairs;      /* (tet, component, cell) candidate pairs (unstructured:
                         (solid tet, fluid tet) pairs) */
  int64_t pieces;     /* pairs whose piece the last assembly kept (volume >
                         1e-14 |T|); -1 for a coupling built with
                         IBVT_NO_STORE_B, which keeps no per-pair data */
  double volume;      /* Σ |T| over the body (area for a planar mesh) */
} ibvt_body_info;

/*
 * coupling_body_info — per-body counters of the last assembly, for meshes
 *   made of several bodies (a diagnostic: it synchronises the stream).
 *   Body b holds tets tet_offsets[b] .. tet_offsets[b+1] - 1; tet_offsets
 *   is a host array of n_bodies + 1 non-decreasing entries, the first 0
 *   and the last n_tet.  out: host array of n_bodies entries.  Summed over
 *   the bodies, the counters equal coupling_info's pairs, pieces and
 *   zero_tets.
 *   Errors: IBVT_E_INVALID (NULL pointers, n_bodies < 1, bad offsets, a
 *   handle whose last assembly failed), IBVT_E_NOMEM, IBVT_E_HIP.
 */
int coupling_body_info(ibvt_coupling* c, int32_t n_bodies, const int64_t* tet_offsets,
                       ibvt_body_info* out, hipStream_t stream);

/*
 * coupling_export_csr — copy B^d (transposed = 0: rows = solid vertices) or
 *   B^dT (transposed = 1: rows = touched fluid nodes, row_map[r] = global
 *   fluid index of row r) to HOST buffers, values as double.  Call first
 *   with row_ptr = col = val = row_map = NULL to get *n_rows and *nnz; then
 *   with buffers of n_rows+1, nnz, nnz and n_rows entries (row_map may stay
 *   NULL).  Synchronizes the device.  Errors: IBVT_E_INVALID, IBVT_E_HIP.
 */
int coupling_export_csr(const ibvt_coupling* c, int comp, int transposed, int64_t* n_rows,
                        int64_t* nnz, int32_t* row_ptr, int32_t* col, double* val,
                        int32_t* row_map);

/* coupling_free — release the handle and its device memory (synchronizes
 * the device).  NULL is a no-op. */
void coupling_free(ibvt_coupling* c);

/* ibvt_status_string — static text for a status code. */
const char* ibvt_status_string(int status);

/* ibvt_last_error — thread-local detail message of the last failing call. */
const char* ibvt_last_error(void);

/*
 * ibvt_lattice_coords — node coordinates of component comp's lattice along
 *   axis (HOST output, n entries; pass out = NULL to get *n).  Component d
 *   uses the face coordinates along axis d and the face midpoints elsewhere
 *   (staggered grid, Section 2.2).  Errors: IBVT_E_INVALID.
 */
int ibvt_lattice_coords(const ibvt_grid* grid, int comp, int axis, double* out, int64_t* n);

/* ibvt_lattice_coords_2d — the same for a planar grid (comp, axis in {0, 1}). */
int ibvt_lattice_coords_2d(const ibvt_grid2d* grid, int comp, int axis, double* out, int64_t* n);

/*
 * Fixed-point (Picard) fluid-structure coupling, Section 3 Steps 1-6.
 *
 * fsi_step advances one time step.  It assembles T = S^{-1} B at the
 * current configuration X = X_ref + u_hat0 (reassemble_coupling; the
 * transfer follows the solid, Section 2.3), then iterates l = 1, 2, ...:
 *   Step 1  w_s = T v_f                         (transfer_velocity, cfg->mass)
 *   Step 2  u_hat = u_hat0 + dt w_s
 *   Step 3  f_fsi = solid(u_hat)                 (caller's solid solver)
 *   Step 4  f_tilde = alpha T^T f_fsi            (the literal transpose
 *           B^T S^{-1} on the load f_fsi; with cfg->force_density != 0 the
 *           result is divided node by node by the fluid nodes' lumped
 *           volume, Q1 over a lattice's hull or P1 on an unstructured
 *           background, giving a force density for the fluid solver)
 *   Step 5  v_f = fluid(f_tilde)                 (caller's fluid solver)
 *   Step 6  stop when ||f_fsi,l − f_fsi,l−1||_inf < eps_abs (eq. AC) or
 *           that norm / ||f_fsi,1||_inf < eps_rel (eq. RC); f_fsi,0 is the
 *           caller's `f_prev` on entry (e.g. the previous step's force).
 * Readings (the paper leaves them open): T is held fixed within the step;
 * the reference norm of eq. RC is the first iteration's force.
 *
 * Callbacks run on the calling thread and enqueue their work on `stream`;
 * they return an ibvt status (non-zero stops the step with that status).
 * With nc the coupling's component count (3, or 2 for a planar coupling):
 *   solid(ctx, u_hat (nc, n_vert), f_fsi (nc, n_vert) out, stream)
 *   fluid(ctx, f_tilde[nc] in, v_f[nc] out (may alias the caller's v_f), stream)
 *
 * Buffers (device, caller-owned; solid fields (nc, n_vert), fluid fields per
 * component as in the transfers, in the coupling's precision; X_ref double
 * (n_vert, dim)): X_ref, u_hat0 in; v_f in/out; u_hat, w_s, f_fsi, f_tilde
 * out; f_prev in (f_fsi,0) and overwritten (workspace).  A planar coupling
 * reads v_f[0..1] and f_tilde[0..1] only.
 * Errors: IBVT_E_INVALID (arguments, consistent mass not built, dual basis
 * with IBVT_CONSISTENT),
 * IBVT_E_NOT_CONVERGED (max_iter reached; results of the last iteration are
 * written), or the status of a failed call or callback.
 */
typedef int (*ibvt_solid_fn)(void* ctx, const void* u_hat, void* f_fsi, hipStream_t stream);
typedef int (*ibvt_fluid_fn)(void* ctx, void* const f_tilde[3], void* const v_f[3],
                             hipStream_t stream);

typedef struct {
  double dt;              /* Δt of Step 2 */
  double alpha;           /* L_ref / (ρ_f U_ref²) of Step 4 */
  double eps_abs;         /* eq. AC threshold (<= 0: not used) */
  double eps_rel;         /* eq. RC threshold (<= 0: not used) */
  int32_t max_iter;       /* Picard iterations, >= 1 */
  int32_t mass;           /* IBVT_LUMPED or IBVT_CONSISTENT for T */
  int32_t force_density;  /* divide f_tilde by the fluid nodes' lumped volume */
  int32_t cg_maxit;       /* consistent-mass solve: iteration limit */
  double cg_rtol;
} ibvt_fsi_config;

typedef struct {
  const double* X_ref;    /* (n_vert, dim) reference configuration */
  const void* u_hat0;     /* (nc, n_vert) displacement at the start of the step */
  void* u_hat;            /* (nc, n_vert) out */
  void* w_s;              /* (nc, n_vert) out: transferred velocity */
  void* f_fsi;            /* (nc, n_vert) out: reaction force, last iteration */
  void* f_prev;           /* (nc, n_vert) in: f_fsi,0; workspace */
  void* v_f[3];           /* fluid velocity, in/out */
  void* f_tilde[3];       /* transferred force, out */
} ibvt_fsi_buffers;

typedef struct {
  int32_t iterations;     /* Picard iterations done */
  int32_t converged;      /* 1 if eq. AC or eq. RC held */
  double res_abs;         /* ||f_fsi,l − f_fsi,l−1||_inf at exit */
  double res_rel;         /* res_abs / ||f_fsi,1||_inf */
  double f1_norm;         /* ||f_fsi,1||_inf */
} ibvt_fsi_report;

int fsi_step(ibvt_coupling* c, const ibvt_fsi_config* cfg, const ibvt_fsi_buffers* buf,
             ibvt_solid_fn solid, void* solid_ctx, ibvt_fluid_fn fluid, void* fluid_ctx,
             hipStream_t stream, ibvt_fsi_report* report);

/*
 * ibvt_fluid_lumped_volume — the Q1 lumped volume ∫ N_j of every node of
 * component comp's lattice (the row sums of the fluid lattice's Q1 mass),
 * a product of 1D hat integrals over the lattice hull: out (device, double,
 * (n_z, n_y, n_x)).  Used to turn transferred loads into force densities.
 * Errors: IBVT_E_INVALID.
 */
int ibvt_fluid_lumped_volume(const ibvt_grid* grid, int comp, double* out, hipStream_t stream);

/*
 * ibvt_fluid_lumped_volume_2d — the planar counterpart: the Q1 lumped area
 * ∫ N_j dA of every node of component comp (0 or 1) of a planar grid, a
 * product of two 1D hat integrals over the lattice hull: out (device,
 * double, (n_y, n_x)).  Errors: IBVT_E_INVALID.
 */
int ibvt_fluid_lumped_volume_2d(const ibvt_grid2d* grid, int comp, double* out,
                                hipStream_t stream);

/*
 * Kernel tracing (process-wide; no paper counterpart).  While enabled, the
 * library records a HIP event pair on the caller's stream around each of
 * its main kernel launches.  ibvt_profile_read synchronizes those events and
 * returns, per kernel name, the number of launches and the summed device
 * time in milliseconds (up to max entries, sorted by name); it also clears
 * the records.  names[k] points to static strings.  Returns the number of
 * entries written, or -IBVT_E_HIP.
 */
void ibvt_profile_enable(int on);
int ibvt_profile_read(const char** names, int64_t* launches, double* ms, int max);

#ifdef __cplusplus
}
#endif

#endif /* IBVT_H */
