/*
 * grb.h — C ABI of an MI355X (gfx950) library for the masked matrix-vector
 * multiply over a semiring, the operation GraphBLAST (Yang, Buluc, Owens,
 * "GraphBLAST: A High-Performance Linear Algebra-based Graph Framework on
 * the GPU", ACM TOMS 2021) builds its graph algorithms on.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - All graph and vector buffers are DEVICE memory owned by the caller and
 *   only borrowed by the library.  The library never allocates device
 *   memory: temporary storage comes from a caller-provided workspace whose
 *   size grb_workspace_size() reports.
 * - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *   Work is enqueued on it and the call returns without waiting, except
 *   where a function is documented as synchronising.
 * - Indices are int32: a matrix may hold at most 2^31 - 1 stored entries
 *   and 2^31 - 1 rows/columns.
 * - Every call returns grb_info.  Argument errors are detected on the host,
 *   before anything is enqueued, and leave all buffers untouched.  A device
 *   fault surfaces as GRB_PANIC from the next synchronising call or from
 *   grb_stream_check().  No C++ exception crosses this interface.
 * - Handles (grb_matrix, grb_vector) are host objects.  A matrix is
 *   read-only once prepared and may be used from several streams at once;
 *   a vector and a workspace may be used by one call at a time.
 */
#ifndef GRB_H
#define GRB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Error codes, named after the GraphBLAS C API codes the paper defers to
 * (caption of the mxv figure, Section 3.3). */
typedef enum grb_info {
  GRB_SUCCESS = 0,
  GRB_NO_VALUE = 1,
  GRB_UNINITIALIZED_OBJECT = 2, /* NULL handle, or matrix not prepared */
  GRB_NULL_POINTER = 3,         /* required pointer argument is NULL */
  GRB_INVALID_VALUE = 4,        /* bad size, flag, enum or parameter */
  GRB_INVALID_INDEX = 5,        /* vertex id out of range */
  GRB_DOMAIN_MISMATCH = 6,      /* vector/matrix type does not fit the semiring */
  GRB_DIMENSION_MISMATCH = 7,   /* operand sizes disagree */
  GRB_NOT_IMPLEMENTED = 8,      /* combination this library does not provide */
  GRB_INSUFFICIENT_SPACE = 9,   /* workspace or metadata buffer too small */
  GRB_OUT_OF_MEMORY = 10,       /* host allocation failed */
  GRB_PANIC = 11                /* HIP runtime or device error */
} grb_info;

/* Element types.  GRB_BOOL is one byte per element (0 = false). */
typedef enum grb_type {
  GRB_BOOL = 0,
  GRB_INT32 = 1,
  GRB_FP32 = 2,
  GRB_FP64 = 3
} grb_type;

/*
 * Semirings (Table 4 of the paper): (add, multiply, domain, identity).
 * A matrix without values acts as if every stored entry were 1 (true).
 *   LOR_LAND    (or, and, {0,1}, false)      structure-only traversal (BFS)
 *   MIN_PLUS    (min, +, R u {+inf}, +inf)   shortest paths
 *   PLUS_TIMES  (+, *, R, 0)                 classical products (PageRank)
 *   MIN_FIRST   (min, first, int32, INT32_MAX)
 *   MIN_SECOND  (min, second, int32, INT32_MAX)
 *   PLUS_PAIR   (+, pair = 1, int32, 0)       common-index counts (masked SpGEMM)
 * For mxv the multiply is A(i,j) (x) u(j); for vxm it is u(i) (x) A(i,j).
 * So vxm with MIN_FIRST, or mxv with MIN_SECOND, returns the smallest
 * vector value among the contributing neighbours: with u(j) = j on the
 * frontier that is the smallest-id parent.
 */
typedef enum grb_semiring {
  GRB_LOR_LAND_BOOL = 0,
  GRB_MIN_PLUS_FP32 = 1,
  GRB_MIN_PLUS_FP64 = 2,
  GRB_PLUS_TIMES_FP32 = 3,
  GRB_PLUS_TIMES_FP64 = 4,
  GRB_MIN_FIRST_INT32 = 5,
  GRB_MIN_SECOND_INT32 = 6,
  GRB_PLUS_PAIR_INT32 = 7 /* structure only: each common index counts 1
                             (grb_mxm_masked only) */
} grb_semiring;

/* Optional accumulator applied between the old output and the product
 * (GraphBLAS C API semantics; the accumulator must be the semiring's add:
 * LOR for LOR_LAND, MIN for MIN_*, PLUS for PLUS_TIMES). */
typedef enum grb_binop {
  GRB_NOACCUM = 0,
  GRB_ACCUM_MIN = 1,
  GRB_ACCUM_PLUS = 2,
  GRB_ACCUM_LOR = 3
} grb_binop;

/* Descriptor flags (Table 3 of the paper, plus REPLACE and a structural
 * mask from the GraphBLAS C API). */
#define GRB_MASK_COMP   0x1u /* use the structural complement of the mask */
#define GRB_MASK_STRUCT 0x2u /* mask by presence instead of by value */
#define GRB_TRAN_A      0x4u /* transpose the matrix operand */
#define GRB_REPLACE     0x8u /* clear output entries outside the mask */
#define GRB_PROFILE     0x10u /* drivers: time expand kernels with HIP events */
/* drivers, test hook for the failure path of the multi-workgroup level loop
 * of BFS / bucketed SSSP on low-degree graphs: every barrier of the loop is
 * given up at its first unfinished poll (as when some of the loop's
 * workgroups are not resident), so the search continues in the level
 * kernels from there; results are unchanged. */
#define GRB_LOOP_NO_WAIT 0x20u

/* Direction of a product (Section 4): push = sparse-vector SpMSpV over the
 * input's nonzeros; pull = masked SpMV over the allowed output rows. */
typedef enum grb_direction {
  GRB_DIR_AUTO = 0,
  GRB_DIR_PUSH = 1,
  GRB_DIR_PULL = 2
} grb_direction;

/*
 * Switch rule for GRB_DIR_AUTO (Table 5 and Section 4.3.1 of the paper).
 *   PAPER: estimate |E_f| = (nnz/n) * nnz(u) and assume |E_u| = nnz, so
 *          pull iff denominator * nnz(u) > n.
 *   EXACT: |E_f| = sum of the input's row degrees (computed on the device
 *          while the input is compacted): pull iff denominator * |E_f| > nnz.
 * Equality picks push.  Results never depend on the rule, only speed.
 */
typedef enum grb_switch_rule {
  GRB_SWITCH_PAPER = 0,
  GRB_SWITCH_EXACT = 1
} grb_switch_rule;

typedef struct grb_descriptor {
  uint32_t flags;             /* GRB_MASK_COMP | GRB_MASK_STRUCT | ... */
  int32_t direction;          /* grb_direction */
  int32_t switch_rule;        /* grb_switch_rule */
  int32_t switch_denominator; /* 0 selects the paper's 10 */
  int32_t max_iter;           /* drivers: iteration cap, 0 = unlimited */
  int32_t reserved[3];        /* must be zero */
} grb_descriptor;

/* Fills d with the defaults: no flags, AUTO, PAPER rule, denominator 10. */
grb_info grb_descriptor_init(grb_descriptor *d);

typedef struct grb_matrix_s *grb_matrix;
typedef struct grb_vector_s *grb_vector;

/* ------------------------------------------------------------------ */
/* Graph construction on the host (setup, not part of any timed path)  */
/* ------------------------------------------------------------------ */

typedef struct grb_csr_builder_s *grb_csr_builder;

/*
 * Builds a CSR graph on the host from a raw edge list (host arrays), as
 * the paper prepares its datasets (dataset table caption, Section 8):
 * self-loops dropped; with `symmetrise` each (u, v) also gives (v, u);
 * duplicates collapse to one entry keeping the smallest weight; rows end up
 * sorted by column.  w may be NULL (structure only).  Swapping src and dst
 * builds the transpose.  Errors: GRB_NULL_POINTER, GRB_INVALID_VALUE (n or
 * m negative, n >= 2^31), GRB_INVALID_INDEX (endpoint outside [0, n)),
 * GRB_OUT_OF_MEMORY, GRB_INVALID_VALUE if the result exceeds 2^31-1 entries.
 */
grb_info grb_csr_build(grb_csr_builder *b, int64_t n, int64_t m, const int32_t *src,
                       const int32_t *dst, const float *w, int symmetrise);
/* Number of stored entries of the built CSR. */
grb_info grb_csr_nnz(grb_csr_builder b, int64_t *nnz);
/* Copies the CSR out to host arrays: row_ptr (n+1), col_idx (nnz), values
 * (nnz floats; may be NULL, must be NULL if built without weights). */
grb_info grb_csr_copy(grb_csr_builder b, int32_t *row_ptr, int32_t *col_idx, float *values);
grb_info grb_csr_free(grb_csr_builder *b);

/*
 * Triangle-counting input (Section 7.5 counts triangles as the sum of
 * L L^T .* L, L the strict lower triangle, rows ordered by degree): from a
 * built symmetric CSR `src`, renumbers the vertices by decreasing degree
 * (ties by increasing id) and keeps, in row i, the neighbours numbered
 * below i (so every row holds at most sqrt(2 nnz) entries), rows sorted.
 * *out receives a new builder (structure only; read it with grb_csr_nnz /
 * grb_csr_copy, release it with grb_csr_free); rank (n entries, may be
 * NULL) the new number of each vertex.  Errors: GRB_NULL_POINTER,
 * GRB_OUT_OF_MEMORY.
 */
grb_info grb_csr_lower_by_degree(grb_csr_builder src, grb_csr_builder *out, int32_t *rank);

/* ------------------------------------------------------------------ */
/* Matrix                                                              */
/* ------------------------------------------------------------------ */

#define GRB_MATRIX_SYMMETRIC 0x1u /* A == A^T: the CSR also serves as CSC */

/*
 * Wraps caller-owned device CSR arrays (borrowed, must stay alive and
 * unchanged while the handle is used):
 *   row_ptr[nrows+1], col_idx[nnz] with columns ascending inside each row,
 *   values[nnz] of vtype (GRB_FP32/GRB_FP64/GRB_INT32) or NULL;
 *   t_row_ptr/t_col_idx/t_values: the CSR of A^T (= CSC of A), or NULL.
 * Paper, Section 4.3.3: CSR serves row access (pull), CSC column access
 * (push).  With GRB_MATRIX_SYMMETRIC the transpose arguments must be NULL
 * and the CSR is used for both.  A product whose chosen direction needs a
 * missing orientation fails with GRB_NOT_IMPLEMENTED (AUTO falls back to
 * the direction that is available).
 */
grb_info grb_matrix_create(grb_matrix *A, int64_t nrows, int64_t ncols, int64_t nnz,
                           const int32_t *row_ptr, const int32_t *col_idx,
                           const void *values, grb_type vtype,
                           const int32_t *t_row_ptr, const int32_t *t_col_idx,
                           const void *t_values, uint32_t flags);
grb_info grb_matrix_free(grb_matrix *A);
grb_info grb_matrix_nrows(grb_matrix A, int64_t *n);
grb_info grb_matrix_ncols(grb_matrix A, int64_t *n);
grb_info grb_matrix_nvals(grb_matrix A, int64_t *nnz);

/*
 * Derived metadata is built into a caller-owned device buffer of at least
 * *bytes bytes, per CSR: pieces of long rows (for the push and pull
 * kernels), runs of bitmap words of about equal work (for full sweeps), a
 * bitmap of the empty rows, and the first two column ids of every row.
 * grb_matrix_prepare synchronises `stream` (it reads the row pointers back
 * to build the lists).  Every product and driver requires a prepared
 * matrix (else GRB_UNINITIALIZED_OBJECT), except the masked matrix product
 * and the triangle count.  The buffer is borrowed like the CSR.
 */
grb_info grb_matrix_meta_size(grb_matrix A, size_t *bytes);
grb_info grb_matrix_prepare(grb_matrix A, void *meta, size_t meta_bytes, void *stream);

/* ------------------------------------------------------------------ */
/* Vector                                                              */
/* ------------------------------------------------------------------ */

/*
 * Wraps caller-owned device storage of a length-n vector (the Vector
 * object of Section 3.1.2; the dense and sparse storage formats of Section
 * 4.3.3, between which the backend, not the user, converts):
 *   values[n]  elements of `type`, the value of index i at values[i]; or
 *              NULL: every present entry has the value 1 (true).  Such a
 *              vector can be an input or a mask, not a product's output;
 *   bitmap[(n+63)/64]  presence words, bit (i % 64) of word i / 64, bits at
 *              positions >= n zero; or NULL;
 *   indices[n] + count  the sparse form: count (one DEVICE int32) present
 *              indices, sorted ascending without repeats, in indices[0..count);
 *              both NULL or both given.
 * At least one of bitmap and indices must be given (n > 0), else
 * GRB_NULL_POINTER.  A vector with both keeps them equal: the library
 * writes both whenever it writes the vector, and a caller that writes one
 * must write the other.  In a product the list form of the input feeds
 * push directly (no compaction), the bitmap feeds pull (built from the list
 * in the workspace when the vector has no bitmap); a mask or output given
 * only as a list is converted through the workspace, and an output's list
 * is rebuilt from its new bitmap after the product.  A list that is not
 * sorted or has repeats gives an undefined result (memory accesses stay
 * inside the arrays).  Errors: GRB_NULL_POINTER, GRB_INVALID_VALUE (n
 * negative or >= 2^31 - 1, bad type), GRB_OUT_OF_MEMORY.
 */
grb_info grb_vector_create(grb_vector *v, int64_t n, grb_type type, void *values,
                           uint64_t *bitmap, int32_t *indices, int32_t *count);
grb_info grb_vector_free(grb_vector *v);
grb_info grb_vector_size(grb_vector v, int64_t *n);
/* Removes every entry (presence bits cleared, count set to 0; values untouched). */
grb_info grb_vector_clear(grb_vector v, void *stream);
/* Every index present with the value *scalar (host pointer to one element;
 * may be NULL for a vector without values); the list becomes 0..n-1. */
grb_info grb_vector_fill(grb_vector v, const void *scalar, void *stream);
/*
 * Clears v, then sets v(idx[k]) = vals[k] for k < count, from DEVICE arrays
 * idx (int32) and vals (`type`, or NULL: every value 1).  Indices must be
 * in [0, n) (out-of-range entries are skipped); with duplicate indices one
 * of their values is kept.  A vector keeping a list gets it rebuilt from the
 * bitmap (one workgroup; a setup-time call).  Needs the bitmap form (a
 * list-only vector is written by its owner: GRB_NOT_IMPLEMENTED); vals with
 * a vector without values: GRB_INVALID_VALUE.
 */
grb_info grb_vector_build(grb_vector v, const int32_t *idx, const void *vals,
                          int64_t count, void *stream);
/* Number of present entries.  Synchronises `stream`; needs a workspace of
 * at least 64 bytes. */
grb_info grb_vector_nvals(grb_vector v, int64_t *nvals, void *ws, size_t ws_bytes,
                          void *stream);
/*
 * Copies the present entries to HOST memory (GraphBLAS extractTuples):
 * indices[k] (int32, ascending) and values[k] (`type`) for k < *nvals;
 * either output may be NULL.  Device-side work (compaction of the bitmap
 * unless the vector keeps a list, gather of the values) uses a workspace of
 * grb_workspace_size(GRB_OP_EXTRACT, NULL, n) bytes.  Synchronises
 * `stream`.  *nvals is always set; with *nvals > capacity nothing is
 * copied and GRB_INSUFFICIENT_SPACE is returned.  Errors also
 * GRB_NULL_POINTER (nvals), GRB_INVALID_VALUE (capacity < 0), GRB_PANIC.
 */
grb_info grb_vector_extract(grb_vector v, int32_t *indices, void *values, int64_t capacity,
                            int64_t *nvals, void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------ */
/* Workspace                                                           */
/* ------------------------------------------------------------------ */

typedef enum grb_op {
  GRB_OP_MXV = 0,      /* grb_mxv / grb_vxm with this matrix */
  GRB_OP_BFS = 1,
  GRB_OP_SSSP = 2,
  GRB_OP_PAGERANK = 3, /* k = 1 for fp32, 2 for fp64 */
  GRB_OP_MSBFS = 4,    /* k = number of sources (batched BFS) */
  GRB_OP_NVALS = 5,
  GRB_OP_MXM = 6,      /* grb_mxm_masked and grb_tricount (A unused) */
  GRB_OP_EXTRACT = 7,  /* grb_vector_extract: k = vector length (A unused) */
  GRB_OP_CC = 8        /* grb_cc */
} grb_op;

/* Bytes of device workspace the operation needs on matrix A.  Workspace
 * contents need no initialisation; the address must be 256-byte aligned. */
grb_info grb_workspace_size(grb_op op, grb_matrix A, int64_t k, size_t *bytes);

/* ------------------------------------------------------------------ */
/* The masked semiring products                                        */
/* ------------------------------------------------------------------ */

/*
 * w<mask> = accum(w, A u) over semiring s (Section 3.3 and the mxv figure
 * caption: w = A u .* mask; descriptor per Table 3).  With GRB_TRAN_A the
 * product uses A^T.  Definition (per output index i):
 *   t(i) = (+)_{j : A'(i,j) stored and u(j) present} A'(i,j) (x) u(j);
 *          t(i) exists iff that set is non-empty;
 *   z = t without accum; with accum z(i) = accum(w(i), t(i)) where both
 *          exist, else whichever exists;
 *   allowed(i) = no mask, or (m(i) xor GRB_MASK_COMP) where m(i) means
 *          "mask(i) present and non-zero" (or "present" with GRB_MASK_STRUCT);
 *   w(i) := z(i) (absent if z(i) is) where allowed; elsewhere w keeps its
 *          entry, or loses it under GRB_REPLACE.
 * Direction: d->direction forces push or pull; AUTO applies d->switch_rule
 * on the device (no host synchronisation).  Push needs the CSR of A'^T,
 * pull the CSR of A'.  Results are identical in either direction for
 * LOR_LAND, MIN_* (any order) and bitwise-reproducible for PLUS_TIMES in
 * pull; PLUS_TIMES in push uses atomic adds (order-dependent rounding).
 * Types: u, w (and accum) must have the semiring's domain type (BOOL,
 * INT32, FP32 or FP64); the mask may have any type.  w must not alias u or
 * the mask.  d may be NULL (defaults).
 * Errors: GRB_UNINITIALIZED_OBJECT, GRB_DIMENSION_MISMATCH, GRB_DOMAIN_MISMATCH,
 * GRB_INVALID_VALUE, GRB_NOT_IMPLEMENTED, GRB_INSUFFICIENT_SPACE, GRB_PANIC.
 */
grb_info grb_mxv(grb_vector w, grb_vector mask, grb_binop accum, grb_semiring s,
                 grb_matrix A, grb_vector u, const grb_descriptor *d, void *ws,
                 size_t ws_bytes, void *stream);

/* w<mask> = accum(w, u A): t(j) = (+)_i u(i) (x) A'(i,j); otherwise as
 * grb_mxv (vxm is mxv on the transposed matrix, decomposition figure). */
grb_info grb_vxm(grb_vector w, grb_vector mask, grb_binop accum, grb_semiring s,
                 grb_vector u, grb_matrix A, const grb_descriptor *d, void *ws,
                 size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------ */
/* Graph algorithms built on the products (Section 7)                  */
/* ------------------------------------------------------------------ */

/*
 * Direction-optimised BFS from `source` (Algorithm 1; Section 7.1):
 * each level computes f <- A^T f .* not(visited) over LOR_LAND, pushing or
 * pulling per the descriptor's rule, with early exit in pull.
 * levels[n]: hop count (source 0, unreached -1; the paper's d minus one).
 * parents[n] (may be NULL): smallest-id neighbour one level closer
 * (source: itself, unreached: -1).  A must be square; the traversal follows
 * stored entries A(u, v) from u to v (push reads the CSR of A, pull the
 * CSR of A^T; a symmetric matrix serves both).
 * Synchronises `stream` once per batch of levels (it reads the frontier
 * size back to detect the end); the first batch covers the depth expected
 * of a random graph of A's size and mean degree, or the depth of the last
 * search on A where that is larger (up to twice the estimate).  A's handle
 * keeps that depth (an atomic int, so concurrent calls on one matrix stay
 * safe; it affects speed only).  d->max_iter caps the levels (0 = none).
 * On graphs whose rows are short (at most 64 entries: road-like, high
 * diameter) the levels run back to back inside one kernel of 16 workgroups,
 * separated by a barrier of its own, while the frontier is small (a launch
 * per level would dominate); a frontier that outgrows its queues (more
 * than 256 vertices found by one wave of 64 lanes, or 65,536 edges), that
 * the switch rule would pull, or a barrier not reached by every workgroup
 * within 1 ms, continues with one kernel per level.  Results do not depend
 * on where that hand-over happens.
 */
grb_info grb_bfs(int32_t *levels, int32_t *parents, grb_matrix A, int32_t source,
                 const grb_descriptor *d, void *ws, size_t ws_bytes, void *stream);

/*
 * grb_bfs for callers that cannot allocate (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): the same BFS,
 * levels and parents as grb_bfs, with its workspace in a device array of
 * the library (9 MiB, held on each GPU the library runs on until
 * the process ends) instead of a caller buffer; read-backs use no pinned
 * staging buffer; GRB_PROFILE is ignored (it would create timing events).
 * Graphs of more than 2^24 vertices: GRB_INSUFFICIENT_SPACE.  Runs on the
 * current device, whose array is found on the first call there.  All calls
 * on one GPU share its array: calls that overlap on one GPU race (issue them
 * from one stream, one at a time).  Other errors and synchronisation as
 * grb_bfs.
 */
grb_info grb_bfs_noalloc(int32_t *levels, int32_t *parents, grb_matrix A, int32_t source,
                         const grb_descriptor *d, void *stream);

/*
 * SSSP from `source` (Section 7.2): Bellman-Ford over MIN_PLUS with the
 * frontier sparsified to the vertices whose distance improved in the last
 * round; stops when none improved.  dist[n] (fp32): +inf where unreached.
 * A must carry FP32 values (else GRB_DOMAIN_MISMATCH), none negative or NaN
 * (checked by grb_matrix_prepare; else GRB_INVALID_VALUE).  Synchronises
 * like grb_bfs.
 */
grb_info grb_sssp(float *dist, grb_matrix A, int32_t source, const grb_descriptor *d,
                  void *ws, size_t ws_bytes, void *stream);

/*
 * SSSP from `source` (the computation of Section 7.2) in distance buckets
 * of width `delta` > 0: each round relaxes, by push, only the pending
 * vertices whose distance is below (B + 1) * delta for the current bucket
 * B; the others stay pending, and B moves to the nearest pending bucket
 * once none is left below the limit.  Reaches the same exact distances as
 * grb_sssp with far fewer relaxations on high-diameter graphs (the paper's
 * Bellman-Ford rounds relax a grid's edges over a hundred times each).
 * dist[n], A, workspace (GRB_OP_SSSP) and synchronisation as grb_sssp; the
 * descriptor's direction must be AUTO or PUSH (PULL: GRB_NOT_IMPLEMENTED);
 * delta not finite and positive: GRB_INVALID_VALUE.  Stats record per round
 * the pending count, the near degree sum, direction 1 and the bucket.  On
 * graphs whose rows are short (at most 64 entries) the rounds run back to
 * back inside one kernel of 32 workgroups (the device-side loop of
 * grb_bfs, with its barrier, limits and hand-over) while the pending set
 * is small; on the 3000 x 3000 grid a width of 384-512 keeps every round
 * there.
 */
grb_info grb_sssp_delta(float *dist, grb_matrix A, int32_t source, float delta,
                        const grb_descriptor *d, void *ws, size_t ws_bytes, void *stream);

/*
 * PageRank (Section 7.3, pull form, always SpMV since the vector stays
 * dense).  A holds the out-edges u -> v and must carry the CSR of A^T (or be
 * symmetric).  p[n] of `type` (GRB_FP32 or GRB_FP64) receives the ranks:
 * p0 = 1/n; per iteration D = sum of p over vertices without out-edges,
 * p'(v) = (1-damping)/n + damping * (sum_{u->v} p(u)/outdeg(u) + D/n),
 * delta = ||p' - p||_1; stops after max_iter iterations or once
 * delta < tol.  *iters receives the number of iterations run and
 * *delta_out (may be NULL) the last delta.  Synchronises once at the end.
 */
grb_info grb_pagerank(void *p, grb_type type, grb_matrix A, double damping,
                      int32_t max_iter, double tol, int32_t *iters, double *delta_out,
                      const grb_descriptor *d, void *ws, size_t ws_bytes, void *stream);

/*
 * Adaptive PageRank (PageRankDelta, the masked PageRank of Sections 5.1
 * and 7.3: the mask holds the vertices that have converged, which are no
 * longer updated, so an iteration touches only the in-edges of the active
 * rows).  As grb_pagerank, except that each iteration updates only the
 * active vertices (a frozen vertex keeps its value, and D still sums the
 * frozen dangling ones) and then freezes every active v whose change
 * satisfies |p'(v) - p(v)| <= eps * p(v), p(v) being the previous iterate.
 * Stops after max_iter iterations, once delta < tol, or when no vertex is
 * left active.  *active_out (may be NULL) receives the count still active.
 * Stats record per iteration the active vertices, their in-edges, direction
 * pull and the count active after it.  Same workspace as grb_pagerank
 * (GRB_OP_PAGERANK).  eps negative or not finite: GRB_INVALID_VALUE; other
 * errors as grb_pagerank.
 */
grb_info grb_pagerank_adaptive(void *p, grb_type type, grb_matrix A, double damping,
                               int32_t max_iter, double tol, double eps, int32_t *iters,
                               double *delta_out, int64_t *active_out,
                               const grb_descriptor *d, void *ws, size_t ws_bytes,
                               void *stream);

/*
 * Connected components (Section 7.4: FastSV, the linear-algebraic form of
 * Shiloach-Vishkin hooking and shortcutting).  labels[n] (int32) receives,
 * for every vertex, the smallest vertex id of its component (weak
 * components of a directed matrix: A must then carry the CSR of A^T, else
 * GRB_NOT_IMPLEMENTED).  Each iteration takes the smallest grandparent among
 * the neighbours with grb_mxv over MIN_SECOND (accumulated with min), then
 * hooks the old parent and the vertex to it, shortcuts to the grandparent
 * and recomputes the grandparents; it stops once no grandparent changes or
 * after d->max_iter iterations (0 = no cap).  *iters (may be
 * NULL) receives the iterations run.  The descriptor may carry no flags but
 * GRB_PROFILE; its direction and switch rule apply to the products.
 * Workspace: GRB_OP_CC.  Synchronises once per batch of iterations.
 */
grb_info grb_cc(int32_t *labels, grb_matrix A, int32_t *iters, const grb_descriptor *d,
                void *ws, size_t ws_bytes, void *stream);

/*
 * Masked sparse matrix-matrix product in the dot-product form (Section 6.3.4,
 * masked SpGEMM): for every entry (i, j) of the mask M,
 *   c[e] = sum over k of A(i, k) * B(j, k)    (e = the entry's position
 *                                              in M's CSR arrays),
 * i.e. C = (A B^T) .* M with B given by its rows, the form triangle
 * counting uses (A = B = M = L).  Only the mask's entries are computed; an
 * entry whose rows share no index gets 0.  Semirings: GRB_PLUS_TIMES_FP32
 * and _FP64 (A and B carry values of that type; c is float / double) and
 * GRB_PLUS_PAIR_INT32 (structure only, every common index counts 1; c is
 * int32); others GRB_NOT_IMPLEMENTED.  Needs M.nrows = A.nrows,
 * M.ncols = B.nrows, A.ncols = B.ncols (else GRB_DIMENSION_MISMATCH); rows
 * of A and B sorted by column; the mask is structural, so the descriptor
 * may only carry GRB_PROFILE (other flags GRB_NOT_IMPLEMENTED).  The
 * matrices need not be prepared.  Workspace: GRB_OP_MXM.  Asynchronous.
 */
grb_info grb_mxm_masked(void *c, grb_matrix M, grb_matrix A, grb_matrix B, grb_semiring s,
                        const grb_descriptor *d, void *ws, size_t ws_bytes, void *stream);

/*
 * Triangle count (Section 7.5): *count (host) receives the sum of
 * (L L^T) .* L over the structure of L, which is the number of triangles
 * when L is the strict lower triangle of a symmetric adjacency under any
 * numbering (grb_csr_lower_by_degree builds the one that bounds the work).
 * The product and the reduction run fused in one kernel; nothing of the
 * product is stored.  L: square, rows sorted (else the result is undefined);
 * need not be prepared.  Workspace: GRB_OP_MXM.  Synchronises the stream.
 */
grb_info grb_tricount(int64_t *count, grb_matrix L, const grb_descriptor *d, void *ws,
                      size_t ws_bytes, void *stream);

/*
 * Batched multi-source BFS: k traversals at once as one masked product of
 * A^T with a bitmask block of frontiers (multi-nodeset traversal, Table 6
 * and Section 3.3; matrix-matrix direction optimisation is the paper's
 * future work, Section 9).  Each level pushes or pulls for the whole batch
 * (the descriptor's switch rule on the batch's frontier; PAPER compares
 * the frontier's (vertex, query) pairs with n*k, EXACT the out-edges of the
 * active (vertex, 64-query word) pairs with nnz per word).
 *   levels[n * k], VERTEX-major: levels[v * k + q] is the hop count from
 *          sources[q] to v (0 at the source, -1 unreached), as one
 *          single-source grb_bfs would give;
 *   sources[k]: device int32 vertex ids, repeats allowed;
 *   tile: query words per pass (1..ceil(k/64); each word is 64 queries)
 *          and workgroups per pass; NULL or zero fields pick defaults (the
 *          autotuner of the Python package writes tuned values).
 * Needs the CSR of A^T (or a symmetric matrix) for pull.  Synchronises
 * once per batch of levels.  Errors as grb_bfs, plus GRB_INVALID_VALUE for
 * k < 1 or a bad tile.  Source ids are device data: one outside [0, n) is
 * skipped on the device (nothing is written for it), the other queries run
 * to the end, and the call returns GRB_INVALID_INDEX.
 */
typedef struct grb_msbfs_tile {
  int32_t words_per_pass; /* kt, 0 = all words of the batch; at most 8 words are
                             taken per pass (larger values act as 8) */
  int32_t grid;           /* workgroups per pass, 0 = default */
  int32_t reserved[2];    /* must be zero */
} grb_msbfs_tile;

grb_info grb_msbfs(int32_t *levels, grb_matrix A, const int32_t *sources, int32_t k,
                   const grb_msbfs_tile *tile, const grb_descriptor *d, void *ws,
                   size_t ws_bytes, void *stream);

/*
 * Continuous batching of BFS queries (multi-nodeset traversal as one masked
 * matrix-matrix product, Table 6 and Section 3.3; a serving loop answers
 * the per-level launch and synchronisation cost the paper discusses in
 * Section 2.1.4): a session keeps k query lanes over one graph; queries
 * join free lanes and retire at level boundaries while the other lanes keep
 * running, so the batch never has to drain before new queries start.
 *   levels[n * k]  vertex-major level block (as grb_msbfs), caller-owned;
 *                  in a session, lane q's entry at v is valid only where the
 *                  lane's query has visited v; read results with
 *                  grb_msbfs_session_extract;
 *   ws             GRB_OP_MSBFS workspace for k (held for the session's life).
 * A lane's levels count from its own start: the source is 0.  Every call of
 * a session must use one stream.  create: all lanes free (tile, descriptor
 * and errors as grb_msbfs).
 */
typedef struct grb_msbfs_session_s *grb_msbfs_session;
grb_info grb_msbfs_session_create(grb_msbfs_session *ss, grb_matrix A, int32_t k,
                                  int32_t *levels, const grb_msbfs_tile *tile,
                                  const grb_descriptor *d, void *ws, size_t ws_bytes,
                                  void *stream);
/*
 * At the current level boundary, lane lanes[i] starts a BFS from
 * sources[i], for i < count (HOST arrays).  Errors (nothing is enqueued):
 * GRB_INVALID_INDEX (a lane outside [0, k) or a source outside [0, n)),
 * GRB_INVALID_VALUE (a lane still running or named twice, count outside
 * [0, k]).  Synchronises `stream`.
 */
grb_info grb_msbfs_session_join(grb_msbfs_session ss, const int32_t *lanes,
                                const int32_t *sources, int32_t count, void *stream);
/*
 * Runs up to max_levels levels (none when no lane is running), then
 * synchronises and reports in done[ceil(k / 64)] (HOST words, bit q % 64 of
 * word q / 64) the lanes whose query ended (its frontier is empty); they are
 * free again and keep their results until they join again.  *levels_run
 * (may be NULL) receives the number of levels run.
 */
grb_info grb_msbfs_session_step(grb_msbfs_session ss, int32_t max_levels, uint64_t *done,
                                int32_t *levels_run, void *stream);
/*
 * out[i * n + v] (DEVICE, lane-major) = level of the query of lane lanes[i]
 * (HOST array) at v, -1 where it did not reach v.  Synchronises `stream`.
 * Errors: GRB_INVALID_INDEX for a lane outside [0, k).
 */
grb_info grb_msbfs_session_extract(grb_msbfs_session ss, const int32_t *lanes, int32_t count,
                                   int32_t *out, void *stream);
grb_info grb_msbfs_session_free(grb_msbfs_session *ss);

/* ------------------------------------------------------------------ */
/* Statistics and errors                                               */
/* ------------------------------------------------------------------ */

#define GRB_STATS_MAX 256

/* Per-iteration record of the last driver call on this host thread. */
typedef struct grb_stats {
  int32_t op;            /* grb_op of the call */
  int32_t iterations;    /* levels / rounds / iterations run */
  int32_t recorded;      /* entries filled below (min(iterations, GRB_STATS_MAX)) */
  int32_t pushes;        /* iterations that ran push */
  int32_t pulls;         /* iterations that ran pull */
  int32_t launches;      /* expand launches enqueued (the last batch may end
                            with launches that find an empty frontier) */
  int64_t edges_push;    /* total sum of frontier degrees over push iterations */
  double expand_ms_push; /* GRB_PROFILE: summed push-expand kernel time */
  double expand_ms_pull; /* GRB_PROFILE: summed pull-expand kernel time */
  double expand_ms_all;  /* GRB_PROFILE: time of all `launches` expand launches */
  int32_t direction[GRB_STATS_MAX]; /* 1 push, 2 pull */
  int64_t frontier[GRB_STATS_MAX];  /* frontier size entering the iteration */
  int64_t edges[GRB_STATS_MAX];     /* sum of frontier degrees */
  float kernel_ms[GRB_STATS_MAX];   /* GRB_PROFILE: expand kernel time */
} grb_stats;

grb_info grb_last_stats(grb_stats *s);

/* Static English text for an error code. */
const char *grb_error_string(grb_info info);

/* Synchronises `stream` and reports a pending HIP error as GRB_PANIC. */
grb_info grb_stream_check(void *stream);

/* Library version as major * 10000 + minor * 100 + patch. */
int32_t grb_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GRB_H */
