/*
 * ifmm.h -- C ABI of the MI355X (gfx950) parallel inverse fast multipole method.
 *
 * The library computes an approximate factorisation of a dense N x N kernel
 * matrix A whose product with a vector an FMM can evaluate (Sec. 2 of
 * Takahashi, Chen and Darve, "Parallelization of the inverse fast multipole
 * method with an application to boundary element method"), and solves
 * A x = b with it, either directly or as the preconditioner of GMRES for a
 * boundary element system (Sec. 4, Alg. 4 and Alg. 5).
 *
 *   A_ij = K(p_i, p_j) * w_j   (i != j),   A_ii = diag_i,
 *   K(x, y) = 1 / (4 pi |x - y|)           (Laplace, 3-D)
 *
 * Method: uniform octree (Sec. 2.1), black-box Chebyshev FMM operators (the
 * "different FMM" Sec. 4.2 allows), the extended sparse system (eq. ext),
 * level-by-level block elimination with low-rank recompression of the
 * fill-in (Alg. 1), run colour by colour over a greedy sigma-separated
 * colouring (Alg. 3, Sec. 3.2 / 3.3), and the colour-ordered substitution
 * (Alg. 2).
 *
 * Conventions
 *  - Every call returns an ifmm_status and never aborts.  On failure a
 *    message is available from ifmm_last_error() (thread-local, valid until
 *    the next call on the same thread).
 *  - Inputs are borrowed for the duration of the call (and copied if kept).
 *    Outputs are allocated by the caller.
 *  - Arrays are row-major for points (N x 3) and column-major for right-hand
 *    sides / solutions (N x nrhs with leading dimension ld >= N).
 *  - Vectors are in the caller's original point order.
 *  - One handle must not be used from two threads at once.  All device work of
 *    a handle runs on its stream (options.stream, or the null stream).
 *  - No CPU fallback exists: when no usable gfx950 device is present the
 *    device calls return IFMM_EDEVICE.
 */
#ifndef IFMM_H
#define IFMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ifmm_handle ifmm_handle;

typedef enum {
  IFMM_OK = 0,
  IFMM_EINVAL = -1,     /* invalid argument (message names it)                    */
  IFMM_ENOMEM = -2,     /* host or device allocation failed / over max_device_bytes */
  IFMM_EDEVICE = -3,    /* HIP runtime error or no usable device                  */
  IFMM_ESINGULAR = -4,  /* exactly singular pivot block (message names level, node) */
  IFMM_ENONFINITE = -5, /* non-finite value produced or supplied                  */
  IFMM_ESTATE = -6,     /* call out of order (e.g. solve before factor)           */
  IFMM_ENOCONV = -7     /* GMRES did not reach the tolerance within maxit          */
} ifmm_status;

typedef enum { IFMM_KERNEL_LAPLACE3D = 0 } ifmm_kernel;

typedef enum { IFMM_PREC_FP64 = 0, IFMM_PREC_MIXED = 1 } ifmm_precision;

typedef struct {
  int32_t leaf_max;         /* max points per leaf box; depth = smallest l >= 2 meeting it (64) */
  int32_t cheb_order;       /* Chebyshev nodes per axis of the IFMM operators, 2..6 (4)          */
  int32_t precision;        /* ifmm_precision (FP64)                                             */
  int32_t rank_cap;         /* upper bound on every node rank, 0 = none (0)                      */
  int64_t max_device_bytes; /* refuse to allocate more device memory than this, 0 = no limit (0) */
  void* stream;             /* hipStream_t for all device work of the handle, NULL = null stream */
} ifmm_options;

/* Fills *opt with the defaults listed above. */
void ifmm_default_options(ifmm_options* opt);

/*
 * Builds the octree, the lists and the colouring on the host and uploads the
 * geometry.  Sec. 2.1 (decomposition), Sec. 3 distance equation, Alg. 3.
 *   points   host, N x 3 row-major FP64; finite; not all coincident.
 *   n        N >= 1.
 *   weights  host, N column scalings w_j (e.g. panel areas) or NULL (= 1).
 *   diag     host, N self terms A_ii, or NULL to use diag_scalar for all.
 *   kernel   IFMM_KERNEL_LAPLACE3D.
 *   eps      relative truncation threshold of every compression, 0 < eps < 1.
 *   sigma    colouring separation, >= 3 (sigma <= 2 serialises everything,
 *            Sec. 3.3); 3 and 6 are the paper's two algorithms.
 *   opt      options or NULL for the defaults.
 *   out      receives the new handle (owned by the caller; ifmm_destroy frees it).
 * Errors: IFMM_EINVAL (bad argument), IFMM_ENOMEM, IFMM_EDEVICE.
 */
ifmm_status ifmm_build(const double* points, int64_t n, const double* weights, const double* diag,
                       double diag_scalar, int32_t kernel, double eps, int32_t sigma,
                       const ifmm_options* opt, ifmm_handle** out);

/*
 * Factorises the extended sparse system on the device: Alg. 1 run colour by
 * colour (Sec. 3.2 / 3.3), followed by the dense LU of the level-2 system.
 * May be called again (refactorises from scratch).
 * Errors: IFMM_EDEVICE, IFMM_ENOMEM, IFMM_ESINGULAR, IFMM_ENONFINITE.
 */
ifmm_status ifmm_factor(ifmm_handle* h);

/*
 * Solves A x = b with the factorisation (Alg. 2, colours ascending on the way
 * up and descending on the way down, Sec. 3.2).
 *   rhs, x     N x nrhs column-major, leading dimension ld >= N; host
 *              pointers (on_device = 0) or device pointers (on_device = 1,
 *              read / written on the handle's stream, which is synchronised
 *              before return).  rhs and x may alias.
 *   nrhs       >= 1.
 * Errors: IFMM_ESTATE (no factorisation), IFMM_EINVAL, IFMM_EDEVICE.
 */
ifmm_status ifmm_solve(ifmm_handle* h, const double* rhs, double* x, int32_t nrhs, int64_t ld,
                       int32_t on_device);

/*
 * Writes a JSON object with per-level statistics (nodes, colours, rank
 * histogram summary, bytes) and phase times into json (NUL-terminated,
 * truncated to cap bytes).  Errors: IFMM_EINVAL.
 */
ifmm_status ifmm_stats(const ifmm_handle* h, char* json, int64_t cap);

/* ---- structure queries (host data; for checking the octree and colouring) ---- */

/* Depth l of the octree (levels 2..l exist). */
ifmm_status ifmm_tree_depth(const ifmm_handle* h, int32_t* depth);

/* Tree-order permutation: perm[t] = original index of the t-th point (N entries). */
ifmm_status ifmm_tree_perm(const ifmm_handle* h, int64_t* perm);

/*
 * Node data of one level.  *nnodes receives the count; every other pointer may
 * be NULL.  coords: 3 * nnodes (i, j, k per node); parent: nnodes (-1 at
 * level 2); colour: nnodes; ncolour: number of colours.
 */
ifmm_status ifmm_tree_level(const ifmm_handle* h, int32_t level, int32_t* nnodes, int32_t* coords,
                            int32_t* parent, int32_t* colour, int32_t* ncolour);

/*
 * Neighbour (which = 0) or interaction (which = 1) lists of one level in CSR
 * form: ptr has nnodes + 1 entries, idx has ptr[nnodes] entries (query with
 * idx = NULL first to get the size from ptr).
 */
ifmm_status ifmm_tree_lists(const ifmm_handle* h, int32_t level, int32_t which, int32_t* ptr, int32_t* idx);

/* Final rank of every node of a level (after ifmm_factor). */
ifmm_status ifmm_ranks(const ifmm_handle* h, int32_t level, int32_t* ranks);

/* Message of the last failed call on this thread ("" if none). */
const char* ifmm_last_error(void);

/* Releases the handle and all its device memory.  NULL is ignored. */
void ifmm_destroy(ifmm_handle* h);

#ifdef __cplusplus
}
#endif

#endif /* IFMM_H */
