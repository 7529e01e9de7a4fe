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

/*
 * IFMM_PREC_FP64: every step in FP64.
 * IFMM_PREC_MIXED: the Schur-complement products of the elimination and the
 * basis-change products of phase B run on FP32 matrix cores (operands
 * rounded to FP32, FP32 accumulation, results combined in FP64); the pivot
 * LU and its triangular solves, the recompression (Gram matrices and their
 * eigen-decomposition, which must resolve eps^2 relative to the largest
 * eigenvalue), the top-level LU and the solve stay FP64.
 */
typedef enum { IFMM_PREC_FP64 = 0, IFMM_PREC_MIXED = 1 } ifmm_precision;

typedef struct {
  int32_t leaf_max;         /* max points per leaf box; the default depth is the smallest l >= 2 meeting it (64) */
  int32_t cheb_order;       /* Chebyshev nodes per axis of the IFMM operators, 2..6 (4)                       */
  int32_t precision;        /* ifmm_precision (FP64)                                                          */
  int32_t top_tau;          /* tau of Sec. 4.2: levels tau..l are eliminated colour by colour (node-parallel),
                               levels 2..tau-1 one node at a time, every node spread over the whole device
                               (matrix-parallel); 2 = every level colour by colour (2)                       */
  const char* rank_model;   /* path of a raw little-endian FP32 file with the rank network's parameters
                               (ifmm_rank_model_params(IFMM_RANK_FEATURES) values), or NULL = no model (NULL) */
  const char* tune_cache;   /* path of the autotuner's cache file, or NULL = the built-in choices (NULL).
                               Tuned: the Schur-update tile per level (FP64: FMA or matrix cores; mixed: lite
                               or deep FP32 tile) and the waves per workgroup of each solve step per level.
                               Read at every ifmm_factor; a level without an entry alternates the two tiles
                               over its colours and keeps the faster, the first solve without entries times
                               one solve per wave count; the file is then rewritten ("key = value" lines).
                               A failed write returns IFMM_EINVAL after the work is done.               */
  int64_t max_device_bytes; /* refuse to allocate more device memory than this, 0 = no limit (0)              */
  int32_t deterministic;    /* 1: results bitwise reproducible run to run.  The only mode: the library uses
                               no floating-point atomics; 0 is accepted and behaves the same (1)             */
  int32_t bottom_level;     /* l, the depth of the IFMM tree: 0 = from leaf_max, >= 2 = this level (leaves
                               may then hold more than leaf_max points), -1 = chosen by the cost model of
                               Sec. 5.2 from the point counts (0)                                            */
  int32_t rank_cap;         /* upper bound on every node rank, 0 = none (0)                                   */
  int32_t colouring;        /* 0: Alg. 3 (sigma-stride greedy); 1: look-back greedy, which takes every box
                               at distance >= sigma from all boxes of the colour so far (the improvement
                               the closing remark of Sec. 3.4 names) (0)                                   */
  void* stream;             /* hipStream_t for all device work of the handle, NULL = null stream              */
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
 * The solve of ifmm_solve without any allocation, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops.
 *   rhs, x     device pointers, N x nrhs column-major, leading dimension
 *              ld >= N; they may alias.
 * The work vector lives in one fixed device array of the library per device
 * (ifmm_solve_noalloc_max_bytes() bytes, 256 MiB, held until the process
 * ends), shared by every handle and every call on that device: calls that
 * overlap on one device race, so serialise them (one stream, or events).
 * The work is enqueued on the handle's stream and the call returns without
 * synchronising; x is valid once that stream has reached this point.  No
 * HIP graph is used and no timing events are recorded.
 * Errors: IFMM_ESTATE (no factorisation), IFMM_EINVAL (bad argument, or the
 * work vector for nrhs right-hand sides exceeds the fixed array; the message
 * gives the bytes needed), IFMM_EDEVICE.
 */
ifmm_status ifmm_solve_noalloc(ifmm_handle* h, const double* rhs, double* x, int32_t nrhs, int64_t ld);

/* Size in bytes of the fixed work array of ifmm_solve_noalloc. */
int64_t ifmm_solve_noalloc_max_bytes(void);

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

/* ---- many independent geometries -------------------------------------------
 * The factorisations (solves) of `count` handles run concurrently: every
 * handle without a stream of its own gets a library-owned one, and `threads`
 * host threads (0 = up to 8) drive the colour-by-colour schedules, so the
 * small per-colour launches of different geometries overlap on the device.
 * On failure *failed (if not NULL) receives the index of the first failing
 * handle and its status is returned; other handles may have completed.
 */
ifmm_status ifmm_factor_batch(ifmm_handle** hs, int32_t count, int32_t threads, int32_t* failed);
ifmm_status ifmm_solve_batch(ifmm_handle** hs, int32_t count, const double* const* rhs, double* const* x,
                             int32_t nrhs, const int64_t* ld, int32_t on_device, int32_t threads, int32_t* failed);

/* ---- learned recompression rank ---------------------------------------------
 * Sec. 5.1 compresses the fill-in with a randomised SVD, whose width has to
 * be chosen.  Here every recompression whose Gram matrix has order >= 128
 * first tries a sketch (randomised range finder of the stacked factor,
 * Rayleigh-Ritz on the Gram matrix) of width s = predicted rank +
 * oversampling; it is accepted only when the eigen-mass outside the sketch,
 * trace(G) - trace(Q^T G Q), is at most eps^2 lambda_1 and fewer than s Ritz
 * values pass the truncation rule, otherwise the full eigen-decomposition
 * runs (fall-back and judge).  Without a model the predicted rank is the
 * node's current rank; with one it is a small network's estimate.
 *
 * The network: IFMM_RANK_FEATURES inputs (level / 8, log10(box half-side) / 4,
 * log2(1 + points in the box) / 20, |interaction list| / 189, n / 1024,
 * current rank / 512, log10(s_1) / 8 and log10(s_i / s_1) / 16 for i = 2..8,
 * s_i the singular values of an 8-column range sample of the source-side
 * stacked factor), two hidden layers of 64 ReLU units, one output (the rank
 * as a fraction of n), FP32.  Parameters, flat: W1 (64 x F row-major), b1
 * (64), W2 (64 x 64 row-major), b2 (64), w3 (64), b3 (1).  Training minimises
 * the pinball loss at quantile tau (an upper quantile keeps fall-backs rare)
 * with full-batch Adam, on the device.
 */
#define IFMM_RANK_FEATURES 14

/* Number of parameters of the network for nfeat inputs (-1 if nfeat < 1). */
int64_t ifmm_rank_model_params(int32_t nfeat);

/* y[i] = network(theta, X[i, :]) for m samples (X row-major m x nfeat; host arrays). */
ifmm_status ifmm_rank_model_eval(const float* theta, int32_t nfeat, const float* X, int64_t m, float* y);

/* Mean pinball loss (quantile tau) of the targets t and its gradient (host arrays). */
ifmm_status ifmm_rank_model_grad(const float* theta, int32_t nfeat, const float* X, const float* t, int64_t m,
                                 float tau, double* loss, float* grad);

/*
 * steps of full-batch Adam (lr; beta 0.9 / 0.999, 1e-8) from theta, updated in
 * place; loss_hist[k] receives the loss before step k + 1 (NULL allowed).
 */
ifmm_status ifmm_rank_model_train(const float* X, const float* t, int64_t m, int32_t nfeat, int32_t steps,
                                  float lr, float tau, float* theta, double* loss_hist);

/* Loads (theta != NULL) or clears the rank model of a handle; used by later ifmm_factor calls. */
ifmm_status ifmm_set_rank_model(ifmm_handle* h, const float* theta, int32_t nfeat);

/* With on != 0 the next ifmm_factor records (features, new rank / n) of every sketch-eligible recompression. */
ifmm_status ifmm_record_ranks(ifmm_handle* h, int32_t on);

/* Copies up to cap recorded samples (X: cap x IFMM_RANK_FEATURES, t: cap); *count = number recorded. */
ifmm_status ifmm_rank_records(const ifmm_handle* h, float* X, float* t, int64_t cap, int64_t* count);

/* ---- FMM matrix-vector product and the preconditioned FMBEM driver ---------
 * Alg. 4 builds an FMM tree, precomputes the FMM operators and runs GMRES from
 * x = 0; Alg. 5 is its preconditioner (the IFMM solve).  Sec. 4.2 allows the
 * matrix-vector FMM to differ from the one the IFMM uses: here it is the
 * Chebyshev FMM with its own interpolation order (5 by default) on the same
 * uniform octree rule.  The product computed is y = A~ x, A~ the FMM
 * representation of A (A on neighbouring leaves, interpolated elsewhere).
 */
typedef struct fmm_handle fmm_handle;

/*
 * Builds the FMM of A (same arguments and meaning as ifmm_build).
 *   cheb_order  2..6 (interpolation points per axis; K = cheb_order^3)
 *   leaf_max    >= 1, the octree depth is the smallest with <= leaf_max points per leaf
 *   stream      hipStream_t for all device work, or NULL (a library-owned stream that is
 *               ordered with the null stream, so device vectors written there are ready)
 * Errors: IFMM_EINVAL, IFMM_ENONFINITE, IFMM_ENOMEM, IFMM_EDEVICE.
 */
ifmm_status fmm_build(const double* points, int64_t n, const double* weights, const double* diag,
                      double diag_scalar, int32_t cheb_order, int32_t leaf_max, void* stream, fmm_handle** out);

/* y = A~ x for one vector of length N (host or device pointers as on_device says). */
ifmm_status fmm_matvec(fmm_handle* h, const double* x, double* y, int32_t on_device);

/*
 * Right-preconditioned flexible GMRES(restart) for A~ x = b from x = 0 (Alg. 4),
 * classical Gram-Schmidt applied twice, stopping when the relative residual
 * estimate falls to tol or after maxit inner iterations.
 *   precond   a factored IFMM handle over the same N points in the same order
 *             (Alg. 5), or NULL for no preconditioner
 *   restart   1..1000
 *   b, x      length N, host or device pointers (on_device); may not alias
 *   iters     receives the number of inner iterations; relres the final
 *             relative residual estimate
 * Returns IFMM_ENOCONV (x and the counters still written) when tol is not met.
 */
ifmm_status fmm_gmres(fmm_handle* h, const double* b, ifmm_handle* precond, double tol, int32_t restart,
                      int32_t maxit, double* x, int32_t on_device, int32_t* iters, double* relres);

/* JSON: N, depth, K, M2L pairs and flops per product, products so far and their time. */
ifmm_status fmm_stats(const fmm_handle* h, char* json, int64_t cap);

void fmm_destroy(fmm_handle* h);

/* ---- block-diagonal preconditioner (BD, Sec. 4.3) ---------------------------
 * M^-1 = blockdiag(A_bb^-1) over the boxes b of level l_BD of the uniform
 * octree (same root cube as the IFMM): A_bb is the dense block of A over the
 * points of box b (A_ij = K(p_i, p_j) w_j, A_ii = diag_i), inverted on the
 * device by a blocked LU with partial pivoting.  The paper's leaf BD uses the
 * leaf level; a coarser l_BD (BDbot l_BD) widens the blocks.
 */
typedef struct bd_handle bd_handle;

/*
 * Builds BD (same geometry arguments as ifmm_build).
 *   level     l_BD in [2, 10], or 0 = the level where every box holds at most
 *             leaf_max points; boxes may hold at most 4096 points
 *   stream    hipStream_t for all device work, or NULL (a library-owned stream
 *             ordered with the null stream)
 * Errors: IFMM_EINVAL (bad argument, coincident points, a box too large),
 * IFMM_ENONFINITE, IFMM_ESINGULAR (a singular block), IFMM_ENOMEM, IFMM_EDEVICE.
 */
ifmm_status bd_build(const double* points, int64_t n, const double* weights, const double* diag, double diag_scalar,
                     int32_t level, int32_t leaf_max, void* stream, bd_handle** out);

/* z = M^-1 r (length N, host or device pointers; r and z may not alias). */
ifmm_status bd_apply(bd_handle* h, const double* r, double* z, int32_t on_device);

/* fmm_gmres (same arguments and results) with BD as the right preconditioner. */
ifmm_status fmm_gmres_bd(fmm_handle* h, const double* b, bd_handle* bd, double tol, int32_t restart, int32_t maxit,
                         double* x, int32_t on_device, int32_t* iters, double* relres);

/* JSON: N, level, boxes, largest box, bytes of the stored inverses, build time. */
ifmm_status bd_stats(const bd_handle* h, char* json, int64_t cap);

void bd_destroy(bd_handle* h);

/*
 * The FMBEM driver in one call (Alg. 4): piecewise-constant collocation,
 * A_ij = areas_j / (4 pi |c_i - c_j|), A_ii = self_terms_i, solved by
 * fmm_gmres with an FMM of order fmm_cheb_order (leaf_max 64) and the given
 * preconditioner (NULL = none).  Host arrays of length n; sol is written.
 */
ifmm_status fmbem_gmres(const double* centroids, const double* areas, const double* self_terms, int64_t n,
                        const double* f, ifmm_handle* precond, int32_t fmm_cheb_order, double tol, int32_t restart,
                        int32_t maxit, double* sol, int32_t* iters, double* relres);

#ifdef __cplusplus
}
#endif

#endif /* IFMM_H */
