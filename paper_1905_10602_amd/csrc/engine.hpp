// Internal state of an IFMM handle: host structure, device storage, factor
// records and the orchestration entry points.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "tree.hpp"

namespace ifmm {

// One elimination (node i of the current colour).  The pivot D_i (d x d) is
// stored LU-factorised; L holds the stacked L-blocks (rows of the neighbours
// that couple to x_i: M x n, ld M) and U the stacked U-blocks (n x W, ld n).
// For every neighbour the row count of its block equals its column count, so
// M == W.  All pointers are device pointers.
struct ElimRec {
  int32_t node, n, r, d;   // node index, |x_i|, rank, d = n + r
  int32_t nnb, nb_begin;   // neighbour entries [nb_begin, nb_begin + nnb) of the ElimNbr table
  int32_t M, inv;          // total rows of L-blocks (== total columns of U-blocks); inv: lu holds D^-1
  double* lu;              // d x d, ld d: LU factors with piv, or the explicit inverse (inv = 1)
  int32_t* piv;            // d
  double* L;               // M x n, ld M
  double* U;               // n x M, ld n
  double* X;               // colour scratch: D^-1 [U 0; 0 I], d x (M + r), ld d
  int64_t wv;              // offset (in doubles per right-hand side) of w_i in the solve work vector
  int32_t far_base, pad1;  // far-pair index table: nnb * nnb entries from far_base
  // FP32 copies of L and of G = X[0:n, 0:M] that the solve reads in the mixed
  // form (L and U then live in colour scratch); null in the FP64 form
  float* Ls;               // M x n, ld M
  float* Us;               // n x M, ld n
};

// One 64-row tile of a stored block in the solve.
// Default order from which eigenvalues take the multi-workgroup Householder
// reduction instead of one workgroup per matrix (N = 1M: factorisation 23.8 s
// in FP64 and 21.3 s mixed with 160, against 25.1 and 21.5 s with 384).
constexpr int TRD_BIG_DEFAULT = 160;

struct STask {
  int32_t rec, r0;  // record (index in the level's elimination order), first row of the tile
  int32_t g0, g1;   // backward step: the 64-column chunks [g0, g1) of the inner dimension this task sums
  int32_t slot;     // backward step split over several tasks: partial-sum slot, else -1 (writes x directly)
};
// Backward-step tile whose inner dimension is split over `ns` tasks: its
// partial sums sit in slots slot0 .. slot0 + ns - 1 and are added in order.
struct SGroup {
  int32_t rec, r0, slot0, ns;
};

struct ElimNbr {
  int32_t p;        // neighbour node
  int32_t elim;     // 1 if p was eliminated before i (its row is R_z_p, its column C_y_p)
  int32_t m;        // rows (== columns) of p's current block: r_p if elim else n_p
  int32_t off;      // offset of p's rows in L (and of p's columns in U and X)
  int64_t blk_pi;   // near block (p, i): m x n_i, ld n_p  (level arena offset)
  int64_t blk_ip;   // near block (i, p): n_i x m, ld n_i
};

// Far fill-in between two neighbours a, b of an eliminated node (dist 2).
struct FarPair {
  int32_t rec, a, b, direct;  // direct: both eliminated, add F straight into the M2L block
  double* F;                  // -L_a X_b, m_a x m_b (ld m_a); later the projected block
  double* D;                  // workspace, m_a x m_b
  double* dst;                // M2L block (p_a, p_b)
  int32_t dst_ld, pad;
};

// Far partner of a changed node: the M2L block (p, q) / (q, p) receives a
// projected fill-in from pair ab / ba.
struct FarRef {
  int32_t q, ab, ba, pad;
};

// A non-eliminated neighbour whose bases change in this colour.
struct Changed {
  int32_t p, rec, a, n;     // node, owner record, position in its neighbour list, n_p
  int32_t r, rnew;          // rank before / after
  int32_t far_begin, far_count;
  double *gs, *gt;          // Gram matrices n x n
  double *vs, *vt;          // eigenvectors n x n
  double *ws, *wt;          // Jacobi workspace n x n
  double *ls, *lt;          // eigenvalues n
  double *T, *S;            // T_p (r x rnew, ld r), S_p (rnew x r, ld rnew)
  double* tmp;              // workspace (max(rc, n) x max(rc, n) of the level)
};

struct ColourInv {
  int32_t count = 0, dmax = 0, nmax = 0, Mmax = 0;
};

struct DevLevel {
  int32_t nn = 0, rcmax = 0, nmax = 0;
  // host mirrors
  std::vector<int32_t> n, r, rc;
  std::vector<int32_t> near_ptr, near_idx, slot_row;  // near list of i: i itself, then N_i
  std::vector<int64_t> near_off, p2m_off, l2p_off, sig_off, m2m_off, l2l_off;
  // M2L blocks of the interaction lists: per slot a pointer into the level's
  // block pool, capacity ilcap[t] x ilcap[s], leading dimension ilcap[t]
  std::vector<double*> il_blk;
  std::vector<int32_t> ilcap;
  std::vector<double*> il_chunks;
  double* il_cur = nullptr;
  int64_t il_left = 0, il_bytes = 0;
  double** d_il_blk = nullptr;
  double** d_il_blk_old = nullptr;
  int32_t *d_ilcap = nullptr, *d_ilcap_old = nullptr;
  std::vector<int64_t> cp2m_off, cl2p_off, T_off, S_off;
  int64_t arena_doubles = 0;
  // device working storage of the level (freed once the level is aggregated)
  double* arena = nullptr;
  int32_t *d_rc = nullptr, *d_coord = nullptr, *d_near_ptr = nullptr, *d_near_idx = nullptr;
  int32_t *d_slot_row = nullptr, *d_il_ptr = nullptr, *d_il_idx = nullptr, *d_chg = nullptr;
  int64_t *d_near_off = nullptr, *d_p2m_off = nullptr, *d_l2p_off = nullptr;
  int64_t *d_sig_off = nullptr, *d_m2m_off = nullptr, *d_l2l_off = nullptr;
  int64_t *d_cp2m_off = nullptr, *d_cl2p_off = nullptr, *d_T_off = nullptr, *d_S_off = nullptr;
  // kept for the solve
  int32_t *d_n = nullptr, *d_r = nullptr, *d_parent = nullptr, *d_child_ptr = nullptr, *d_child = nullptr;
  std::vector<ElimRec> recs;   // elimination order
  std::vector<ElimNbr> nbrs;
  std::vector<int32_t> col_ptr;  // recs of colour c: [col_ptr[c], col_ptr[c + 1])
  std::vector<ColourInv> cinv;   // per colour: records solved with an explicit inverse
  // solve: 64-row tiles of the pivot inverses (w), of L (upd) and of G (b),
  // colour c's tiles at [st*_ptr[c], st*_ptr[c + 1]); on the device one table
  // holding w, then upd, then b
  std::vector<STask> st_w, st_u, st_b;
  std::vector<int32_t> stw_ptr, stu_ptr, stb_ptr;
  std::vector<SGroup> sg;          // per colour (sg_ptr) the split backward tiles
  std::vector<int32_t> sg_ptr;
  SGroup* d_sg = nullptr;
  int32_t part_slots = 0;          // most partial-sum slots of one colour
  STask* d_st = nullptr;
  ElimRec* d_recs = nullptr;
  ElimNbr* d_nbrs = nullptr;
  int64_t wv_total = 0;
  std::vector<int64_t> vx_off, vz_off;
  int64_t vx_total = 0, vz_total = 0;
  int64_t *d_vx_off = nullptr, *d_vz_off = nullptr;
};

struct Handle {
  // problem (points, weights and diagonal in tree order)
  int64_t N = 0;
  std::vector<double> pts, w, diag;
  double eps = 0;
  int sigma = 0, leaf_max = 64, nc = 4, K = 64, precision = 0, rank_cap = 0;
  int64_t max_bytes = 0;
  hipStream_t stream = nullptr;
  Tree tree;
  // device
  bool dev_ready = false;
  int device = -1;
  std::vector<std::pair<void*, int64_t>> allocs;
  int64_t dev_bytes = 0;
  double *d_pts = nullptr, *d_w = nullptr, *d_diag = nullptr, *d_lo = nullptr;
  int64_t *d_perm = nullptr, *d_pt_begin = nullptr;
  double* d_unit = nullptr;  // 343 unit-side Chebyshev M2L matrices (offsets in [-3, 3]^3)
  double* d_uus = nullptr;   // U_d^T U_d per offset
  double* d_m2m8 = nullptr;  // the 8 child -> parent M2M matrices
  std::vector<double*> weights_G;  // per level: nn * K * K far-field weights
  std::vector<DevLevel> lv;
  // persistent factor store (bump allocated in chunks)
  std::vector<double*> store_chunks;
  std::vector<int64_t> store_used;  // doubles handed out from each chunk
  double* store_cur = nullptr;
  int64_t store_left = 0, store_bytes = 0;
  // FP32 part of the factor store (the solve's L and G blocks in the mixed form)
  std::vector<float*> store32_chunks;
  std::vector<int64_t> store32_used;  // floats per chunk
  float* store32_cur = nullptr;
  int64_t store32_left = 0;
  bool solve32 = false;  // mixed form, IFMM_SOLVE32=1: the solve reads FP32 L and G blocks
  bool solve_split = true;  // IFMM_SOLVE_SPLIT=0: no split backward tiles (one task per row tile)
  // IFMM_SCHUR_SPLIT=1: the mixed form's near and far Schur products as two
  // kernels on two streams (20.9 s against 21.1 s for the factorisation at
  // N = 1M; off by default, the single kernel's timing stays a clean roofline)
  bool schur_split = false;
  int trd_big = TRD_BIG_DEFAULT;  // order from which eigenvalues take the multi-workgroup reduction (IFMM_TRD_BIG)
  // growable buffers
  double* scratch = nullptr;
  int64_t scratch_bytes = 0;
  char* meta = nullptr;
  int64_t meta_bytes = 0;
  char* meta2 = nullptr;  // slot moves of grown M2L blocks
  int64_t meta2_bytes = 0;
  std::vector<char> host_meta;
  double* svec = nullptr;
  int64_t svec_bytes = 0;
  double* scratch2 = nullptr;  // eigenvector workspace, sized after the rank decision
  int64_t scratch2_bytes = 0;
  bool symmetric = false;      // unit weights: source and target sides coincide
  // top level
  double* d_top = nullptr;      // LU factors of the level-2 system
  double* d_top_inv = nullptr;  // its inverse (the solve applies it as a GEMM)
  int32_t* d_top_piv = nullptr;
  int64_t* d_top_off = nullptr;
  int32_t top_n = 0;
  std::vector<int64_t> top_off;
  bool factored = false;
  // statistics
  double t_init = 0, t_factor = 0, t_solve = 0;
  int64_t stat_far = 0, stat_changed = 0, stat_grown = 0;
  std::vector<double> t_level_setup, t_level_elim;  // per level: set-up + rank reduction, colour loop
  double t_top = 0;
  bool log = false;         // IFMM_LOG set: one progress line per level on stderr
  bool poison = false;      // IFMM_POISON set: fill new device allocations with a huge value (debugging)
  bool check = false;       // IFMM_CHECK set: scan the level arena after every step (debugging)
  // IFMM_PROF set: per kernel class, launches / time (hipEvents on the launch
  // stream) / algorithmic flops and bytes of the instrumented launches
  bool prof = false;
  // sketched recompression (randomised range finder with a rank guess; the
  // full eigen-decomposition remains the fall-back and the judge)
  bool sketch = true;       // IFMM_SKETCH=0 disables
  bool pb_wave = true;      // IFMM_PB_WAVE=0: mixed-form phase B without the wave form
  // IFMM_DEEP_N: pivot order from which the Schur update takes the deep FP32
  // tile; off by default (the lite tile's occupancy wins at every level measured)
  int deep_n = 1 << 30;
  // FP64 Schur products on the FP64 matrix cores (LDS-staged tile; the FMA
  // tile with IFMM_F64_MFMA=0).  The matrix-core peak equals the vector peak
  // on this chip, but the tile reads a quarter of the LDS bytes per
  // multiply-add: k_schur 2.6 s against 3.1 s (FP64 form, N = 1M)
  bool f64_mfma = true;
  int sketch_min = 128;     // Gram order from which a sketch is tried (IFMM_SKETCH_MIN)
  double* skbuf = nullptr;
  int64_t skbuf_bytes = 0;
  double* eigtab = nullptr;  // task tables and counts of a colour's full decompositions
  int64_t eigtab_bytes = 0;
  double* skbuf2 = nullptr;  // second-round (wider) sketches
  double* orthbuf = nullptr;  // block Gram-Schmidt tables and coefficients
  int64_t orthbuf_bytes = 0;
  int64_t skbuf2_bytes = 0;
  char* meta2b = nullptr;
  int64_t meta2b_bytes = 0;
  int64_t stat_sketch = 0, stat_sketch_rejected = 0, stat_sketch_narrow = 0;
  int64_t stat_full = 0;         // full eigen-decompositions of recompressions (incl. fall-backs of rejected sketches)
  int64_t stat_sketch_cols = 0;  // columns of all first-round sketches
  bool record_ranks = false;
  bool prof_level = false;  // IFMM_PROF_LEVEL: profile classes keyed "name@level"
  int cur_level = 0;
  // learned rank model (FP32 parameters on the device) and recorded samples
  float* d_model = nullptr;
  std::vector<float> model_host;  // parameters read from options.rank_model (uploaded by the first factor)
  int top_tau = 2;                // levels below tau: one node per step (matrix-parallel)
  int bottom_level = 0;           // requested depth: 0 from leaf_max, -1 cost model, >= 2 forced
  int colouring = 0;              // 0 Alg. 3, 1 look-back greedy
  std::vector<double> depth_costs;  // cost-model estimates of the candidate depths (bottom_level = -1)
  std::string tune_cache;         // autotuner cache file ("" = built-in tile choices)
  // Autotuner: per key "<kernel> <form> d<depth> l<level>[ k<rhs chunk>]" the
  // chosen variant (Schur tile) or wave count (solve steps).  Read from the
  // cache file at each factorisation; a key missing from it is tuned on the
  // fly (Schur: the level's colours alternate between the two tiles; solve:
  // one timed solve per wave count) and the file is rewritten.
  std::map<std::string, int> tune;
  bool tune_dirty = false;
  struct TuneMeas {
    hipEvent_t a, b;
    std::string key;
    int variant;      // index of the candidate
    int value;        // what the table stores when this candidate wins
    double work;      // flops (Schur) or launches (solve) between the events
  };
  std::vector<TuneMeas> tune_pending;
  int solve_nw_force = 0;  // tuning: every solve launch uses this many waves
  int solve_tune_var = -1; // tuning: candidate index of the timed solve (-1: not tuning)
  double* fbuf = nullptr;
  int64_t fbuf_bytes = 0;
  std::vector<float> rec_X, rec_t;                   // features (14 per row) and r_new / n
  std::vector<std::vector<int64_t>> pt_count;        // points in each node's box, per level
  int64_t stat_predicted = 0;
  double t_sync = 0;
  double t_h2d = 0;
  // host copies of tables whose uploads may still be in flight: released at
  // the next stream synchronisation of the factorisation
  std::vector<std::shared_ptr<void>> hold;   // time the host spent inside table uploads of the factorisation  // time the host waited in stream synchronisations of the elimination
  // solve captured into a HIP graph, replayed while (nrhs, ld, rhs, x) repeat (IFMM_GRAPH=0 disables)
  bool graph_solve = true;
  hipStream_t batch_stream = nullptr;  // library-owned stream given by the batch calls
  hipStream_t cap_stream = nullptr;
  // second stream of the factorisation (default priority): independent work of
  // a colour runs there between a fork and a join event on the main stream
  hipStream_t side_stream = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  hipGraph_t g_graph = nullptr;
  hipGraphExec_t g_exec = nullptr;
  int g_key_k = -1;
  int64_t g_key_ld = 0;
  const double* g_key_rhs = nullptr;
  double* g_key_x = nullptr;
  int big_d = 256;          // pivots of at least this order take the blocked multi-workgroup path (IFMM_BIG_D)
  bool il_tight = false;    // IFMM_IL_TIGHT set: no capacity headroom for M2L blocks (tests the growth path)
  struct KStat {
    int64_t launches = 0;
    double ms = 0, flops = 0, bytes = 0;
  };
  std::map<std::string, KStat> kstat;
  std::map<std::string, double> host_ms;  // host time of the factorisation by phase, stream waits excluded
  std::map<std::string, double> aux;      // further counters (e.g. the far fill-in share of the Schur flops)
  struct Pending {
    hipEvent_t a, b;
    std::string name;
    double flops, bytes;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> event_pool;
  int32_t* d_flag = nullptr;
  bool eig_jacobi = false;  // IFMM_EIG=jacobi: cyclic Jacobi instead of tridiagonal + bisection
  // work buffers of the multi-workgroup tridiagonal reduction, one per stream
  double* trd_buf = nullptr;
  double* trd_buf_side = nullptr;
  int64_t trd_cap = 0, trd_cap_side = 0;
};

// Block-diagonal preconditioner (Sec. 4.3): the inverses of the dense
// diagonal blocks of the boxes of one level.
struct BdHandle {
  Tree tree;
  int64_t N = 0;
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int nbox = 0, nmax = 0;
  int64_t block_doubles = 0;
  double *d_pts = nullptr, *d_w = nullptr, *d_diag = nullptr, *d_mem = nullptr, *d_dinv = nullptr;
  int64_t *d_perm = nullptr, *d_pt_begin = nullptr;
  int32_t *d_piv = nullptr, *d_info = nullptr;
  void* d_tasks = nullptr;  // BluTask table
  double t_build = 0;
};
int bd_setup(BdHandle& h, const double* pts, int64_t n, const double* w, const double* diag, double diag_scalar,
             int level, int leaf_max, std::string& err);
int bd_apply(BdHandle& h, const double* r, double* z, std::string& err);  // device vectors, caller order
void bd_release(BdHandle& h);

// status helpers
void set_error(const std::string& msg);
const char* get_error();

int build_host(Handle& h, const double* pts, int64_t n, const double* w, const double* diag, double diag_scalar,
               std::string& err);
int device_init(Handle& h, std::string& err);
int factor(Handle& h, std::string& err);
int solve(Handle& h, const double* rhs, double* x, int nrhs, int64_t ld, int on_device, std::string& err);
// The same solve with device vectors only, its work vector in a fixed per-device
// array (no allocation, no synchronisation: the work is left queued on h.stream).
int solve_noalloc(Handle& h, const double* rhs, double* x, int nrhs, int64_t ld, std::string& err);
int64_t solve_noalloc_limit_bytes();
void release(Handle& h);

}  // namespace ifmm
