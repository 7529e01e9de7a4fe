// Host scheduler of the IFMM on one gfx950 device.
//
// Factorisation (Alg. 1 with the colour loops of Sec. 3.2 / 3.3):
//   for every level, leaves first:
//     set up the level (leaf operators, or aggregation of the finer level),
//     initial rank reduction (square pivots), then for every colour:
//       phase A  gather -> LU -> X = D^-1 U -> Schur update / far fill-in ->
//                Gram -> Jacobi eigen-decomposition -> (host reads ranks) ->
//                new bases -> projection of the far fill-in
//       phase B  basis change pushed into the M2L blocks of the interaction
//                lists and into M2M / L2L (owner-computes, no atomics)
//   dense LU of the level-2 M2L system.
// Solve (Alg. 2): per level, colours ascending (up) then descending (down).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <numeric>
#include <mutex>
#include <thread>

#include "engine.hpp"
#include "kernels.hpp"
#include "mlp.hpp"

namespace ifmm {

#define HIPCHK(x)                                                                   \
  do {                                                                              \
    hipError_t e_ = (x);                                                            \
    if (e_ != hipSuccess) {                                                         \
      err = std::string(#x) + " failed: " + hipGetErrorString(e_);                  \
      return -3;                                                                    \
    }                                                                               \
  } while (0)

// stream synchronisation of the factorisation, its waiting time accounted
#define HSYNC(hh)                                                     \
  do {                                                                \
    const double t_s0_ = now_s();                                     \
    HIPCHK(hipStreamSynchronize((hh).stream));                        \
    (hh).t_sync += now_s() - t_s0_;                                   \
    (hh).hold.clear();                                                \
  } while (0)

static double now_s();
// host worker threads for table building: IFMM_HOST_THREADS, else the
// hardware's count, at most 16
static int host_threads() {
  static const int n = [] {
    int t = (int)std::thread::hardware_concurrency();
    if (const char* e = std::getenv("IFMM_HOST_THREADS")) t = std::atoi(e);
    return std::max(1, std::min(t > 0 ? t : 1, 16));
  }();
  return n;
}
// fn(chunk, begin, end) over [0, n) split into `chunks` contiguous ranges, in parallel
template <class F>
static void parallel_chunks(int n, int chunks, F&& fn) {
  if (chunks <= 1) {
    fn(0, 0, n);
    return;
  }
  std::vector<std::thread> th;
  th.reserve(chunks - 1);
  for (int c = 1; c < chunks; ++c) {
    const int b = (int)((int64_t)n * c / chunks), e = (int)((int64_t)n * (c + 1) / chunks);
    th.emplace_back([&fn, c, b, e] { fn(c, b, e); });
  }
  fn(0, 0, (int)((int64_t)n / chunks));
  for (auto& t : th) t.join();
}
// upload of a host table; the time the call holds the host is booked apart
#define H2D(hh, dst, src, bytes)                                                          \
  do {                                                                                   \
    const double t_h0_ = now_s();                                                        \
    HIPCHK(hipMemcpyAsync((dst), (src), (bytes), hipMemcpyHostToDevice, (hh).stream));   \
    (hh).t_h2d += now_s() - t_h0_;                                                       \
  } while (0)

static double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}
// Host time of the factorisation split by phase: mark() books the time since
// the previous mark, less the stream waits and table uploads in between.
struct HostLap {
  Handle& h;
  double t, s;
  explicit HostLap(Handle& hh) : h(hh), t(now_s()), s(hh.t_sync + hh.t_h2d) {}
  void mark(const char* name) {
    const double t1 = now_s();
    h.host_ms[name] += 1e3 * ((t1 - t) - (h.t_sync + h.t_h2d - s));
    t = t1;
    s = h.t_sync + h.t_h2d;
  }
};

// ------------------------------------------------------------------ device memory
template <class T>
static int dalloc(Handle& h, T** p, int64_t count, std::string& err) {
  *p = nullptr;
  if (count <= 0) return 0;
  const int64_t bytes = count * (int64_t)sizeof(T);
  if (h.max_bytes > 0 && h.dev_bytes + bytes > h.max_bytes) {
    err = "device memory limit exceeded (" + std::to_string(h.dev_bytes + bytes) + " > " +
          std::to_string(h.max_bytes) + " bytes)";
    return -2;
  }
  hipError_t e = hipMalloc((void**)p, (size_t)bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    err = "hipMalloc of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e);
    return -2;
  }
  h.dev_bytes += bytes;
  h.allocs.push_back({(void*)*p, bytes});
  // debugging: fill with a huge finite value, which exposes reads of unset memory
  if (h.poison) (void)hipMemsetD32Async((hipDeviceptr_t)*p, 0x7FEFFFFF, (size_t)(bytes / 4), h.stream);
  return 0;
}

static void dfree(Handle& h, void* p) {
  if (!p) return;
  for (size_t k = 0; k < h.allocs.size(); ++k)
    if (h.allocs[k].first == p) {
      h.dev_bytes -= h.allocs[k].second;
      h.allocs.erase(h.allocs.begin() + (long)k);
      break;
    }
  (void)hipFree(p);
}

template <class T>
static int upload(Handle& h, T** p, const std::vector<T>& v, std::string& err) {
  int rc = dalloc(h, p, (int64_t)std::max<size_t>(v.size(), 1), err);
  if (rc) return rc;
  if (!v.empty()) {
    H2D(h, *p, v.data(), v.size() * sizeof(T));
    HSYNC(h);  // v may be a temporary
  }
  return 0;
}

// bump allocator for the persistent factor store
static int store_take(Handle& h, int64_t doubles, double** out, std::string& err) {
  doubles = (doubles + 31) & ~31LL;  // 256-byte alignment
  if (doubles > h.store_left) {
    const int64_t chunk = std::max<int64_t>(doubles, (int64_t)1 << 26);  // >= 512 MiB
    double* p = nullptr;
    int rc = dalloc(h, &p, chunk, err);
    if (rc) return rc;
    // zeroed, so that the padding between records is finite for the final scan
    HIPCHK(hipMemsetAsync(p, 0, (size_t)chunk * 8, h.stream));
    h.store_chunks.push_back(p);
    h.store_used.push_back(0);
    h.store_cur = p;
    h.store_left = chunk;
  }
  *out = h.store_cur;
  h.store_cur += doubles;
  h.store_left -= doubles;
  h.store_used.back() += doubles;
  h.store_bytes += doubles * 8;
  return 0;
}

// FP32 blocks of the factor store, same scheme (256-byte aligned, zeroed chunks).
static int store32_take(Handle& h, int64_t floats, float** out, std::string& err) {
  floats = (floats + 63) & ~63LL;
  if (floats > h.store32_left) {
    const int64_t chunk = std::max<int64_t>(floats, (int64_t)1 << 27);  // >= 512 MiB
    double* p = nullptr;
    int rc = dalloc(h, &p, chunk / 2, err);
    if (rc) return rc;
    HIPCHK(hipMemsetAsync(p, 0, (size_t)chunk * 4, h.stream));
    h.store32_chunks.push_back((float*)p);
    h.store32_used.push_back(0);
    h.store32_cur = (float*)p;
    h.store32_left = chunk;
  }
  *out = h.store32_cur;
  h.store32_cur += floats;
  h.store32_left -= floats;
  h.store32_used.back() += floats;
  h.store_bytes += floats * 4;
  return 0;
}

// A copy of a host table that stays alive until the next stream
// synchronisation: the source of an upload that the host does not wait for.
template <class T>
static const T* held(Handle& h, const std::vector<T>& v) {
  auto c = std::make_shared<std::vector<T>>(v);
  const T* p = c->data();
  h.hold.push_back(std::move(c));
  return p;
}

// growable scratch / meta buffers
static int ensure(Handle& h, void** buf, int64_t* cap, int64_t bytes, std::string& err) {
  if (bytes <= *cap) return 0;
  HSYNC(h);
  const int64_t nb = std::max<int64_t>(bytes, (*cap) * 3 / 2);
  dfree(h, *buf);
  *buf = nullptr;
  *cap = 0;
  char* p = nullptr;
  int rc = dalloc(h, &p, nb, err);
  if (rc) return rc;
  *buf = p;
  *cap = nb;
  return 0;
}

// ---- per-kernel-class timing (IFMM_PROF)
static hipEvent_t take_event(Handle& h) {
  if (!h.event_pool.empty()) {
    hipEvent_t e = h.event_pool.back();
    h.event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}
struct ProfScope {
  Handle& h;
  Handle::Pending p;
  bool on;
  hipStream_t st;
  ProfScope(Handle& hh, const char* name, double flops, double bytes, bool side = false)
      : h(hh), on(hh.prof), st(side ? hh.side_stream : hh.stream) {
    if (!on) return;
    p.a = take_event(h);
    p.b = take_event(h);
    p.name = h.prof_level && h.cur_level > 0 ? std::string(name) + "@" + std::to_string(h.cur_level) : name;
    p.flops = flops;
    p.bytes = bytes;
    (void)hipEventRecord(p.a, st);
  }
  ~ProfScope() {
    if (!on) return;
    (void)hipEventRecord(p.b, st);
    h.pending.push_back(p);
  }
};

// ---- autotuner (options.tune_cache)
static std::string form_name(const Handle& h) { return h.precision == 1 ? "mixed" : "fp64"; }
static std::string schur_key(const Handle& h, int l) {
  return "schur " + form_name(h) + " d" + std::to_string(h.tree.depth) + " l" + std::to_string(l);
}
static std::string solve_key(const Handle& h, const char* step, int l, int sk) {
  return std::string(step) + " " + form_name(h) + " d" + std::to_string(h.tree.depth) + " l" + std::to_string(l) +
         " k" + std::to_string(sk);
}
// The cache file: one "key = value" per line, '#' comments; a missing file
// is an empty table.
static void tune_load(Handle& h) {
  h.tune.clear();
  h.tune_dirty = false;
  if (h.tune_cache.empty()) return;
  std::ifstream f(h.tune_cache);
  std::string line;
  while (std::getline(f, line)) {
    if (line.empty() || line[0] == '#') continue;
    const size_t p = line.rfind(" = ");
    if (p == std::string::npos) continue;
    h.tune[line.substr(0, p)] = std::atoi(line.c_str() + p + 3);
  }
}
static int tune_save(Handle& h, std::string& err) {
  if (h.tune_cache.empty() || !h.tune_dirty) return 0;
  std::ofstream f(h.tune_cache, std::ios::trunc);
  if (!f) {
    err = "cannot write the autotuner cache " + h.tune_cache;
    return -1;
  }
  f << "# ifmm autotuner: <kernel> <form> d<depth> l<level>[ k<rhs chunk>] = <choice>\n";
  for (const auto& kv : h.tune) f << kv.first << " = " << kv.second << "\n";
  h.tune_dirty = false;
  return f ? 0 : (err = "cannot write the autotuner cache " + h.tune_cache, -1);
}
// After a stream synchronisation: per key, the candidate with the most work
// per millisecond over its timed launches wins (a candidate never timed loses).
static hipEvent_t take_event(Handle& h);
static void tune_collect(Handle& h) {
  if (h.tune_pending.empty()) return;
  struct Acc { double work[3] = {0, 0, 0}, ms[3] = {0, 0, 0}; int value[3] = {0, 0, 0}; };
  std::map<std::string, Acc> acc;
  for (const auto& m : h.tune_pending) {
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, m.a, m.b);
    Acc& a = acc[m.key];
    a.work[m.variant] += m.work;
    a.ms[m.variant] += ms;
    a.value[m.variant] = m.value;
    h.event_pool.push_back(m.a);
    h.event_pool.push_back(m.b);
  }
  h.tune_pending.clear();
  for (const auto& kv : acc) {
    const Acc& a = kv.second;
    int best = -1;
    double rate = -1.0;
    for (int v = 0; v < 3; ++v)
      if (a.ms[v] > 0.0 && a.work[v] / a.ms[v] > rate) {
        rate = a.work[v] / a.ms[v];
        best = v;
      }
    if (best >= 0) {
      h.tune[kv.first] = a.value[best];
      h.tune_dirty = true;
    }
  }
}

// Fork: work launched on h.side_stream after this waits for everything
// queued on the main stream so far.  Join: the main stream waits for the
// side stream's work so far.  Both streams have the default priority.
static int fork_side(Handle& h, std::string& err) {
  if (!h.side_stream) {
    HIPCHK(hipStreamCreateWithFlags(&h.side_stream, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&h.ev_fork, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&h.ev_join, hipEventDisableTiming));
  }
  HIPCHK(hipEventRecord(h.ev_fork, h.stream));
  HIPCHK(hipStreamWaitEvent(h.side_stream, h.ev_fork, 0));
  return 0;
}
static int join_side(Handle& h, std::string& err) {
  HIPCHK(hipEventRecord(h.ev_join, h.side_stream));
  HIPCHK(hipStreamWaitEvent(h.stream, h.ev_join, 0));
  return 0;
}
// called after a stream synchronisation
static void prof_collect(Handle& h) {
  for (auto& p : h.pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      auto& k = h.kstat[p.name];
      k.launches += 1;
      k.ms += ms;
      k.flops += p.flops;
      k.bytes += p.bytes;
    }
    h.event_pool.push_back(p.a);
    h.event_pool.push_back(p.b);
  }
  h.pending.clear();
}

// IFMM_CHECK: after a step, scan the level arena for non-finite / huge values.
static int check_arena(Handle& h, int l, const char* step, int c, std::string& err) {
  if (!h.check) return 0;
  DevLevel& L = h.lv[l];
  if (!L.arena || L.arena_doubles == 0) return 0;
  if (!h.d_flag) {
    HIPCHK(hipMalloc((void**)&h.d_flag, 4));
  }
  HIPCHK(hipMemsetAsync(h.d_flag, 0, 4, h.stream));
  hipLaunchKernelGGL(k_check_finite, dim3(1024), dim3(NT), 0, h.stream, L.arena, L.arena_doubles, h.d_flag);
  int32_t f = 0;
  HIPCHK(hipMemcpyAsync(&f, h.d_flag, 4, hipMemcpyDeviceToHost, h.stream));
  HIPCHK(hipStreamSynchronize(h.stream));
  if (f) {
    err = std::string("check: non-finite or huge value in the level arena after ") + step + " at level " +
          std::to_string(l) + " colour " + std::to_string(c);
    return -5;
  }
  return 0;
}

// ------------------------------------------------------------------ eigenvalues
// Eigenvalues of the matrices of T (device table d_T, counts above eps2 *
// lam_1 into d_cnt) on stream st: orders below h.trd_big take the one-workgroup
// solver, larger ones the multi-workgroup reduction (their work vectors in a
// buffer of this stream; the stream is synchronised before it grows).
static int eig_values(Handle& h, const std::vector<EigTask>& T, const EigTask* d_T, double eps2, int32_t* d_cnt,
                      hipStream_t st, std::string& err) {
  if (T.empty()) return 0;
  std::vector<int32_t> big;
  int nmax = 0;
  int64_t need = 0;
  for (size_t a = 0; a < T.size(); ++a)
    if (!h.eig_jacobi && T[a].n >= h.trd_big && T[a].n <= TRD_MAXN) {
      big.push_back((int32_t)a);
      nmax = std::max(nmax, T[a].n);
      need += 3LL * T[a].n + (int64_t)T[a].n * ((T[a].n + 63) / 64) + 32;
    }
  if (h.eig_jacobi)
    hipLaunchKernelGGL(k_eig_jacobi, dim3((unsigned)T.size()), dim3(NT), 0, st, d_T, eps2, d_cnt);
  else
    hipLaunchKernelGGL(k_eig_values, dim3((unsigned)T.size()), dim3(NT), 0, st, d_T, eps2, d_cnt, h.trd_big);
  if (big.empty()) return 0;
  const bool side = st == h.side_stream && st != nullptr;
  double*& buf = side ? h.trd_buf_side : h.trd_buf;
  int64_t& cap = side ? h.trd_cap_side : h.trd_cap;
  const int64_t tb = ((int64_t)(big.size() * sizeof(TrdTask)) + 255) & ~255LL;
  const int64_t bytes = tb + need * 8 + 256;
  if (bytes > cap) {
    HIPCHK(hipStreamSynchronize(st));
    dfree(h, buf);
    buf = nullptr;
    cap = 0;
    int rc;
    if ((rc = dalloc(h, &buf, (bytes + 7) / 8, err))) return rc;
    cap = ((bytes + 7) / 8) * 8;
  }
  TrdTask* d_trd = (TrdTask*)buf;
  double* w0 = (double*)((char*)buf + tb);
  std::vector<TrdTask> tt(big.size());
  int64_t o = 0;
  for (size_t q = 0; q < big.size(); ++q) {
    const EigTask& e = T[big[q]];
    TrdTask& t = tt[q];
    t.A = e.A;
    t.W = e.W;
    t.vec = w0 + o;
    o += 3LL * e.n;
    t.part = w0 + o;
    o += (int64_t)e.n * ((e.n + 63) / 64) + 32;
    t.n = e.n;
    t.slot = big[q];
  }
  HIPCHK(hipMemcpyAsync(d_trd, held(h, tt), tt.size() * sizeof(TrdTask), hipMemcpyHostToDevice, st));
  const unsigned nb = (unsigned)big.size();
  double fl = 0;
  for (int32_t a : big) fl += 4.0 / 3.0 * (double)T[a].n * T[a].n * T[a].n;
  ProfScope ps(h, "group:trd_multi", fl, 0, side);
  hipLaunchKernelGGL(k_trd_start, dim3(nb), dim3(NT), 0, st, d_trd);
  auto tiles = [&](int k) {
    const int m = nmax - k - 2, b = (m + 63) / 64;
    if (m > 0) hipLaunchKernelGGL(k_trd_tiles, dim3((unsigned)(b * (b + 1) / 2), nb), dim3(NT), 0, st, d_trd, k);
  };
  tiles(-1);
  for (int k = 0; k + 2 < nmax; ++k) {
    hipLaunchKernelGGL(k_trd_step, dim3(nb), dim3(NT), 0, st, d_trd, k);
    tiles(k);
  }
  hipLaunchKernelGGL(k_trd_bisect, dim3((unsigned)((nmax + NT - 1) / NT), nb), dim3(NT), 0, st, d_trd, d_T);
  hipLaunchKernelGGL(k_trd_count, dim3(nb), dim3(NT), 0, st, d_trd, d_T, eps2, d_cnt);
  HIPCHK(hipGetLastError());
  return 0;
}

// Batched GEMM over `count` tasks (host copy `host`, device table d_tasks):
// the FP64 matrix-core tile when every task leaves B untransposed, else (or
// with the matrix cores switched off) the FMA tile.
static void gemm_batch(Handle& h, dim3 grid, const GemmTask* host, size_t count, const GemmTask* d_tasks,
                       hipStream_t st) {
  bool mf = h.f64_mfma;
  for (size_t a = 0; mf && a < count; ++a) mf = host[a].tB == 0;
  if (mf) hipLaunchKernelGGL(k_gemm_batch<true>, grid, dim3(NT), 0, st, d_tasks);
  else hipLaunchKernelGGL(k_gemm_batch<false>, grid, dim3(NT), 0, st, d_tasks);
}

// Eigenvectors of the tasks T (device table d_T, the k of each already set)
// on stream st: one workgroup per task, except the back-transform of orders
// from h.trd_big on, which runs over blocks of 64 columns (k_ev_mask,
// k_ev_apply).
static void eig_vectors(Handle& h, const std::vector<EigTask>& T, const EigTask* d_T, hipStream_t st) {
  if (T.empty()) return;
  const int big = h.trd_big;
  int nmax = 0, kmax = 0;
  for (const EigTask& e : T)
    if (big > 0 && e.n >= big && e.n >= 34 && e.k > 0) {
      nmax = std::max(nmax, e.n);
      kmax = std::max(kmax, e.k);
    }
  const unsigned nt = (unsigned)T.size();
  hipLaunchKernelGGL(k_eig_vectors, dim3(nt), dim3(NT), 0, st, d_T, big);
  if (nmax) {
    hipLaunchKernelGGL(k_ev_mask, dim3((unsigned)((nmax + 63) / 64), nt), dim3(NT), 0, st, d_T, big);
    hipLaunchKernelGGL(k_ev_apply, dim3((unsigned)((kmax + 63) / 64), nt), dim3(NT), 0, st, d_T, big);
  }
}

// ------------------------------------------------------------------ level set-up
static LevelView view_of(DevLevel& L) {
  LevelView V;
  V.arena = L.arena;
  V.n = L.d_n; V.r = L.d_r; V.rc = L.d_rc; V.coord = L.d_coord;
  V.near_ptr = L.d_near_ptr; V.near_idx = L.d_near_idx; V.il_ptr = L.d_il_ptr; V.il_idx = L.d_il_idx;
  V.near_off = L.d_near_off; V.p2m_off = L.d_p2m_off; V.l2p_off = L.d_l2p_off;
  V.il_blk = L.d_il_blk; V.ilcap = L.d_ilcap;
  V.sig_off = L.d_sig_off; V.m2m_off = L.d_m2m_off; V.l2l_off = L.d_l2l_off;
  V.cp2m_off = L.d_cp2m_off; V.cl2p_off = L.d_cl2p_off; V.T_off = L.d_T_off; V.S_off = L.d_S_off;
  V.chg = L.d_chg;
  return V;
}

// Allocates the working storage of level l for the node sizes L.n (exact).
static int setup_level(Handle& h, int l, std::string& err) {
  const Level& T = h.tree.levels[l];
  DevLevel& L = h.lv[l];
  const int K = h.K;
  const int32_t nn = T.n;
  L.nn = nn;
  L.r.assign(nn, 0);
  L.rc.resize(nn);
  int32_t rcmax = 0, nmax = 0;
  for (int32_t i = 0; i < nn; ++i) {
    L.rc[i] = h.rank_cap > 0 ? std::min(L.n[i], h.rank_cap) : L.n[i];
    rcmax = std::max(rcmax, L.rc[i]);
    nmax = std::max(nmax, L.n[i]);
  }
  L.rcmax = rcmax;
  L.nmax = nmax;
  if (nmax > TRD_MAXN) {
    err = "level " + std::to_string(l) + " has a node with " + std::to_string(nmax) +
          " unknowns, above the supported 2048 (lower eps or set rank_cap)";
    return -1;
  }
  L.near_ptr.assign(1, 0);
  L.near_idx.clear();
  L.slot_row.clear();
  for (int32_t i = 0; i < nn; ++i) {
    L.near_idx.push_back(i);
    L.slot_row.push_back(i);
    for (int s = T.nbr_ptr[i]; s < T.nbr_ptr[i + 1]; ++s) {
      L.near_idx.push_back(T.nbr[s]);
      L.slot_row.push_back(i);
    }
    L.near_ptr.push_back((int32_t)L.near_idx.size());
  }
  int64_t off = 0;
  auto take = [&](int64_t cnt) {
    const int64_t o = off;
    off += (cnt + 3) & ~3LL;
    return o;
  };
  L.near_off.resize(L.near_idx.size());
  for (int32_t i = 0; i < nn; ++i)
    for (int s = L.near_ptr[i]; s < L.near_ptr[i + 1]; ++s) L.near_off[s] = take((int64_t)L.n[i] * L.n[L.near_idx[s]]);
  // M2L blocks are allocated once the ranks are known (reduce_level)
  L.il_blk.assign(T.il.size(), nullptr);
  L.ilcap.assign(nn, 0);
  L.p2m_off.resize(nn); L.l2p_off.resize(nn); L.sig_off.resize(nn); L.m2m_off.resize(nn); L.l2l_off.resize(nn);
  L.cp2m_off.resize(nn); L.cl2p_off.resize(nn); L.T_off.resize(nn); L.S_off.resize(nn);
  for (int32_t i = 0; i < nn; ++i) {
    const int64_t n = L.n[i], rc = L.rc[i];
    L.p2m_off[i] = take(rc * n);
    L.l2p_off[i] = take(n * rc);
    L.sig_off[i] = take(2 * rc);
    L.m2m_off[i] = take(K * rc);
    L.l2l_off[i] = take(rc * K);
    L.cp2m_off[i] = take(K * n);
    L.cl2p_off[i] = take(n * K);
    L.T_off[i] = take(K * rc);
    L.S_off[i] = take(rc * K);
  }
  L.arena_doubles = off;
  int rc;
  if ((rc = dalloc(h, &L.arena, std::max<int64_t>(off, 1), err))) return rc;
  HIPCHK(hipMemsetAsync(L.arena, 0, (size_t)std::max<int64_t>(off, 1) * 8, h.stream));
  if ((rc = upload(h, &L.d_n, L.n, err))) return rc;
  if ((rc = upload(h, &L.d_r, L.r, err))) return rc;
  if ((rc = upload(h, &L.d_rc, L.rc, err))) return rc;
  if ((rc = upload(h, &L.d_coord, T.coord, err))) return rc;
  if ((rc = upload(h, &L.d_near_ptr, L.near_ptr, err))) return rc;
  if ((rc = upload(h, &L.d_near_idx, L.near_idx, err))) return rc;
  if ((rc = upload(h, &L.d_slot_row, L.slot_row, err))) return rc;
  if ((rc = upload(h, &L.d_il_ptr, T.il_ptr, err))) return rc;
  if ((rc = upload(h, &L.d_il_idx, T.il, err))) return rc;
  if ((rc = upload(h, &L.d_near_off, L.near_off, err))) return rc;
  if ((rc = upload(h, &L.d_p2m_off, L.p2m_off, err))) return rc;
  if ((rc = upload(h, &L.d_l2p_off, L.l2p_off, err))) return rc;
  if ((rc = upload(h, &L.d_sig_off, L.sig_off, err))) return rc;
  if ((rc = upload(h, &L.d_m2m_off, L.m2m_off, err))) return rc;
  if ((rc = upload(h, &L.d_l2l_off, L.l2l_off, err))) return rc;
  if ((rc = upload(h, &L.d_cp2m_off, L.cp2m_off, err))) return rc;
  if ((rc = upload(h, &L.d_cl2p_off, L.cl2p_off, err))) return rc;
  if ((rc = upload(h, &L.d_T_off, L.T_off, err))) return rc;
  if ((rc = upload(h, &L.d_S_off, L.S_off, err))) return rc;
  std::vector<int32_t> minus(nn, -1);
  if ((rc = upload(h, &L.d_chg, minus, err))) return rc;
  if (l > 2) {
    if ((rc = upload(h, &L.d_parent, T.parent, err))) return rc;
  }
  if (l < h.tree.depth) {
    if ((rc = upload(h, &L.d_child_ptr, T.child_ptr, err))) return rc;
    if ((rc = upload(h, &L.d_child, T.child, err))) return rc;
  }
  return 0;
}

// Frees the working storage of a level (the factor records stay).
static void release_level_work(Handle& h, int l) {
  DevLevel& L = h.lv[l];
  void* ptrs[] = {L.arena, L.d_near_ptr, L.d_near_idx, L.d_slot_row, L.d_il_ptr, L.d_il_idx, L.d_near_off,
                  L.d_p2m_off, L.d_l2p_off, L.d_sig_off, L.d_m2m_off, L.d_l2l_off, L.d_cp2m_off,
                  L.d_cl2p_off, L.d_T_off, L.d_S_off, L.d_chg, L.d_rc, L.d_coord,
                  (void*)L.d_il_blk, (void*)L.d_il_blk_old, L.d_ilcap, L.d_ilcap_old};
  for (void* p : ptrs) dfree(h, p);
  for (double* c : L.il_chunks) dfree(h, c);
  L.il_chunks.clear();
  L.il_cur = nullptr;
  L.il_left = 0;
  L.d_il_blk = L.d_il_blk_old = nullptr;
  L.d_ilcap = L.d_ilcap_old = nullptr;
  L.arena = nullptr;
  L.d_near_ptr = L.d_near_idx = L.d_slot_row = L.d_il_ptr = L.d_il_idx = nullptr;
  L.d_near_off = L.d_p2m_off = L.d_l2p_off = L.d_sig_off = L.d_m2m_off = L.d_l2l_off = nullptr;
  L.d_cp2m_off = L.d_cl2p_off = L.d_T_off = L.d_S_off = nullptr;
  L.d_chg = nullptr;
  L.d_rc = nullptr;
  L.d_coord = nullptr;
}

// Bump allocator of the level's M2L block pool (chunks of >= 256 MiB).
static int il_take(Handle& h, DevLevel& L, int64_t doubles, double** out, std::string& err) {
  doubles = (std::max<int64_t>(doubles, 1) + 7) & ~7LL;
  if (doubles > L.il_left) {
    const int64_t chunk = std::max<int64_t>(doubles, (int64_t)1 << 25);
    double* p = nullptr;
    int rc = dalloc(h, &p, chunk, err);
    if (rc) return rc;
    L.il_chunks.push_back(p);
    L.il_cur = p;
    L.il_left = chunk;
  }
  *out = L.il_cur;
  L.il_cur += doubles;
  L.il_left -= doubles;
  L.il_bytes += doubles * 8;
  return 0;
}

// Capacity of a node's M2L rows / columns for rank r: headroom for the growth
// that later recompressions bring, never above rc.
static int32_t il_capacity(const Handle& h, int32_t r, int32_t rc) {
  return h.il_tight ? std::min(rc, r) : std::min(rc, r + std::max(8, r / 2));
}

// Initial rank reduction of every node of level l (square pivots, far-field
// weighted), then the reduced M2L / M2M / L2L of the level.
static int reduce_level(Handle& h, int l, std::string& err) {
  DevLevel& L = h.lv[l];
  const int K = h.K;
  const int32_t nn = L.nn;
  const bool sym = h.symmetric;
  std::vector<int64_t> woff(nn);
  int64_t wtot = 0;
  for (int32_t i = 0; i < nn; ++i) {
    const int64_t n = L.n[i];
    woff[i] = wtot;
    wtot += 4 * n * n + (int64_t)K * n + 8 * n + (h.eig_jacobi ? 2 * n * n : 0);
    wtot = (wtot + 31) & ~31LL;
  }
  int rc;
  if ((rc = ensure(h, (void**)&h.scratch, &h.scratch_bytes, wtot * 8 + 64, err))) return rc;
  double* work = h.scratch;
  const int sides = sym ? 1 : 2;
  std::vector<EigTask> tasks((size_t)sides * nn);
  for (int32_t i = 0; i < nn; ++i) {
    const int64_t n = L.n[i];
    double* b = work + woff[i];
    double* gs = b;
    double* gt = b + n * n;
    double* vs = b + 2 * n * n + (int64_t)K * n;
    double* vt = vs + n * n;
    double* ls = vt + n * n;
    double* lt = ls + n;
    double* ws = lt + n;
    double* wt = ws + (h.eig_jacobi ? n * n : 3 * n);
    tasks[(size_t)sides * i] = {gs, vs, ws, ls, nullptr, (int32_t)n, 0};
    if (!sym) tasks[(size_t)sides * i + 1] = {gt, vt, wt, lt, nullptr, (int32_t)n, 0};
  }
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t o_t = 0, o_w = al(tasks.size() * sizeof(EigTask)), o_c = o_w + al(nn * sizeof(int64_t));
  const size_t mtot = o_c + al(tasks.size() * 4 + 4);
  if ((rc = ensure(h, (void**)&h.meta, &h.meta_bytes, (int64_t)mtot, err))) return rc;
  EigTask* d_tasks = (EigTask*)(h.meta + o_t);
  int64_t* d_woff = (int64_t*)(h.meta + o_w);
  int32_t* d_cnt = (int32_t*)(h.meta + o_c);
  H2D(h, d_tasks, tasks.data(), tasks.size() * sizeof(EigTask));
  H2D(h, d_woff, woff.data(), nn * sizeof(int64_t));
  LevelView V = view_of(L);
  const double* G = h.weights_G[l];
  if (nn > 0) {
    hipLaunchKernelGGL(k_reduce_gram, dim3(nn), dim3(NT), 0, h.stream, V, K, G, work, d_woff);
    int rc2;
    if ((rc2 = eig_values(h, tasks, d_tasks, h.eps * h.eps, d_cnt, h.stream, err))) return rc2;
  }
  HIPCHK(hipGetLastError());
  std::vector<int32_t> cnt(tasks.size());
  HSYNC(h);  // the copy below waits for the queue: accounted here
  if (nn > 0) HIPCHK(hipMemcpyAsync(cnt.data(), d_cnt, cnt.size() * 4, hipMemcpyDeviceToHost, h.stream));
  HSYNC(h);
  int64_t iw = 0;
  for (int32_t i = 0; i < nn; ++i) {
    int r = sym ? cnt[i] : std::max(cnt[2 * i], cnt[2 * i + 1]);
    r = std::min(r, L.rc[i]);
    L.r[i] = r;
    for (int s2 = 0; s2 < sides; ++s2) iw += 5LL * L.n[i] * r + 32;
  }
  if ((rc = ensure(h, (void**)&h.scratch2, &h.scratch2_bytes, iw * 8 + 64, err))) return rc;
  iw = 0;
  for (int32_t i = 0; i < nn; ++i)
    for (int s2 = 0; s2 < sides; ++s2) {
      EigTask& t = tasks[(size_t)sides * i + s2];
      t.k = L.r[i];
      t.IW = h.scratch2 + iw;
      iw += 5LL * L.n[i] * L.r[i] + 32;
    }
  H2D(h, d_tasks, tasks.data(), tasks.size() * sizeof(EigTask));
  H2D(h, L.d_r, L.r.data(), nn * 4);
  // M2L block pool sized from the ranks just found
  {
    const Level& T = h.tree.levels[l];
    for (int32_t i = 0; i < nn; ++i) L.ilcap[i] = il_capacity(h, L.r[i], L.rc[i]);
    for (int32_t i = 0; i < nn; ++i)
      for (int s2 = T.il_ptr[i]; s2 < T.il_ptr[i + 1]; ++s2)
        if ((rc = il_take(h, L, (int64_t)L.ilcap[i] * L.ilcap[T.il[s2]], &L.il_blk[s2], err))) return rc;
    if ((rc = upload(h, &L.d_il_blk, L.il_blk, err))) return rc;
    if ((rc = upload(h, &L.d_il_blk_old, L.il_blk, err))) return rc;
    if ((rc = upload(h, &L.d_ilcap, L.ilcap, err))) return rc;
    if ((rc = upload(h, &L.d_ilcap_old, L.ilcap, err))) return rc;
  }
  V = view_of(L);
  const double side = 2.0 * h.tree.H / (double)(1LL << l);
  if (nn > 0) {
    if (!h.eig_jacobi) eig_vectors(h, tasks, d_tasks, h.stream);
    hipLaunchKernelGGL(k_reduce_basis, dim3(nn), dim3(NT), 0, h.stream, V, K, work, d_woff, h.d_m2m8, l > 2 ? 1 : 0,
                       sym ? 1 : 0);
    HIPCHK(hipGetLastError());
  }
  // M2L of the interaction pairs (needs T of every node: separate launch)
  HSYNC(h);
  if (nn > 0 && K <= 64) {
    const Level& TL = h.tree.levels[l];
    int ilmax = 1;
    for (int32_t i = 0; i < nn; ++i) ilmax = std::max(ilmax, TL.il_ptr[i + 1] - TL.il_ptr[i]);
    hipLaunchKernelGGL(k_reduce_m2l_lds, dim3(nn, (unsigned)((ilmax + RM2L_SLOTS - 1) / RM2L_SLOTS)), dim3(NT), 0,
                       h.stream, V, K, h.d_unit, 1.0 / side);
    HIPCHK(hipGetLastError());
  } else if (nn > 0) {
    std::vector<int64_t> toff2(nn);
    for (int32_t i = 0; i < nn; ++i) toff2[i] = (int64_t)i * K * std::max(L.rcmax, 1);
    if ((rc = ensure(h, (void**)&h.meta, &h.meta_bytes, (int64_t)nn * 8 + 256, err))) return rc;
    int64_t* d_toff = (int64_t*)h.meta;
    H2D(h, d_toff, toff2.data(), nn * sizeof(int64_t));
    if ((rc = ensure(h, (void**)&h.scratch, &h.scratch_bytes, (int64_t)nn * K * std::max(L.rcmax, 1) * 8 + 64, err)))
      return rc;
    hipLaunchKernelGGL(k_reduce_m2l, dim3(nn), dim3(NT), 0, h.stream, V, K, h.d_unit, 1.0 / side, h.scratch, d_toff);
    HIPCHK(hipGetLastError());
  }
  HSYNC(h);
  return 0;
}

// ------------------------------------------------------------------ one colour
// Rank guess that sizes a sketch when no learned model is loaded: the node's
// current rank.
static int predict_rank(const Handle& h, int l, const Changed& C, int side) {
  (void)h;
  (void)l;
  (void)side;
  return std::max(1, C.r);
}

constexpr int RANK_NF = 14;

// Features of the rank predictor for changed nodes `ids` (level, box size,
// points in the box, interaction-list size, n, current rank and the top-8
// singular values of an 8-column range sample of the source-side stacked
// factor), and, when a model is loaded, its predictions (fraction of n).
static int rank_features(Handle& h, int l, std::vector<Changed>& chg, const std::vector<int32_t>& ids,
                         const std::vector<int64_t>& wrows, const Changed* d_chg, const FarRef* d_refs,
                         const FarPair* d_far, const ElimNbr* d_nbrs, const ElimRec* d_recs, std::vector<float>& feats,
                         std::vector<float>& pred, std::string& err) {
  const size_t nf = ids.size();
  feats.assign(nf * RANK_NF, 0.f);
  pred.assign(nf, -1.f);
  if (!nf) return 0;
  const Level& T = h.tree.levels[l];
  int64_t need = 0;
  int nmax = 1;
  for (int32_t k : ids) {
    need += (std::max<int64_t>(wrows[k], chg[k].n) + chg[k].n) * 8 + 64;
    nmax = std::max(nmax, chg[k].n);
  }
  const size_t tb = (nf * sizeof(SkTask) + nf * 8 * 8 + nf * RANK_NF * 4 + nf * 4 + 1024 + 255) & ~(size_t)255;
  const int64_t mlpw = mlp_work_floats((int64_t)nf);
  int rc;
  if ((rc = ensure(h, (void**)&h.fbuf, &h.fbuf_bytes, (int64_t)tb + need * 8 + mlpw * 4 + 512, err))) return rc;
  char* base = (char*)h.fbuf;
  SkTask* d_t = (SkTask*)base;
  double* d_sv = (double*)(d_t + nf);
  float* d_X = (float*)(d_sv + 8 * nf);
  float* d_y = d_X + nf * RANK_NF;
  double* W0 = (double*)(base + tb);
  float* d_mw = (float*)(W0 + need);
  std::vector<SkTask> tt(nf);
  int64_t o = 0;
  for (size_t a = 0; a < nf; ++a) {
    const Changed& C = chg[ids[a]];
    SkTask& t = tt[a];
    std::memset(&t, 0, sizeof t);
    t.O = W0 + o; o += std::max<int64_t>(wrows[ids[a]], C.n) * 8;
    t.Y = W0 + o; o += (int64_t)C.n * 8 + 64;
    t.n = C.n; t.s = 8; t.R = (int32_t)wrows[ids[a]]; t.chg = ids[a];
    t.seed = (uint32_t)(0x51ED + 2 * C.p); t.side = 0;
  }
  H2D(h, d_t, tt.data(), nf * sizeof(SkTask));
  hipLaunchKernelGGL(k_sk_omega, dim3(16, (unsigned)nf), dim3(NT), 0, h.stream, d_t);
  hipLaunchKernelGGL(k_sk_range<false>, dim3((unsigned)((nmax + 63) / 64), 1, (unsigned)nf), dim3(NT), 0, h.stream, d_chg,
                     d_refs, d_far, d_nbrs, d_recs, d_t);
  hipLaunchKernelGGL(k_feat_sv, dim3((unsigned)nf), dim3(NT), 0, h.stream, d_t, d_sv);
  std::vector<double> sv(8 * nf);
  HSYNC(h);  // the copy below waits for the queue: accounted here
  HIPCHK(hipMemcpyAsync(sv.data(), d_sv, sv.size() * 8, hipMemcpyDeviceToHost, h.stream));
  HSYNC(h);
  const double half = h.tree.H / (double)(1 << l);
  for (size_t a = 0; a < nf; ++a) {
    const Changed& C = chg[ids[a]];
    float* f = &feats[a * RANK_NF];
    const double s1 = std::max(sv[8 * a], 1e-300);
    f[0] = (float)(l / 8.0);
    f[1] = (float)(std::log10(half) / 4.0);
    f[2] = (float)(std::log2(1.0 + (double)h.pt_count[l][C.p]) / 20.0);
    f[3] = (float)((T.il_ptr[C.p + 1] - T.il_ptr[C.p]) / 189.0);
    f[4] = (float)(C.n / 1024.0);
    f[5] = (float)(C.r / 512.0);
    f[6] = (float)(std::log10(s1) / 8.0);
    for (int i = 1; i < 8; ++i) f[6 + i] = (float)(std::log10(std::max(sv[8 * a + i], 1e-300) / s1) / 16.0);
  }
  if (h.d_model) {
    H2D(h, d_X, feats.data(), feats.size() * 4);
    if (mlp_forward_dev(h.d_model, RANK_NF, d_X, (int64_t)nf, d_y, d_mw, h.stream)) {
      err = "rank model forward failed";
      return -3;
    }
    HSYNC(h);
    HIPCHK(hipMemcpyAsync(pred.data(), d_y, nf * 4, hipMemcpyDeviceToHost, h.stream));
    HSYNC(h);
  }
  return 0;
}

// Orthonormalises the range samples of a batch of sketches (BCGS2 over
// 64-column blocks): per block two passes of C = Q_prev^T Y_blk,
// Y_blk -= Q_prev C as batched GEMMs, then the in-block Gram-Schmidt.
static int sk_orthonormalise(Handle& h, const std::vector<SkTask>& T, const SkTask* d_T, double drop,
                             std::string& err) {
  const size_t nt = T.size();
  if (!nt) return 0;
  int smax = 1, nmax = 1;
  for (const SkTask& t : T) {
    smax = std::max(smax, t.s);
    nmax = std::max(nmax, t.n);
  }
  const int nblk = (smax + 63) / 64;
  const int ldn0 = smax;
  int64_t cdoubles = 0;
  for (const SkTask& t : T) cdoubles += (int64_t)t.s * 64 + 64;
  const size_t gtab = ((size_t)nblk * 4 * nt * sizeof(GemmTask) + 255) & ~(size_t)255;
  const int64_t bytes = (int64_t)gtab + (cdoubles + (int64_t)nt * ldn0 + 64) * 8;
  int rc;
  if ((rc = ensure(h, (void**)&h.orthbuf, &h.orthbuf_bytes, bytes, err))) return rc;
  GemmTask* d_g = (GemmTask*)h.orthbuf;
  double* Cb = (double*)((char*)h.orthbuf + gtab);
  double* n0 = Cb + cdoubles;
  std::vector<double*> cptr(nt);
  int64_t o = 0;
  for (size_t a = 0; a < nt; ++a) {
    cptr[a] = Cb + o;
    o += (int64_t)T[a].s * 64 + 64;
  }
  // tables: for block b, [proj C (nt)] [update Y (nt)], twice (the same tables serve both passes)
  std::vector<GemmTask> g((size_t)nblk * 2 * nt);
  for (int b = 0; b < nblk; ++b)
    for (size_t a = 0; a < nt; ++a) {
      const SkTask& t = T[a];
      const int j0 = b * 64;
      const int bs = j0 < t.s ? std::min(64, t.s - j0) : 0;
      const int J0 = bs > 0 ? j0 : 0;
      // C (J0 x bs, ld s) = Y[:, :J0]^T Y[:, j0:j0+bs]
      g[((size_t)b * 2 + 0) * nt + a] = {t.Y, t.Y + (int64_t)j0 * t.n, cptr[a], J0, bs, t.n, t.n, t.n, t.s, 1, 0, 1.0,
                                         0.0};
      // Y[:, j0:j0+bs] -= Y[:, :J0] C
      g[((size_t)b * 2 + 1) * nt + a] = {t.Y, cptr[a], t.Y + (int64_t)j0 * t.n, t.n, bs, J0, t.n, t.s, t.n, 0, 0, -1.0,
                                         1.0};
    }
  H2D(h, d_g, held(h, g), g.size() * sizeof(GemmTask));
  hipLaunchKernelGGL(k_sk_colnorm, dim3((unsigned)std::max(1, std::min(64, (smax + 3) / 4)), (unsigned)nt), dim3(NT), 0,
                     h.stream, d_T, n0, ldn0);
  for (int b = 0; b < nblk; ++b) {
    if (b > 0) {
      const unsigned tj = (unsigned)((b * 64 + 63) / 64), tn = (unsigned)((nmax + 63) / 64);
      for (int pass = 0; pass < 2; ++pass) {
        gemm_batch(h, dim3(tj, 1, (unsigned)nt), g.data() + ((size_t)b * 2) * nt, nt, d_g + ((size_t)b * 2) * nt,
                   h.stream);
        gemm_batch(h, dim3(tn, 1, (unsigned)nt), g.data() + ((size_t)b * 2 + 1) * nt, nt,
                   d_g + ((size_t)b * 2 + 1) * nt, h.stream);
      }
    }
    hipLaunchKernelGGL(k_sk_orth_block, dim3((unsigned)nt), dim3(NT), 0, h.stream, d_T, b * 64, drop, n0, ldn0);
  }
  return 0;
}

// X = D^-1 X for the nb large pivots of tasks (orders <= dmax, X widths <=
// wmax): the right-looking blocked LU of [D | X] with the panel steps, then
// the blocked backward substitution, every step one launch over all pivots.
static void enqueue_blocked_lu(const BluTask* d_blu, unsigned nb, int dmax, int wmax, hipStream_t st) {
  const unsigned wch = (unsigned)std::max(1, (wmax + 63) / 64);
  const int nsteps = (dmax + BLU_NB - 1) / BLU_NB;
  for (int s = 0; s < nsteps; ++s) {
    const int j0 = s * BLU_NB;
    const unsigned rows = (unsigned)std::max(1, (dmax - j0 - BLU_NB + 63) / 64);
    const unsigned cols = (unsigned)((std::max(0, dmax - j0 - BLU_NB) + 63) / 64 + (wmax + 63) / 64 + 1);
    const unsigned swp = (unsigned)((dmax + wmax + NT - 1) / NT);
    hipLaunchKernelGGL(k_blu_panel, dim3(nb), dim3(NT), 0, st, d_blu, j0);
    hipLaunchKernelGGL(k_blu_swap, dim3(swp, nb), dim3(NT), 0, st, d_blu, j0);
    hipLaunchKernelGGL(k_blu_trsm, dim3(cols, nb), dim3(NT), 0, st, d_blu, j0);
    if (dmax - j0 - BLU_NB > 0) hipLaunchKernelGGL(k_blu_gemm, dim3(rows, cols, nb), dim3(NT), 0, st, d_blu, j0);
  }
  hipLaunchKernelGGL(k_blu_uinv, dim3((unsigned)nsteps, nb), dim3(NT), 0, st, d_blu);
  for (int s = nsteps - 1; s >= 0; --s) {
    const int j0 = s * BLU_NB;
    hipLaunchKernelGGL(k_bu_trsm, dim3(wch, nb), dim3(NT), 0, st, d_blu, s);
    if (j0 > 0) hipLaunchKernelGGL(k_bu_gemm, dim3((unsigned)((j0 + 63) / 64), wch, nb), dim3(NT), 0, st, d_blu, s);
  }
}

// State of one colour's elimination, shared by its steps: the host tables
// (records, neighbour entries, far pairs, changed nodes, tasks), their device
// copies in the meta buffer, the algorithmic counts, and the recompression's
// per-task bookkeeping.
struct ColourWork {
  int l = 0, c = 0, g0 = 0, nrec = 0, sides = 1, nchg = 0, nbase = 0;
  bool sym = true;
  std::vector<ElimRec> recs;
  std::vector<ElimNbr> nbrs;
  std::vector<int32_t> far_idx;
  std::vector<FarPair> far;
  std::vector<Changed> chg;
  std::vector<FarRef> refs;
  std::vector<SchurTask> tasks;
  std::vector<XTask> xtasks;
  std::vector<EigTask> etasks;  // per changed node and side: its Gram matrix
  std::vector<int64_t> dinv_off;
  double* S0 = nullptr;         // colour scratch
  std::vector<BluTask> blu;     // large pivots (blocked LU)
  std::vector<int32_t> blu_rec;
  int blu_dmax = 0, blu_wmax = 0;
  char* M = nullptr;            // meta buffer (device tables)
  size_t o_blu = 0, o_blur = 0;
  const ElimRec* d_recs = nullptr;
  const ElimNbr* d_nbrs = nullptr;
  const SchurTask* d_tasks = nullptr;
  const int32_t* d_fidx = nullptr;
  const FarPair* d_far = nullptr;
  Changed* d_chg = nullptr;
  const FarRef* d_refs = nullptr;
  const EigTask* d_et = nullptr;
  int32_t* d_cnt = nullptr;
  int32_t* d_info = nullptr;
  const XTask* d_xt = nullptr;
  LevelView V;
  double fl_lu = 0, fl_x = 0, fl_schur = 0, by_gather = 0, by_schur = 0, fl_gram = 0, fl_ev = 0, fl_evec = 0;
  double fl_far = 0;  // the far fill-in products' share of fl_schur
  // recompression: counts per task, pivot info per record, the tasks that
  // ended with a full decomposition and the accepted sketches
  std::vector<int32_t> cnt, info, full_ids, sk_ids, fe_ids;
  std::vector<EigTask> fullT, skE;
  std::vector<SkTask> skT;
  std::vector<float> rfeat;
  // capacity growth of M2L blocks (moves of slot pointers, new capacities)
  std::vector<SlotMove> moves;
  std::vector<int32_t> capset;
};

// Records, neighbour entries, far pairs, Schur and pivot-solve tasks, changed
// nodes; scratch offsets and persistent factor storage, in record order.
static int colour_tables(Handle& h, ColourWork& W, std::string& err) {
  const int l = W.l, c = W.c, nrec = W.nrec, sides = W.sides, K = h.K;
  const bool sym = W.sym;
  const Level& T = h.tree.levels[l];
  DevLevel& L = h.lv[l];
  auto& recs = W.recs;
  auto& nbrs = W.nbrs;
  auto& far_idx = W.far_idx;
  auto& far = W.far;
  auto& chg = W.chg;
  auto& refs = W.refs;
  auto& tasks = W.tasks;
  auto& xtasks = W.xtasks;
  auto& etasks = W.etasks;
  auto& dinv_off = W.dinv_off;
  auto& S0 = W.S0;
  auto& cnt = W.cnt;
  const int g0 = W.g0;
  int rc = 0;
  // ---- records, neighbour entries, far pairs, changed nodes (host; sizes are known)
  recs.assign(nrec, ElimRec());
  int64_t sc = 0;  // scratch doubles
  auto stake = [&](int64_t cnt) {
    const int64_t o = sc;
    sc += (std::max<int64_t>(cnt, 1) + 31) & ~31LL;
    return o;
  };
  std::vector<int64_t> x_off(nrec), l_off(nrec, 0), u_off(nrec, 0);
  dinv_off.assign(nrec, 0);
  std::vector<std::vector<int64_t>> far_off_F, far_off_D;
  struct ChgOff { int64_t gs, gt, vs, vt, ws, wt, ls, lt, T, S, tmp; };
  std::vector<ChgOff> coff;
  // topology and sizes per record, in parallel over contiguous record chunks
  // (each chunk's entries are local; they are concatenated in record order)
  struct Part {
    std::vector<ElimNbr> nbrs;
    std::vector<int32_t> far_idx;  // chunk-local far indices
    std::vector<FarPair> far;
    std::vector<SchurTask> tasks;
    std::vector<XTask> xtasks;
    bool bad = false;
  };
  const int nparts = std::max(1, std::min(host_threads(), nrec / 64));
  std::vector<Part> parts(nparts);
  std::vector<int> part_end(nparts);
  parallel_chunks(nrec, nparts, [&](int pc, int k0, int k1) {
    Part& P = parts[pc];
    part_end[pc] = k1;
    for (int k = k0; k < k1; ++k) {
      const int i = T.grp[g0 + k];
      ElimRec& R = recs[k];
      R.node = i;
      R.n = L.n[i];
      R.r = L.r[i];
      R.d = R.n + R.r;
      R.nnb = T.nbr_ptr[i + 1] - T.nbr_ptr[i];
      R.nb_begin = (int)P.nbrs.size();
      int off = 0;
      for (int s = T.nbr_ptr[i]; s < T.nbr_ptr[i + 1]; ++s) {
        const int p = T.nbr[s];
        ElimNbr B;
        B.p = p;
        B.elim = T.colour[p] < c ? 1 : 0;
        B.m = B.elim ? L.r[p] : L.n[p];
        B.off = off;
        off += B.m;
        // block (p, i) in p's near list, block (i, p) in i's
        B.blk_pi = -1;
        for (int t = L.near_ptr[p]; t < L.near_ptr[p + 1]; ++t)
          if (L.near_idx[t] == i) B.blk_pi = L.near_off[t];
        B.blk_ip = -1;
        for (int t = L.near_ptr[i]; t < L.near_ptr[i + 1]; ++t)
          if (L.near_idx[t] == p) B.blk_ip = L.near_off[t];
        P.nbrs.push_back(B);
      }
      R.M = off;
      R.far_base = (int)P.far_idx.size();
      R.inv = R.d >= h.big_d ? 1 : 0;  // blocked path: X also carries the x-columns of D^-1
      // far pairs (a, b) with dist(p_a, p_b) >= 2
      const ElimNbr* E = &P.nbrs[R.nb_begin];
      for (int a = 0; a < R.nnb; ++a)
        for (int b = 0; b < R.nnb; ++b) {
          if (T.dist(E[a].p, E[b].p) <= 1) {
            P.far_idx.push_back(-1);
            continue;
          }
          P.far_idx.push_back((int32_t)P.far.size());
          FarPair F;
          F.rec = k; F.a = a; F.b = b;
          F.direct = (E[a].elim && E[b].elim) ? 1 : 0;
          F.F = nullptr; F.D = nullptr;
          // M2L block (p_a, p_b): p_b is in the interaction list of p_a
          const int pa = E[a].p, pb = E[b].p;
          int lo = T.il_ptr[pa], hi = T.il_ptr[pa + 1] - 1, found = -1;
          while (lo <= hi) {
            const int mid = (lo + hi) >> 1;
            if (T.il[mid] == pb) { found = mid; break; }
            if (T.il[mid] < pb) lo = mid + 1; else hi = mid - 1;
          }
          if (found < 0) {
            P.bad = true;
            return;
          }
          F.dst = L.il_blk[found];
          F.dst_ld = L.ilcap[pa];
          F.pad = 0;
          P.far.push_back(F);
        }
      // schur tasks: one per neighbour row block plus the row R_z_i; large
      // nodes get one task per (row block, column block) pair, and those
      // with long products (n >= 128) one per 64 x 64 output tile of each
      // pair (the blocks of the row R_z_i stay whole)
      const bool split = (int64_t)R.n * R.M >= (int64_t)64 * 1024;
      for (int a = 0; a <= R.nnb; ++a) {
        if (!split) {
          P.tasks.push_back({k, a, -2, -1});
        } else if (a == R.nnb || R.n < 128) {
          for (int b = -1; b < R.nnb; ++b) P.tasks.push_back({k, a, b, -1});
        } else {
          const int mt = (E[a].m + 63) / 64;
          for (int b = -1; b < R.nnb; ++b) {
            const int nt = ((b >= 0 ? E[b].m : R.r) + 63) / 64;
            for (int tj = 0; tj < nt; ++tj)
              for (int ti = 0; ti < mt; ++ti) P.tasks.push_back({k, a, b, ti | (tj << 16)});
          }
        }
      }
      if (R.d < h.big_d)
        for (int c0 = 0; c0 < R.M + R.r + R.n; c0 += XCOLS) P.xtasks.push_back({k, c0});
    }
  });
  {
    size_t nn = 0, nf = 0, nfi = 0, nt = 0, nx = 0;
    for (const Part& P : parts) {
      if (P.bad) {
        err = "internal: far neighbour pair is not in the interaction list";
        return -1;
      }
      nn += P.nbrs.size(); nf += P.far.size(); nfi += P.far_idx.size(); nt += P.tasks.size(); nx += P.xtasks.size();
    }
    nbrs.reserve(nn); far.reserve(nf); far_idx.reserve(nfi); tasks.reserve(nt); xtasks.reserve(nx);
    int k0 = 0;
    for (int pc = 0; pc < nparts; ++pc) {
      Part& P = parts[pc];
      const int nb0 = (int)nbrs.size(), fi0 = (int)far_idx.size(), f0 = (int)far.size();
      for (int k = k0; k < part_end[pc]; ++k) {
        recs[k].nb_begin += nb0;
        recs[k].far_base += fi0;
      }
      k0 = part_end[pc];
      nbrs.insert(nbrs.end(), P.nbrs.begin(), P.nbrs.end());
      for (int32_t v : P.far_idx) far_idx.push_back(v < 0 ? v : v + f0);
      far.insert(far.end(), P.far.begin(), P.far.end());
      tasks.insert(tasks.end(), P.tasks.begin(), P.tasks.end());
      xtasks.insert(xtasks.end(), P.xtasks.begin(), P.xtasks.end());
    }
  }
  // scratch and persistent factor storage, in record order
  for (int k = 0; k < nrec; ++k) {
    ElimRec& R = recs[k];
    x_off[k] = stake((int64_t)R.d * (R.M + R.r + R.n));
    dinv_off[k] = R.inv ? stake((int64_t)((R.d + BLU_NB - 1) / BLU_NB) * 2 * 4096) : 0;
    double* p;
    if ((rc = store_take(h, (int64_t)R.d * R.d, &R.lu, err))) return rc;
    if ((rc = store_take(h, (R.d + 1) / 2 + 1, &p, err))) return rc;
    R.piv = (int32_t*)p;
    R.Ls = R.Us = nullptr;
    if (h.solve32) {
      // L and U are colour work; the solve keeps FP32 copies
      l_off[k] = stake((int64_t)R.M * R.n);
      u_off[k] = stake((int64_t)R.n * R.M);
      if ((rc = store32_take(h, (int64_t)R.M * R.n, &R.Ls, err))) return rc;
      if ((rc = store32_take(h, (int64_t)R.n * R.M, &R.Us, err))) return rc;
    } else {
      if ((rc = store_take(h, (int64_t)R.M * R.n, &R.L, err))) return rc;
      if ((rc = store_take(h, (int64_t)R.n * R.M, &R.U, err))) return rc;
    }
    R.wv = L.wv_total;
    L.wv_total += R.d;
  }
  // scratch for far pairs
  std::vector<int64_t> fF(far.size()), fD(far.size());
  for (size_t f = 0; f < far.size(); ++f) {
    const ElimRec& R = recs[far[f].rec];
    const int ma = nbrs[R.nb_begin + far[f].a].m, mb = nbrs[R.nb_begin + far[f].b].m;
    fF[f] = stake((int64_t)ma * mb);
    fD[f] = stake((int64_t)ma * mb);
  }
  // changed nodes: non-eliminated neighbours with at least one far partner
  for (int k = 0; k < nrec; ++k) {
    const ElimRec& R = recs[k];
    for (int a = 0; a < R.nnb; ++a) {
      const ElimNbr& A = nbrs[R.nb_begin + a];
      if (A.elim) continue;
      const int fb = (int)refs.size();
      for (int b = 0; b < R.nnb; ++b) {
        const int ab = far_idx[R.far_base + a * R.nnb + b];
        if (ab < 0) continue;
        const int ba = far_idx[R.far_base + b * R.nnb + a];
        refs.push_back({nbrs[R.nb_begin + b].p, ab, ba, 0});
      }
      if ((int)refs.size() == fb) continue;
      Changed C;
      std::memset(&C, 0, sizeof(C));
      C.p = A.p; C.rec = k; C.a = a; C.n = L.n[A.p]; C.r = L.r[A.p]; C.rnew = 0;
      C.far_begin = fb; C.far_count = (int)refs.size() - fb;
      const int64_t n = C.n;
      const int64_t big = std::max<int64_t>(std::max<int64_t>(L.rcmax, K), n);
      ChgOff o;
      const int64_t wsz = h.eig_jacobi ? n * n : 3 * n;
      o.gs = stake(n * n); o.vs = stake(n * n); o.ws = stake(wsz); o.ls = stake(n);
      if (sym) {
        o.gt = o.gs; o.vt = o.vs; o.wt = o.ws; o.lt = o.ls;
      } else {
        o.gt = stake(n * n); o.vt = stake(n * n); o.wt = stake(wsz); o.lt = stake(n);
      }
      o.T = stake((int64_t)std::max(C.r, 1) * n);
      o.S = stake(n * std::max(C.r, 1));
      o.tmp = stake(std::max<int64_t>(big * std::max<int64_t>(std::max<int64_t>(L.rc[A.p], n), 1),
                                      (int64_t)sides * C.r * n));
      coff.push_back(o);
      chg.push_back(C);
    }
  }
  if ((rc = ensure(h, (void**)&h.scratch, &h.scratch_bytes, sc * 8 + 256, err))) return rc;
  S0 = h.scratch;
  for (int k = 0; k < nrec; ++k) {
    recs[k].X = S0 + x_off[k];
    if (h.solve32) {
      recs[k].L = S0 + l_off[k];
      recs[k].U = S0 + u_off[k];
    }
  }
  for (size_t f = 0; f < far.size(); ++f) { far[f].F = S0 + fF[f]; far[f].D = S0 + fD[f]; }
  for (size_t k = 0; k < chg.size(); ++k) {
    Changed& C = chg[k];
    const ChgOff& o = coff[k];
    C.gs = S0 + o.gs; C.gt = S0 + o.gt; C.vs = S0 + o.vs; C.vt = S0 + o.vt; C.ws = S0 + o.ws; C.wt = S0 + o.wt;
    C.ls = S0 + o.ls; C.lt = S0 + o.lt; C.T = S0 + o.T; C.S = S0 + o.S; C.tmp = S0 + o.tmp;
    etasks.push_back({C.gs, C.vs, C.ws, C.ls, nullptr, C.n, 0});
    if (!sym) etasks.push_back({C.gt, C.vt, C.wt, C.lt, nullptr, C.n, 0});
  }
  return 0;
}

// Packs the tables into the meta buffer, uploads them, and counts the
// algorithmic work of the phase-A steps from the block sizes.
static int colour_upload(Handle& h, ColourWork& W, std::string& err) {
  const int l = W.l, nrec = W.nrec, sides = W.sides;
  DevLevel& L = h.lv[l];
  auto& recs = W.recs;
  auto& nbrs = W.nbrs;
  auto& far_idx = W.far_idx;
  auto& far = W.far;
  auto& chg = W.chg;
  auto& refs = W.refs;
  auto& tasks = W.tasks;
  auto& xtasks = W.xtasks;
  auto& etasks = W.etasks;
  auto& dinv_off = W.dinv_off;
  auto& S0 = W.S0;
  auto& blu = W.blu;
  auto& blu_rec = W.blu_rec;
  auto& blu_dmax = W.blu_dmax;
  auto& blu_wmax = W.blu_wmax;
  auto& M = W.M;
  auto& o_blu = W.o_blu;
  auto& o_blur = W.o_blur;
  auto& d_recs = W.d_recs;
  auto& d_nbrs = W.d_nbrs;
  auto& d_tasks = W.d_tasks;
  auto& d_fidx = W.d_fidx;
  auto& d_far = W.d_far;
  auto& d_chg = W.d_chg;
  auto& d_refs = W.d_refs;
  auto& d_et = W.d_et;
  auto& d_cnt = W.d_cnt;
  auto& d_info = W.d_info;
  auto& d_xt = W.d_xt;
  auto& V = W.V;
  auto& nchg = W.nchg;
  auto& fl_lu = W.fl_lu;
  auto& fl_x = W.fl_x;
  auto& fl_schur = W.fl_schur;
  auto& by_gather = W.by_gather;
  auto& by_schur = W.by_schur;
  auto& fl_gram = W.fl_gram;
  auto& fl_ev = W.fl_ev;
  int rc = 0;
  // ---- pack the tables into the meta buffer
  auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t o_recs = 0;
  const size_t o_nbrs = o_recs + al(recs.size() * sizeof(ElimRec));
  const size_t o_tasks = o_nbrs + al(std::max<size_t>(nbrs.size(), 1) * sizeof(ElimNbr));
  const size_t o_fidx = o_tasks + al(tasks.size() * sizeof(SchurTask));
  const size_t o_far = o_fidx + al(std::max<size_t>(far_idx.size(), 1) * 4);
  const size_t o_chg = o_far + al(std::max<size_t>(far.size(), 1) * sizeof(FarPair));
  const size_t o_refs = o_chg + al(std::max<size_t>(chg.size(), 1) * sizeof(Changed));
  const size_t o_et = o_refs + al(std::max<size_t>(refs.size(), 1) * sizeof(FarRef));
  const size_t o_cnt = o_et + al(std::max<size_t>(etasks.size(), 1) * sizeof(EigTask));
  const size_t o_xt = o_cnt + al(std::max<size_t>(etasks.size(), 1) * 4);
  // large pivots (blocked LU of the augmented matrix, many workgroups each)
  for (int k = 0; k < nrec; ++k)
    if (recs[k].inv) {
      const int W = recs[k].M + recs[k].r + recs[k].n;
      blu.push_back({recs[k].lu, recs[k].X, recs[k].piv, nullptr, S0 + dinv_off[k], recs[k].d, W});
      blu_rec.push_back(k);
      blu_dmax = std::max(blu_dmax, recs[k].d);
      blu_wmax = std::max(blu_wmax, W);
    }
  const size_t o_info = o_xt + al(std::max<size_t>(xtasks.size(), 1) * sizeof(XTask));
  o_blu = o_info + al((size_t)nrec * 4);
  o_blur = o_blu + al(std::max<size_t>(blu.size(), 1) * sizeof(BluTask));
  const size_t total = o_blur + al(std::max<size_t>(blu_rec.size(), 1) * 4);
  if ((rc = ensure(h, (void**)&h.meta, &h.meta_bytes, (int64_t)total, err))) return rc;
  M = (char*)h.meta;
  h.host_meta.assign(total, 0);
  char* Hm = h.host_meta.data();
  std::memcpy(Hm + o_recs, recs.data(), recs.size() * sizeof(ElimRec));
  if (!nbrs.empty()) std::memcpy(Hm + o_nbrs, nbrs.data(), nbrs.size() * sizeof(ElimNbr));
  std::memcpy(Hm + o_tasks, tasks.data(), tasks.size() * sizeof(SchurTask));
  if (!far_idx.empty()) std::memcpy(Hm + o_fidx, far_idx.data(), far_idx.size() * 4);
  if (!far.empty()) std::memcpy(Hm + o_far, far.data(), far.size() * sizeof(FarPair));
  if (!chg.empty()) std::memcpy(Hm + o_chg, chg.data(), chg.size() * sizeof(Changed));
  if (!refs.empty()) std::memcpy(Hm + o_refs, refs.data(), refs.size() * sizeof(FarRef));
  if (!etasks.empty()) std::memcpy(Hm + o_et, etasks.data(), etasks.size() * sizeof(EigTask));
  if (!xtasks.empty()) std::memcpy(Hm + o_xt, xtasks.data(), xtasks.size() * sizeof(XTask));
  for (size_t b = 0; b < blu.size(); ++b) blu[b].info = (int32_t*)(M + o_info) + blu_rec[b];
  if (!blu.empty()) {
    std::memcpy(Hm + o_blu, blu.data(), blu.size() * sizeof(BluTask));
    std::memcpy(Hm + o_blur, blu_rec.data(), blu_rec.size() * 4);
  }
  H2D(h, M, Hm, o_info);
  if (!blu.empty())
    H2D(h, M + o_blu, Hm + o_blu, total - o_blu);
  d_recs = (const ElimRec*)(M + o_recs);
  d_nbrs = (const ElimNbr*)(M + o_nbrs);
  d_tasks = (const SchurTask*)(M + o_tasks);
  d_fidx = (const int32_t*)(M + o_fidx);
  d_far = (const FarPair*)(M + o_far);
  d_chg = (Changed*)(M + o_chg);
  d_refs = (const FarRef*)(M + o_refs);
  d_et = (const EigTask*)(M + o_et);
  d_cnt = (int32_t*)(M + o_cnt);
  d_info = (int32_t*)(M + o_info);
  d_xt = (const XTask*)(M + o_xt);
  V = view_of(L);
  nchg = (int)chg.size();
  // algorithmic work of the phase-A steps (counted from the block sizes)
  double& fl_far = W.fl_far;
  fl_far = 0;
  for (const FarPair& F : far) {  // far fill-in products (FP32 in the mixed form)
    const ElimRec& R = recs[F.rec];
    fl_far += 2.0 * nbrs[R.nb_begin + F.a].m * (double)R.n * nbrs[R.nb_begin + F.b].m;
  }
  h.aux["schur_far_flops"] += fl_far;
  for (const ElimRec& R : recs) {
    const double d = R.d, n = R.n, M = R.M, r = R.r;
    fl_lu += 2.0 / 3.0 * d * d * d;
    fl_x += 2.0 * d * d * (M + r);
    fl_schur += 2.0 * M * n * (M + r);
    by_schur += 8.0 * (M * n + (double)R.d * (M + r) + 2.0 * M * (M + r));  // L, X once; blocks read + written
    by_gather += 8.0 * (d * d + 2.0 * M * n) * 2.0;
  }
  for (const Changed& C : chg) {
    double sm = C.r;
    for (int q = 0; q < C.far_count; ++q) {
      const FarPair& F = far[refs[C.far_begin + q].ba];
      sm += nbrs[recs[F.rec].nb_begin + F.a].m;
    }
    fl_gram += sides * (double)C.n * (C.n + 1) * sm;  // symmetric product: lower triangle
    fl_ev += sides * 4.0 / 3.0 * (double)C.n * C.n * C.n;
  }
  return 0;
}

// Phase A: gather of the pivots and their neighbour blocks, pivot LU and
// solves (small pivots on the side stream, large ones blocked), the solve's
// stored blocks, the Schur-complement update, the Gram matrices of the fill-in.
static int colour_phase_a(Handle& h, ColourWork& W, std::string& err) {
  const int l = W.l, c = W.c, nrec = W.nrec, sides = W.sides;
  DevLevel& L = h.lv[l];
  auto& recs = W.recs;
  auto& nbrs = W.nbrs;
  auto& chg = W.chg;
  auto& tasks = W.tasks;
  auto& xtasks = W.xtasks;
  auto& blu = W.blu;
  auto& blu_dmax = W.blu_dmax;
  auto& blu_wmax = W.blu_wmax;
  auto& M = W.M;
  auto& o_blu = W.o_blu;
  auto& o_blur = W.o_blur;
  auto& d_recs = W.d_recs;
  auto& d_nbrs = W.d_nbrs;
  auto& d_tasks = W.d_tasks;
  auto& d_fidx = W.d_fidx;
  auto& d_far = W.d_far;
  auto& d_chg = W.d_chg;
  auto& d_refs = W.d_refs;
  auto& d_info = W.d_info;
  auto& d_xt = W.d_xt;
  auto& V = W.V;
  auto& nchg = W.nchg;
  auto& fl_lu = W.fl_lu;
  auto& fl_x = W.fl_x;
  auto& fl_schur = W.fl_schur;
  auto& by_gather = W.by_gather;
  auto& by_schur = W.by_schur;
  auto& fl_gram = W.fl_gram;
  const double fl_far = W.fl_far;
  int rc = 0;
  // ---- phase A
  {
    ProfScope ps(h, "k_gather", 0, by_gather);
    int wmax = 1, pmax = 1;
    for (const ElimRec& R : recs) {
      wmax = std::max(wmax, R.d);
      pmax = std::max(pmax, 1 + R.nnb);
    }
    for (const ElimNbr& B : nbrs) wmax = std::max(wmax, B.m);
    hipLaunchKernelGGL(k_gather, dim3((unsigned)nrec, (unsigned)pmax, (unsigned)((wmax + GATHER_COLS - 1) / GATHER_COLS)),
                       dim3(NT), 0, h.stream, V, d_recs, d_nbrs);
  }
  if ((rc = check_arena(h, l, "gather", c, err))) return rc;
  // small pivots (unblocked LU and solve) on the side stream while the large
  // ones go through the blocked LU on the main stream (different records)
  const bool aside = !blu.empty() && !xtasks.empty();
  if (aside && (rc = fork_side(h, err))) return rc;
  const hipStream_t sa = aside ? h.side_stream : h.stream;
  {
    ProfScope ps(h, "k_getrf", fl_lu, 0, aside);
    hipLaunchKernelGGL(k_getrf, dim3(nrec), dim3(NT), 0, sa, d_recs, d_info, h.big_d);
  }
  if (!xtasks.empty()) {
    ProfScope ps(h, "k_xsolve", fl_x, 0, aside);
    int dmx = 0;
    for (const ElimRec& R : recs)
      if (R.d < h.big_d) dmx = std::max(dmx, R.d);
    // one row per thread up to order NT (every small pivot with the default
    // threshold), else the slice in LDS or in place
    auto kx = dmx <= NT ? k_xsolve_rows : dmx <= 64 ? k_xsolve<64> : k_xsolve<256>;
    hipLaunchKernelGGL(kx, dim3((unsigned)xtasks.size()), dim3(NT), 0, sa, d_recs, d_xt);
  }
  if (!blu.empty()) {
    const BluTask* d_blu = (const BluTask*)(M + o_blu);
    const int32_t* d_blur = (const int32_t*)(M + o_blur);
    const unsigned nb = (unsigned)blu.size();
    double fl_blu = 0;
    for (const BluTask& b : blu) fl_blu += 2.0 / 3.0 * b.d * (double)b.d * b.d + 2.0 * (double)b.d * b.d * b.W;  // LU + both triangular solves
    ProfScope ps(h, "group:blocked_lu", fl_blu, 0);
    const unsigned wch = (unsigned)std::max(1, (blu_wmax + 63) / 64);
    hipLaunchKernelGGL(k_blu_xinit, dim3(wch, nb), dim3(NT), 0, h.stream, d_blu, d_recs, d_blur);
    enqueue_blocked_lu(d_blu, nb, blu_dmax, blu_wmax, h.stream);
  }
  if (aside && (rc = join_side(h, err))) return rc;
  {
    // the solve's blocks: explicit pivot inverses and G = x-rows of X
    int wmax = 1;
    for (const ElimRec& R : recs) wmax = std::max(wmax, std::max(R.d, R.M));
    hipLaunchKernelGGL(k_store_solve, dim3((unsigned)((wmax + 63) / 64), (unsigned)nrec), dim3(NT), 0, h.stream, d_recs);
  }
  {
    // inner dimension of the products = n of the pivot; the double-buffered
    // FP32 tile only from pivot order h.deep_n on (off unless set: the lite
    // tile keeps more workgroups resident and measured faster at every level)
    int nmx = 0;
    for (const ElimRec& R : recs) nmx = std::max(nmx, R.n);
    // FP64 products on the FMA tile (0) or the FP64 matrix cores (1): the
    // built-in choice unless the autotuner has one; a level it has not seen
    // alternates the two over its colours, timed.  The mixed form's FP32
    // products take the deep tile from pivot order h.deep_n on.
    bool alt = h.f64_mfma;
    bool explore = false;
    std::string tkey;
    if (!h.tune_cache.empty()) {
      tkey = schur_key(h, l);
      const auto it = h.tune.find(tkey);
      explore = it == h.tune.end();
      alt = explore ? (c % 2) == 1 : it->second != 0;
    }
    const bool deep = nmx >= h.deep_n;
    // mixed form: the near products (FP64) on the main stream and the far
    // fill-in products (FP32) on the side stream at the same time, as two
    // kernels with one tile each (they write disjoint blocks)
    const bool split = h.precision == 1 && h.schur_split && fl_far > 0;
    if (split && (rc = fork_side(h, err))) return rc;
    {
      ProfScope ps(h, "k_schur", split ? fl_schur - fl_far : fl_schur, by_schur);
      auto ks = h.precision != 1 ? (alt ? k_schur<false, false, true, 0> : k_schur<false, false, false, 0>)
                : split ? (alt ? k_schur<true, false, true, 1> : k_schur<true, false, false, 1>)
                : deep  ? (alt ? k_schur<true, true, true, 0> : k_schur<true, true, false, 0>)
                        : (alt ? k_schur<true, false, true, 0> : k_schur<true, false, false, 0>);
      hipEvent_t ta_ = nullptr, tb_ = nullptr;
      if (explore) {
        ta_ = take_event(h);
        tb_ = take_event(h);
        HIPCHK(hipEventRecord(ta_, h.stream));
      }
      hipLaunchKernelGGL(ks, dim3((unsigned)tasks.size()), dim3(NT), 0, h.stream, V, d_recs, d_nbrs, d_tasks, d_fidx,
                         d_far);
      if (explore) {
        HIPCHK(hipEventRecord(tb_, h.stream));
        h.tune_pending.push_back({ta_, tb_, tkey, alt ? 1 : 0, alt ? 1 : 0, std::max(fl_schur, 1.0)});
      }
    }
    if (split) {
      ProfScope ps(h, "k_schur_far", fl_far, 0, true);
      auto kf = deep ? k_schur<true, true, false, 2> : k_schur<true, false, false, 2>;
      hipLaunchKernelGGL(kf, dim3((unsigned)tasks.size()), dim3(NT), 0, h.side_stream, V, d_recs, d_nbrs, d_tasks,
                         d_fidx, d_far);
    }
    if (split && (rc = join_side(h, err))) return rc;
  }
  if ((rc = check_arena(h, l, "schur", c, err))) return rc;
  if (nchg) {
    hipLaunchKernelGGL(k_set_chg, dim3((nchg + NT - 1) / NT), dim3(NT), 0, h.stream, L.d_chg, d_chg, nchg, 0);
    {
      int nmax = 0;
      for (const Changed& C : chg) nmax = std::max(nmax, C.n);
      const int nbt = (nmax + 63) / 64;
      hipLaunchKernelGGL(k_gram_prep, dim3(sides * nchg), dim3(NT), 0, h.stream, V, d_chg, sides);
      ProfScope ps(h, "k_gram", fl_gram, 0);
      hipLaunchKernelGGL(k_gram, dim3((unsigned)std::max(1, nbt * (nbt + 1) / 2), sides * nchg), dim3(NT), 0,
                         h.stream, V, d_chg, d_refs, d_far, d_nbrs, d_recs, sides);
    }
  }
  return 0;
}

// One batch of sketches (the randomised range finder of Sec. 5.1): for task
// e of the colour (changed node e / sides, side e % sides) with width w, the
// range sample of the stacked factor with a seeded Gaussian test matrix, its
// orthonormalisation, the Rayleigh-Ritz step with the Gram matrix and the
// a-posteriori check.  Tables and work space live in *buf (grown as needed);
// the Ritz counts and the verdicts land in B.d_cnt and B.d_ok.
struct SketchBatch {
  std::vector<SkTask> T;
  std::vector<EigTask> E;  // Rayleigh-Ritz eigen-problems (order = width)
  SkTask* d_T = nullptr;
  EigTask* d_E = nullptr;
  int32_t* d_cnt = nullptr;
  int32_t* d_ok = nullptr;
};
static int sketch_batch(Handle& h, const ColourWork& W, const std::vector<int32_t>& ids,
                        const std::vector<int32_t>& width, const std::vector<int64_t>& wrows, uint32_t salt,
                        double** buf, int64_t* buf_bytes, SketchBatch& B, std::string& err) {
  const int sides = W.sides;
  const size_t ns = ids.size();
  B.T.clear();
  B.E.clear();
  if (!ns) return 0;
  int64_t need = 0;
  for (size_t q = 0; q < ns; ++q) {
    const int64_t n = W.chg[ids[q] / sides].n, sw = width[q];
    need += std::max<int64_t>(wrows[ids[q] / sides], n) * sw + n * sw + 2 * sw * sw + 3 * sw + 64;
  }
  const size_t tb = (ns * (sizeof(EigTask) + sizeof(SkTask) + 2 * sizeof(GemmTask) + 8) + 4096 + 255) & ~(size_t)255;
  int rc;
  if ((rc = ensure(h, (void**)buf, buf_bytes, (int64_t)tb + need * 8 + 256, err))) return rc;
  char* base = (char*)*buf;
  B.d_E = (EigTask*)base;
  B.d_T = (SkTask*)(B.d_E + ns);
  GemmTask* d_G = (GemmTask*)(B.d_T + ns);
  B.d_cnt = (int32_t*)(d_G + 2 * ns);
  B.d_ok = B.d_cnt + ns;
  double* W0 = (double*)(base + tb);
  int64_t o = 0;
  int smax = 1, nmax = 1;
  for (size_t q = 0; q < ns; ++q) {
    const int e = ids[q];
    const Changed& C = W.chg[e / sides];
    const int side = e % sides, n = C.n, sw = width[q];
    SkTask t;
    t.G = side ? C.gt : C.gs;
    t.O = W0 + o; o += std::max<int64_t>(wrows[e / sides], n) * sw;
    t.Y = W0 + o; o += (int64_t)n * sw;
    t.B = W0 + o; o += (int64_t)sw * sw;
    double* U = W0 + o; o += (int64_t)sw * sw;
    double* Wk = W0 + o; o += 3LL * sw;
    t.tr = W0 + o; o += 64;
    t.n = n; t.s = sw;
    t.R = (int32_t)wrows[e / sides];
    t.chg = e / sides;
    t.seed = (uint32_t)(C.p * 2 + side) + salt;
    t.side = (uint32_t)side;
    B.T.push_back(t);
    B.E.push_back({t.B, U, Wk, side ? C.lt : C.ls, nullptr, sw, 0});
    smax = std::max(smax, sw);
    nmax = std::max(nmax, n);
  }
  // Z = G Q (into O), B = Q^T Z
  std::vector<GemmTask> g;
  for (const SkTask& t : B.T) g.push_back({t.G, t.Y, t.O, t.n, t.s, t.n, t.n, t.n, t.n, 0, 0, 1.0, 0.0});
  for (const SkTask& t : B.T) g.push_back({t.Y, t.O, t.B, t.s, t.s, t.n, t.n, t.n, t.s, 1, 0, 1.0, 0.0});
  H2D(h, B.d_E, held(h, B.E), ns * sizeof(EigTask));
  H2D(h, B.d_T, held(h, B.T), ns * sizeof(SkTask));
  H2D(h, d_G, held(h, g), 2 * ns * sizeof(GemmTask));
  double fl = 0;
  for (const SkTask& t : B.T)
    fl += 2.0 * t.n * (double)t.R * t.s + 2.0 * t.n * (double)t.n * t.s + 6.0 * t.n * (double)t.s * t.s;
  const unsigned tn = (unsigned)((nmax + 63) / 64), ts = (unsigned)((smax + 63) / 64);
  const double drop = std::max(1e-13, std::min(1e-9, 1e-3 * h.eps));
  const double eps2 = h.eps * h.eps;
  {
    ProfScope ps(h, "group:sketch_range", fl, 0);
    hipLaunchKernelGGL(k_sk_omega, dim3(64, (unsigned)ns), dim3(NT), 0, h.stream, B.d_T);
    hipLaunchKernelGGL(h.precision == 1 ? k_sk_range<true> : k_sk_range<false>, dim3(tn, ts, (unsigned)ns), dim3(NT),
                       0, h.stream, W.d_chg, W.d_refs, W.d_far, W.d_nbrs, W.d_recs, B.d_T);
  }
  {
    ProfScope ps(h, "group:sketch_orth", 0, 0);
    if ((rc = sk_orthonormalise(h, B.T, B.d_T, drop, err))) return rc;
  }
  ProfScope ps(h, "group:sketch_rr", 0, 0);
  gemm_batch(h, dim3(tn, ts, (unsigned)ns), g.data(), ns, d_G, h.stream);
  gemm_batch(h, dim3(ts, ts, (unsigned)ns), g.data() + ns, ns, d_G + ns, h.stream);
  hipLaunchKernelGGL(k_sk_trace, dim3((unsigned)ns), dim3(NT), 0, h.stream, B.d_T);
  if ((rc = eig_values(h, B.E, B.d_E, eps2, B.d_cnt, h.stream, err))) return rc;
  hipLaunchKernelGGL(k_sk_check, dim3((unsigned)((ns + NT - 1) / NT)), dim3(NT), 0, h.stream, B.d_T, B.d_E, B.d_cnt,
                     eps2, B.d_ok, (int)ns);
  return 0;
}

// Recompression of the fill-in: per changed node and side a sketch of width
// s (predicted rank plus oversampling) or the full eigen-decomposition;
// rejected sketches are retried once wider, then decomposed in full.
static int colour_recompress(Handle& h, ColourWork& W, HostLap& lap, std::string& err) {
  const int l = W.l, nrec = W.nrec, sides = W.sides;
  const Level& T = h.tree.levels[l];
  auto& recs = W.recs;
  auto& nbrs = W.nbrs;
  auto& far = W.far;
  auto& chg = W.chg;
  auto& refs = W.refs;
  auto& tasks = W.tasks;
  auto& etasks = W.etasks;
  auto& d_recs = W.d_recs;
  auto& d_nbrs = W.d_nbrs;
  auto& d_far = W.d_far;
  auto& d_chg = W.d_chg;
  auto& d_refs = W.d_refs;
  auto& d_info = W.d_info;
  auto& nchg = W.nchg;
  auto& fl_ev = W.fl_ev;
  auto& cnt = W.cnt;
  auto& info = W.info;
  auto& full_ids = W.full_ids;
  auto& sk_ids = W.sk_ids;
  auto& fullT = W.fullT;
  auto& skE = W.skE;
  auto& skT = W.skT;
  auto& rfeat = W.rfeat;
  auto& fe_ids = W.fe_ids;
  int rc = 0;
  // ---- recompression: per changed node and side, either a sketch of width s
  // (predicted rank plus oversampling) or the full eigen-decomposition
  const int ne = (int)etasks.size();
  std::vector<int32_t> skw(ne, 0);
  cnt.assign(ne, 0);
  info.assign(nrec, 0);
  std::vector<int32_t> cnt_full, cnt_sk, ok_sk;
  std::vector<float> rpred;
  std::vector<int32_t> fe_of;
  if (nchg) {
    // rows of the stacked factor of each changed node's Gram matrix
    std::vector<int64_t> wrows(nchg, 0);
    for (int k = 0; k < nchg; ++k) {
      const Changed& C = chg[k];
      int64_t rr = C.r;
      for (int q = 0; q < C.far_count; ++q) {
        const FarPair& F = far[refs[C.far_begin + q].ba];
        rr += nbrs[recs[F.rec].nb_begin + F.a].m;
      }
      wrows[k] = rr;
    }
    // learned rank: features and predictions of the sketch-eligible nodes
    fe_of.assign(nchg, -1);
    if ((h.d_model || h.record_ranks) && h.sketch && !h.eig_jacobi)
      for (int k = 0; k < nchg; ++k)
        if (chg[k].n >= h.sketch_min) {
          fe_of[k] = (int32_t)fe_ids.size();
          fe_ids.push_back(k);
        }
    if (!fe_ids.empty() &&
        (rc = rank_features(h, l, chg, fe_ids, wrows, d_chg, d_refs, d_far, d_nbrs, d_recs, rfeat, rpred, err)))
      return rc;
    for (int e = 0; e < ne; ++e) {
      const int k = e / sides;
      const Changed& C = chg[k];
      int s = 0;
      if (h.sketch && !h.eig_jacobi && C.n >= h.sketch_min) {
        int pred;
        if (h.d_model && fe_of[k] >= 0) {
          const float fr = std::min(1.f, std::max(0.f, rpred[fe_of[k]]));
          pred = std::max(1, (int)std::ceil(fr * C.n));
          ++h.stat_predicted;
          s = std::min(C.n, pred + std::max(8, pred / 8));
        } else {
          pred = predict_rank(h, l, C, e % sides);
          s = std::min(C.n, pred + std::max(16, pred / 4));
        }
        if (s < 1 || s > (int)(0.6 * C.n)) s = 0;
      }
      skw[e] = s;
      (s ? sk_ids : full_ids).push_back(e);
    }
    // tables of the full decompositions (and of the fall-backs of rejected
    // sketches, at most one per sketch); the sketches have their own buffer
    const size_t nsk = sk_ids.size(), nfull = full_ids.size();
    const size_t tb = ((nfull + nsk) * sizeof(EigTask) + (nfull + nsk) * 4 + 1024 + 255) & ~(size_t)255;
    if ((rc = ensure(h, (void**)&h.eigtab, &h.eigtab_bytes, (int64_t)tb, err))) return rc;
    EigTask* d_fullT = (EigTask*)h.eigtab;
    EigTask* d_fbT = d_fullT + nfull;  // fall-back full tasks of rejected sketches
    int32_t* d_cf = (int32_t*)(d_fbT + nsk);
    int32_t* d_cfb = d_cf + nfull;
    for (int e : full_ids) fullT.push_back(etasks[e]);
    if (nfull) H2D(h, d_fullT, fullT.data(), nfull * sizeof(EigTask));
    std::vector<int32_t> sk_w;
    for (int e : sk_ids) sk_w.push_back(skw[e]);
    const double eps2 = h.eps * h.eps;
    // the full decompositions (their own Gram matrices and work space) run on
    // the side stream while the sketches run on the main stream
    const bool side = nfull && nsk;
    if (side && (rc = fork_side(h, err))) return rc;
    if (nfull) {
      ProfScope ps(h, "k_eig_values", fl_ev, 0, side);
      const hipStream_t st = side ? h.side_stream : h.stream;
      if ((rc = eig_values(h, fullT, d_fullT, eps2, d_cf, st, err))) return rc;
    }
    SketchBatch S1;
    if ((rc = sketch_batch(h, W, sk_ids, sk_w, wrows, 1, &h.skbuf, &h.skbuf_bytes, S1, err))) return rc;
    skT = S1.T;
    skE = S1.E;
    if (side && (rc = join_side(h, err))) return rc;
    HIPCHK(hipGetLastError());
    cnt_full.assign(nfull, 0);
    cnt_sk.assign(nsk, 0);
    ok_sk.assign(nsk, 0);
    lap.mark("plan_recomp");
    HSYNC(h);  // the copies below wait for the queue: accounted here
    if (nfull) HIPCHK(hipMemcpyAsync(cnt_full.data(), d_cf, nfull * 4, hipMemcpyDeviceToHost, h.stream));
    if (nsk) {
      HIPCHK(hipMemcpyAsync(cnt_sk.data(), S1.d_cnt, nsk * 4, hipMemcpyDeviceToHost, h.stream));
      HIPCHK(hipMemcpyAsync(ok_sk.data(), S1.d_ok, nsk * 4, hipMemcpyDeviceToHost, h.stream));
    }
    HIPCHK(hipMemcpyAsync(info.data(), d_info, nrec * 4, hipMemcpyDeviceToHost, h.stream));
    HSYNC(h);
    for (size_t a = 0; a < nfull; ++a) cnt[full_ids[a]] = cnt_full[a];
    // rejected sketches: full eigen-decomposition of their Gram matrices
    std::vector<EigTask> fb;
    std::vector<int32_t> fb_of;
    for (size_t a = 0; a < nsk; ++a) {
      const int e = sk_ids[a];
      if (ok_sk[a] == 0) ++h.stat_sketch_narrow;
      if (ok_sk[a] > 0) {
        cnt[e] = cnt_sk[a];
      } else {
        fb.push_back(etasks[e]);
        fb_of.push_back((int32_t)a);
      }
    }
    h.stat_sketch += (int64_t)nsk;
    h.stat_sketch_rejected += (int64_t)fb.size();
    // second chance: a rejected sketch is retried once at about twice the width
    // (still far cheaper than the full decomposition of a large Gram matrix)
    std::vector<int32_t> r2_ids, r2_w;
    {
      std::vector<EigTask> fb_keep;
      std::vector<int32_t> fbof_keep;
      for (size_t q = 0; q < fb.size(); ++q) {
        const int a = fb_of[q], e = sk_ids[a];
        const int n = chg[e / sides].n;
        const int s2 = std::min(n, 2 * skw[e] + 16);
        if (s2 <= (int)(0.8 * n)) {
          r2_ids.push_back(e);
          r2_w.push_back(s2);
        } else {
          fb_keep.push_back(fb[q]);
          fbof_keep.push_back(a);
        }
      }
      fb.swap(fb_keep);
      fb_of.swap(fbof_keep);
    }
    std::vector<int32_t> r2_ok;
    SketchBatch S2;
    if (!r2_ids.empty()) {
      const size_t n2 = r2_ids.size();
      if ((rc = sketch_batch(h, W, r2_ids, r2_w, wrows, 0x9E37, &h.skbuf2, &h.skbuf2_bytes, S2, err))) return rc;
      std::vector<int32_t> c2(n2);
      r2_ok.assign(n2, 0);
      HSYNC(h);
      HIPCHK(hipMemcpyAsync(c2.data(), S2.d_cnt, n2 * 4, hipMemcpyDeviceToHost, h.stream));
      HIPCHK(hipMemcpyAsync(r2_ok.data(), S2.d_ok, n2 * 4, hipMemcpyDeviceToHost, h.stream));
      HSYNC(h);
      h.stat_sketch += (int64_t)n2;
      for (size_t q = 0; q < n2; ++q) {
        if (r2_ok[q] > 0) {
          cnt[r2_ids[q]] = c2[q];
          --h.stat_sketch_rejected;  // recovered by the wider sketch
        } else {
          fb.push_back(etasks[r2_ids[q]]);
          fb_of.push_back(-1 - (int32_t)q);  // marks a second-round task
        }
      }
    }
    if (!fb.empty()) {
      H2D(h, d_fbT, fb.data(), fb.size() * sizeof(EigTask));
      {
        ProfScope ps(h, "k_eig_values", 0, 0);
        if ((rc = eig_values(h, fb, d_fbT, eps2, d_cfb, h.stream, err))) return rc;
      }
      std::vector<int32_t> cfb(fb.size());
      HSYNC(h);
      HIPCHK(hipMemcpyAsync(cfb.data(), d_cfb, fb.size() * 4, hipMemcpyDeviceToHost, h.stream));
      HSYNC(h);
      for (size_t a = 0; a < fb.size(); ++a) cnt[fb_of[a] >= 0 ? sk_ids[fb_of[a]] : r2_ids[-1 - fb_of[a]]] = cfb[a];
    }
    // the full-path task list now holds every non-accepted task
    for (size_t a = 0; a < fb.size(); ++a) {
      full_ids.push_back(fb_of[a] >= 0 ? sk_ids[fb_of[a]] : r2_ids[-1 - fb_of[a]]);
      fullT.push_back(fb[a]);
    }
    h.stat_full += (int64_t)full_ids.size();  // every decomposition that was not a sketch in the end
    for (int e : sk_ids) h.stat_sketch_cols += skw[e];
    std::vector<int32_t> keep_ids;
    std::vector<EigTask> keepE;
    std::vector<SkTask> keepT;
    for (size_t a = 0; a < nsk; ++a)
      if (ok_sk[a] > 0) {
        keep_ids.push_back(sk_ids[a]);
        keepE.push_back(skE[a]);
        keepT.push_back(skT[a]);
      }
    for (size_t q = 0; q < r2_ids.size(); ++q)
      if (r2_ok[q] > 0) {
        keep_ids.push_back(r2_ids[q]);
        keepE.push_back(S2.E[q]);
        keepT.push_back(S2.T[q]);
      }
    sk_ids.swap(keep_ids);
    skE.swap(keepE);
    skT.swap(keepT);
  } else {
    HIPCHK(hipGetLastError());
    HSYNC(h);
    HIPCHK(hipMemcpyAsync(info.data(), d_info, nrec * 4, hipMemcpyDeviceToHost, h.stream));
    HSYNC(h);
  }
  prof_collect(h);
  return 0;
}

// New ranks, eigenvectors of the accepted decompositions, new bases.
static int colour_ranks_vectors(Handle& h, ColourWork& W, HostLap& lap, std::string& err) {
  const int l = W.l, c = W.c, nrec = W.nrec, sides = W.sides;
  const bool sym = W.sym;
  DevLevel& L = h.lv[l];
  auto& recs = W.recs;
  auto& chg = W.chg;
  auto& d_chg = W.d_chg;
  auto& V = W.V;
  auto& nchg = W.nchg;
  auto& fl_evec = W.fl_evec;
  auto& cnt = W.cnt;
  auto& info = W.info;
  auto& full_ids = W.full_ids;
  auto& sk_ids = W.sk_ids;
  auto& fullT = W.fullT;
  auto& skE = W.skE;
  auto& skT = W.skT;
  auto& rfeat = W.rfeat;
  auto& fe_ids = W.fe_ids;
  int rc = 0;
  for (int k = 0; k < nrec; ++k)
    if (info[k]) {
      err = "singular pivot block at level " + std::to_string(l) + ", node " + std::to_string(recs[k].node);
      return -4;
    }
  if (nchg) {
    int64_t iw = 0;
    for (int k = 0; k < nchg; ++k) {
      Changed& C = chg[k];
      int rn = sym ? cnt[k] : std::max(cnt[2 * k], cnt[2 * k + 1]);
      rn = std::min(rn, std::min(C.n, L.rc[C.p]));
      C.rnew = rn;
    }
    if (h.record_ranks)
      for (size_t a = 0; a < fe_ids.size(); ++a) {
        const Changed& C = chg[fe_ids[a]];
        h.rec_X.insert(h.rec_X.end(), rfeat.begin() + a * RANK_NF, rfeat.begin() + (a + 1) * RANK_NF);
        h.rec_t.push_back((float)C.rnew / (float)C.n);
      }
    // every accepted sketch can supply rn vectors: rn <= max count < s on both sides
    for (size_t a = 0; a < sk_ids.size(); ++a) {
      const Changed& C = chg[sk_ids[a] / sides];
      if (C.rnew >= skT[a].s) {
        err = "sketch narrower than the selected rank";
        return -6;
      }
    }
    for (int e : full_ids) iw += 5LL * chg[e / sides].n * chg[e / sides].rnew + 32;
    for (size_t a = 0; a < sk_ids.size(); ++a) iw += 5LL * skT[a].s * chg[sk_ids[a] / sides].rnew + 32;
    if ((rc = ensure(h, (void**)&h.scratch2, &h.scratch2_bytes, iw * 8 + 64, err))) return rc;
    iw = 0;
    for (size_t a = 0; a < full_ids.size(); ++a) {
      const Changed& C = chg[full_ids[a] / sides];
      fullT[a].k = C.rnew;
      fullT[a].IW = h.scratch2 + iw;
      iw += 5LL * C.n * C.rnew + 32;
    }
    for (size_t a = 0; a < sk_ids.size(); ++a) {
      const Changed& C = chg[sk_ids[a] / sides];
      skE[a].k = C.rnew;
      skE[a].IW = h.scratch2 + iw;
      iw += 5LL * skT[a].s * C.rnew + 32;
    }
    const size_t nf2 = fullT.size(), ns2 = sk_ids.size();
    std::vector<GemmTask> vT;
    for (size_t a = 0; a < ns2; ++a) {
      const int e = sk_ids[a];
      const Changed& C = chg[e / sides];
      double* Vout = (e % sides) ? C.vt : C.vs;
      vT.push_back({skT[a].Y, skE[a].V, Vout, C.n, C.rnew, skT[a].s, C.n, skT[a].s, C.n, 0, 0, 1.0, 0.0});
    }
    const size_t need_tab = (nf2 + ns2) * sizeof(EigTask) + ns2 * sizeof(GemmTask) + 1024;
    if ((rc = ensure(h, (void**)&h.meta2b, &h.meta2b_bytes, (int64_t)need_tab, err))) return rc;
    EigTask* d_vf = (EigTask*)h.meta2b;
    EigTask* d_vs = d_vf + nf2;
    GemmTask* d_vg = (GemmTask*)(d_vs + ns2);
    // uploads the host does not wait for (the sources are held)
    if (nf2) H2D(h, d_vf, held(h, fullT), nf2 * sizeof(EigTask));
    if (ns2) {
      H2D(h, d_vs, held(h, skE), ns2 * sizeof(EigTask));
      H2D(h, d_vg, held(h, vT), ns2 * sizeof(GemmTask));
    }
    H2D(h, d_chg, held(h, chg), chg.size() * sizeof(Changed));
    for (int e : full_ids) fl_evec += 2.0 * (double)chg[e / sides].n * chg[e / sides].n * chg[e / sides].rnew;
    // eigenvectors of the full decompositions on the side stream, those of
    // the sketches on the main stream
    const bool vside = !h.eig_jacobi && nf2 && ns2;
    if (vside && (rc = fork_side(h, err))) return rc;
    if (!h.eig_jacobi && nf2) {
      ProfScope ps(h, "k_eig_vectors", fl_evec, 0, vside);
      eig_vectors(h, fullT, d_vf, vside ? h.side_stream : h.stream);
    }
    if (ns2) {
      double fl = 0;
      int rmax = 1, nmx = 1;
      for (size_t a = 0; a < ns2; ++a) {
        const Changed& C = chg[sk_ids[a] / sides];
        fl += 2.0 * (double)skT[a].s * skT[a].s * C.rnew + 2.0 * (double)C.n * skT[a].s * C.rnew;
        rmax = std::max(rmax, C.rnew);
        nmx = std::max(nmx, C.n);
      }
      ProfScope ps(h, "group:sketch_vectors", fl, 0);
      eig_vectors(h, skE, d_vs, h.stream);
      gemm_batch(h, dim3((unsigned)((nmx + 63) / 64), (unsigned)((rmax + 63) / 64), (unsigned)ns2), vT.data(), ns2,
                 d_vg, h.stream);
    }
    if (vside && (rc = join_side(h, err))) return rc;
    lap.mark("plan_vectors");
    {
      ProfScope ps(h, "k_basis", 0, 0);
      hipLaunchKernelGGL(k_basis, dim3(nchg), dim3(NT), 0, h.stream, V, d_chg);
    }
    if ((rc = check_arena(h, l, "basis", c, err))) return rc;
  }
  return 0;
}

// Capacity growth of the M2L blocks of nodes whose new rank exceeds it, and
// the projection of the far fill-in onto the new bases.
static int colour_grow_project(Handle& h, ColourWork& W, std::string& err) {
  const int l = W.l, c = W.c;
  DevLevel& L = h.lv[l];
  auto& far = W.far;
  auto& chg = W.chg;
  auto& d_recs = W.d_recs;
  auto& d_nbrs = W.d_nbrs;
  auto& d_far = W.d_far;
  auto& d_chg = W.d_chg;
  auto& V = W.V;
  auto& nchg = W.nchg;
  auto& moves = W.moves;
  auto& capset = W.capset;
  int rc = 0;
  // capacity growth of the M2L blocks of nodes whose new rank exceeds it
  if (nchg) {
    const Level& TL = h.tree.levels[l];
    std::vector<int32_t> newcap(chg.size(), 0);
    std::vector<char> grown_mark;
    bool any = false;
    for (size_t k = 0; k < chg.size(); ++k) {
      const int p = chg[k].p;
      if (chg[k].rnew > L.ilcap[p]) {
        newcap[k] = h.il_tight ? chg[k].rnew
                               : std::min(L.rc[p], std::max(chg[k].rnew, L.ilcap[p] + L.ilcap[p] / 2 + 8));
        any = true;
      }
    }
    if (any) {
      std::vector<int32_t> cap_now(L.ilcap);  // capacities after growth
      for (size_t k = 0; k < chg.size(); ++k)
        if (newcap[k]) cap_now[chg[k].p] = newcap[k];
      for (size_t k = 0; k < chg.size(); ++k) {
        if (!newcap[k]) continue;
        const int p = chg[k].p;
        for (int s2 = TL.il_ptr[p]; s2 < TL.il_ptr[p + 1]; ++s2) {
          const int lq = TL.il[s2];
          double* ptr = nullptr;
          if ((rc = il_take(h, L, (int64_t)cap_now[p] * cap_now[lq], &ptr, err))) return rc;
          moves.push_back({s2, 0, ptr});
          L.il_blk[s2] = ptr;
          if (cap_now[lq] == L.ilcap[lq]) {  // l keeps its capacity: move its column block too
            int lo = TL.il_ptr[lq], hi = TL.il_ptr[lq + 1] - 1, f = -1;
            while (lo <= hi) {
              const int mid = (lo + hi) >> 1;
              if (TL.il[mid] == p) { f = mid; break; }
              if (TL.il[mid] < p) lo = mid + 1; else hi = mid - 1;
            }
            double* ptr2 = nullptr;
            if ((rc = il_take(h, L, (int64_t)cap_now[lq] * cap_now[p], &ptr2, err))) return rc;
            moves.push_back({f, 0, ptr2});
            L.il_blk[f] = ptr2;
          }
        }
      }
      for (size_t k = 0; k < chg.size(); ++k)
        if (newcap[k]) {
          capset.push_back(chg[k].p);
          capset.push_back(newcap[k]);
        }
      const int64_t need = (int64_t)(moves.size() * sizeof(SlotMove) + capset.size() * 4 + 512);
      if ((rc = ensure(h, (void**)&h.meta2, &h.meta2_bytes, need, err))) return rc;
      SlotMove* d_mv = (SlotMove*)h.meta2;
      int32_t* d_cs = (int32_t*)(h.meta2 + ((moves.size() * sizeof(SlotMove) + 255) & ~(size_t)255));
      H2D(h, d_mv, held(h, moves), moves.size() * sizeof(SlotMove));
      H2D(h, d_cs, held(h, capset), capset.size() * 4);
      const int nm = (int)moves.size(), nc2 = (int)capset.size() / 2;
      hipLaunchKernelGGL(k_slot_moves, dim3((nm + NT - 1) / NT), dim3(NT), 0, h.stream, L.d_il_blk, d_mv, nm);
      hipLaunchKernelGGL(k_set_caps, dim3((nc2 + NT - 1) / NT), dim3(NT), 0, h.stream, L.d_ilcap, d_cs, nc2);
      for (size_t k = 0; k < chg.size(); ++k)
        if (newcap[k]) L.ilcap[chg[k].p] = newcap[k];
      h.stat_grown += nc2;
    }
  }
  if (!far.empty()) {
    ProfScope ps(h, "k_project", 0, 0);
    hipLaunchKernelGGL(k_project, dim3((unsigned)far.size()), dim3(NT), 0, h.stream, V, d_far, d_recs, d_nbrs, d_chg);
  }
  if ((rc = check_arena(h, l, "project", c, err))) return rc;
  return 0;
}

// Phase B: basis changes of the M2L / M2M / L2L blocks touching a changed node.
static int colour_phase_b(Handle& h, ColourWork& W, std::string& err) {
  const int l = W.l, c = W.c, K = h.K;
  DevLevel& L = h.lv[l];
  auto& chg = W.chg;
  auto& d_far = W.d_far;
  auto& d_chg = W.d_chg;
  auto& d_refs = W.d_refs;
  auto& V = W.V;
  auto& nchg = W.nchg;
  auto& moves = W.moves;
  auto& capset = W.capset;
  int rc = 0;
  // ---- phase B
  if (nchg) {
    {
      double fl_b = 0;
      for (const Changed& C : chg) {
        const Level& TL = h.tree.levels[l];
        const double nil = TL.il_ptr[C.p + 1] - TL.il_ptr[C.p];
        fl_b += 2.0 * nil * 2.0 * (double)C.r * C.rnew * std::max(C.r, C.rnew) + 4.0 * K * C.r * C.rnew;
      }
      ProfScope ps(h, "group:phase_b", fl_b, 0);
      int rmax = 0;
      for (const Changed& C : chg) rmax = std::max(rmax, std::max(C.r, C.rnew));
      // wave form: every block a single 32 x 32 tile (all ranks involved <= 32),
      // so each wave reads a block completely before it overwrites it in place
      int rlev = 0;
      if (h.precision == 1 && h.pb_wave && rmax <= 32)
        for (int32_t rv : L.r) rlev = std::max(rlev, rv);
      if (h.precision == 1 && h.pb_wave && rmax <= 32 && rlev <= 32) {
        hipLaunchKernelGGL(k_phase_b_wave, dim3(nchg), dim3(NT), 0, h.stream, V, K, d_chg, d_refs, d_far,
                           l > 2 ? 1 : 0, L.d_il_blk_old, L.d_ilcap_old);
      } else if (rmax <= 48) {  // one workgroup per changed node
        if (h.precision == 1)
          hipLaunchKernelGGL(k_phase_b<true>, dim3(nchg), dim3(NT), 0, h.stream, V, K, d_chg, d_refs, d_far,
                             l > 2 ? 1 : 0, L.d_il_blk_old, L.d_ilcap_old);
        else
          hipLaunchKernelGGL(k_phase_b<false>, dim3(nchg), dim3(NT), 0, h.stream, V, K, d_chg, d_refs, d_far,
                             l > 2 ? 1 : 0, L.d_il_blk_old, L.d_ilcap_old);
      } else {
      // one task per transformed block, each with its own temporary; launched
      // in chunks whose temporaries fit a bounded buffer
      const Level& TL = h.tree.levels[l];
      std::vector<int32_t> chg_of(TL.n, -1);
      for (int k = 0; k < nchg; ++k) chg_of[chg[k].p] = k;
      // task table built on worker threads over changed-node ranges, joined in order
      const int nparts = std::max(1, std::min(host_threads(), nchg / 32));
      std::vector<std::vector<PBTask>> pbp(nparts);
      std::vector<std::vector<int64_t>> pbszp(nparts);
      std::vector<char> pbbad(nparts, 0);
      parallel_chunks(nchg, nparts, [&](int pc, int k0, int k1) {
        std::vector<PBTask>& pb = pbp[pc];
        std::vector<int64_t>& pbsz = pbszp[pc];
        for (int k = k0; k < k1; ++k) {
          const Changed& C = chg[k];
          const int p = C.p;
          for (int s2 = TL.il_ptr[p]; s2 < TL.il_ptr[p + 1]; ++s2) {
            const int lq = TL.il[s2];
            const int lc = chg_of[lq];
            const int rln = lc >= 0 ? chg[lc].rnew : L.r[lq];
            pb.push_back({k, s2, 0, 0, nullptr});
            pbsz.push_back((int64_t)std::max(C.r, 1) * std::max(rln, 1));
            if (lc < 0) {
              int lo = TL.il_ptr[lq], hi = TL.il_ptr[lq + 1] - 1, f = -1;
              while (lo <= hi) {
                const int mid = (lo + hi) >> 1;
                if (TL.il[mid] == p) { f = mid; break; }
                if (TL.il[mid] < p) lo = mid + 1; else hi = mid - 1;
              }
              if (f < 0) {
                pbbad[pc] = 1;
                return;
              }
              pb.push_back({k, f, 1, lq, nullptr});
              pbsz.push_back((int64_t)std::max(L.r[lq], 1) * std::max(C.rnew, 1));
            }
          }
          if (l > 2) {
            pb.push_back({k, 0, 2, 0, nullptr});
            pbsz.push_back((int64_t)K * std::max(C.rnew, 1) + (int64_t)std::max(C.rnew, 1) * K);
          }
        }
      });
      std::vector<PBTask> pb;
      std::vector<int64_t> pbsz;
      {
        size_t tot = 0;
        for (int pc = 0; pc < nparts; ++pc) {
          if (pbbad[pc]) {
            err = "interaction lists not symmetric";
            return -6;
          }
          tot += pbp[pc].size();
        }
        pb.reserve(tot);
        pbsz.reserve(tot);
        for (int pc = 0; pc < nparts; ++pc) {
          pb.insert(pb.end(), pbp[pc].begin(), pbp[pc].end());
          pbsz.insert(pbsz.end(), pbszp[pc].begin(), pbszp[pc].end());
        }
      }
      const int64_t budget = (int64_t)256 << 20;  // doubles (2 GiB)
      size_t b0 = 0;
      while (b0 < pb.size()) {
        int64_t used = 0;
        size_t b1 = b0;
        while (b1 < pb.size() && (b1 == b0 || used + ((pbsz[b1] + 31) & ~31LL) <= budget)) {
          used += (pbsz[b1] + 31) & ~31LL;
          ++b1;
        }
        const int64_t tbytes = (int64_t)((b1 - b0) * sizeof(PBTask) + 255) & ~255LL;
        if ((rc = ensure(h, (void**)&h.scratch2, &h.scratch2_bytes, used * 8 + tbytes + 256, err))) return rc;
        double* T0 = (double*)((char*)h.scratch2 + tbytes);
        int64_t o = 0;
        for (size_t b = b0; b < b1; ++b) {
          pb[b].t = T0 + o;
          o += (pbsz[b] + 31) & ~31LL;
        }
        const bool last = b1 == pb.size();
        H2D(h, h.scratch2, last ? held(h, pb) + b0 : pb.data() + b0, (b1 - b0) * sizeof(PBTask));
        if (h.precision == 1)
          hipLaunchKernelGGL(k_phase_b_blocks<true>, dim3((unsigned)(b1 - b0)), dim3(NT), 0, h.stream, V, K, d_chg,
                             d_refs, d_far, (const PBTask*)h.scratch2, L.d_il_blk_old, L.d_ilcap_old);
        else
          hipLaunchKernelGGL(k_phase_b_blocks<false>, dim3((unsigned)(b1 - b0)), dim3(NT), 0, h.stream, V, K, d_chg,
                             d_refs, d_far, (const PBTask*)h.scratch2, L.d_il_blk_old, L.d_ilcap_old);
        b0 = b1;
        if (!last) HSYNC(h);  // the next chunk reuses the task table and buffer
      }
      }
    }
    if (!moves.empty()) {  // old tables follow the new ones again
      SlotMove* d_mv = (SlotMove*)h.meta2;
      int32_t* d_cs = (int32_t*)(h.meta2 + ((moves.size() * sizeof(SlotMove) + 255) & ~(size_t)255));
      const int nm = (int)moves.size(), nc2 = (int)capset.size() / 2;
      hipLaunchKernelGGL(k_slot_moves, dim3((nm + NT - 1) / NT), dim3(NT), 0, h.stream, L.d_il_blk_old, d_mv, nm);
      hipLaunchKernelGGL(k_set_caps, dim3((nc2 + NT - 1) / NT), dim3(NT), 0, h.stream, L.d_ilcap_old, d_cs, nc2);
    }
    if ((rc = check_arena(h, l, "phase_b", c, err))) return rc;
    hipLaunchKernelGGL(k_set_rank, dim3((nchg + NT - 1) / NT), dim3(NT), 0, h.stream, L.d_r, d_chg, nchg);
    hipLaunchKernelGGL(k_set_chg, dim3((nchg + NT - 1) / NT), dim3(NT), 0, h.stream, L.d_chg, d_chg, nchg, 1);
    for (const Changed& C : chg) L.r[C.p] = C.rnew;
  }
  HIPCHK(hipGetLastError());
  return 0;
}

// Keeps the records for the solve (neighbour entries rebased on the level
// table) and its 64-row tiles: pivot rows, L rows, G rows.
static int colour_keep(Handle& h, ColourWork& W, std::string& err) {
  const int l = W.l;
  DevLevel& L = h.lv[l];
  auto& recs = W.recs;
  auto& nbrs = W.nbrs;
  auto& far = W.far;
  auto& nchg = W.nchg;
  const int nbase = W.nbase;
  // keep the records for the solve (neighbour entries rebased on the level
  // table) and its 64-row tiles: pivot rows, L rows, G rows
  for (ElimRec R : recs) {
    R.nb_begin += nbase;
    R.X = nullptr;
    const int32_t ri = (int32_t)L.recs.size();
    for (int r0 = 0; r0 < R.d; r0 += 64) L.st_w.push_back({ri, r0, 0, INT32_MAX, -1});
    for (int r0 = 0; r0 < R.M; r0 += 64) L.st_u.push_back({ri, r0, 0, INT32_MAX, -1});
    L.recs.push_back(R);
  }
  // backward step: a colour of few row tiles (the upper levels) splits each
  // tile's inner dimension (64-column chunks over the neighbours' G blocks,
  // then E_tb) over several tasks, up to about 1024 tasks in all and at least
  // 8 chunks per task; their partial sums are added in order by a second
  // kernel, so the result does not depend on the split's timing
  {
    const int rb = (int)L.recs.size() - (int)recs.size();
    int ntile = 0;
    for (const ElimRec& R : recs) ntile += (R.n + 63) / 64;
    int32_t slots = 0;
    for (int k = 0; k < (int)recs.size(); ++k) {
      const ElimRec& R = recs[k];
      int G = (R.r + 63) / 64;
      for (int q = 0; q < R.nnb; ++q) G += (nbrs[R.nb_begin + q].m + 63) / 64;
      int ns = 1;
      if (h.solve_split && ntile > 0 && ntile < 512) ns = std::max(1, std::min((1024 + ntile - 1) / ntile, G / 8));
      for (int r0 = 0; r0 < R.n; r0 += 64) {
        if (ns == 1) {
          L.st_b.push_back({rb + k, r0, 0, INT32_MAX, -1});
          continue;
        }
        L.sg.push_back({rb + k, r0, slots, ns});
        for (int s = 0; s < ns; ++s)
          L.st_b.push_back({rb + k, r0, (int32_t)((int64_t)G * s / ns), (int32_t)((int64_t)G * (s + 1) / ns), slots + s});
        slots += ns;
      }
    }
    L.part_slots = std::max(L.part_slots, slots);
  }
  L.stw_ptr.push_back((int32_t)L.st_w.size());
  L.stu_ptr.push_back((int32_t)L.st_u.size());
  L.stb_ptr.push_back((int32_t)L.st_b.size());
  L.sg_ptr.push_back((int32_t)L.sg.size());
  L.nbrs.insert(L.nbrs.end(), nbrs.begin(), nbrs.end());
  L.col_ptr.push_back((int32_t)L.recs.size());
  ColourInv ci;
  for (const ElimRec& R : recs)
    if (R.inv) {
      ++ci.count;
      ci.dmax = std::max(ci.dmax, R.d);
      ci.nmax = std::max(ci.nmax, R.n);
      ci.Mmax = std::max(ci.Mmax, R.M);
    }
  L.cinv.push_back(ci);
  h.stat_far += (int64_t)far.size();
  h.stat_changed += nchg;
  return 0;
}

static int eliminate_colour(Handle& h, int l, int c, std::string& err) {
  const Level& T = h.tree.levels[l];
  ColourWork W;
  W.l = l;
  W.c = c;
  W.g0 = T.grp_ptr[c];
  W.nrec = T.grp_ptr[c + 1] - W.g0;
  if (W.nrec == 0) return 0;
  W.sym = h.symmetric;
  W.sides = W.sym ? 1 : 2;
  W.nbase = (int)h.lv[l].nbrs.size();
  HostLap lap(h);
  int rc;
  if ((rc = colour_tables(h, W, err))) return rc;
  lap.mark("tables");
  if ((rc = colour_upload(h, W, err))) return rc;
  lap.mark("pack");
  if ((rc = colour_phase_a(h, W, err))) return rc;
  lap.mark("launch_a");
  if ((rc = colour_recompress(h, W, lap, err))) return rc;
  lap.mark("select");
  if ((rc = colour_ranks_vectors(h, W, lap, err))) return rc;
  if ((rc = colour_grow_project(h, W, err))) return rc;
  lap.mark("moves_project");
  if ((rc = colour_phase_b(h, W, err))) return rc;
  lap.mark("phase_b");
  if ((rc = colour_keep(h, W, err))) return rc;
  lap.mark("keep");
  // no wait here: the host goes on to the next colour's tables while the
  // device finishes this one (pending uploads read held copies)
  return 0;
}

// ------------------------------------------------------------------ factor
static int init_leaf_level(Handle& h, std::string& err) {
  const int l = h.tree.depth;
  const Level& T = h.tree.levels[l];
  DevLevel& L = h.lv[l];
  L.n.resize(T.n);
  for (int32_t i = 0; i < T.n; ++i) L.n[i] = (int32_t)(T.pt_end[i] - T.pt_begin[i]);
  int rc;
  if ((rc = setup_level(h, l, err))) return rc;
  LevelView V = view_of(L);
  const double side = 2.0 * h.tree.H / (double)(1LL << l);
  hipLaunchKernelGGL(k_leaf_cheb, dim3(T.n), dim3(NT), 0, h.stream, V, h.nc, h.d_pts, h.d_w, h.d_pt_begin, h.d_lo,
                     side);
  hipLaunchKernelGGL(k_p2p, dim3((unsigned)L.near_idx.size()), dim3(NT), 0, h.stream, V, L.d_slot_row, h.d_pts, h.d_w,
                     h.d_diag, h.d_pt_begin);
  HIPCHK(hipGetLastError());
  if ((rc = check_arena(h, l, "leaf operators", -1, err))) return rc;
  if ((rc = reduce_level(h, l, err))) return rc;
  return check_arena(h, l, "rank reduction", -1, err);
}

static int aggregate_level(Handle& h, int l, std::string& err) {
  // level l (eliminated) -> level l - 1
  const Level& C = h.tree.levels[l - 1];
  DevLevel& F = h.lv[l];
  DevLevel& P = h.lv[l - 1];
  P.n.assign(C.n, 0);
  for (int32_t q = 0; q < C.n; ++q)
    for (int s = C.child_ptr[q]; s < C.child_ptr[q + 1]; ++s) P.n[q] += F.r[C.child[s]];
  int rc;
  if ((rc = setup_level(h, l - 1, err))) return rc;
  LevelView VC = view_of(P), VF = view_of(F);
  hipLaunchKernelGGL(k_agg_cheb, dim3(C.n), dim3(NT), 0, h.stream, VC, VF, h.K, P.d_child_ptr, P.d_child);
  hipLaunchKernelGGL(k_agg_near, dim3((unsigned)P.near_idx.size()), dim3(NT), 0, h.stream, VC, VF, P.d_slot_row,
                     P.d_child_ptr, P.d_child);
  HIPCHK(hipGetLastError());
  HSYNC(h);
  if ((rc = check_arena(h, l - 1, "aggregation", -1, err))) return rc;
  release_level_work(h, l);
  if ((rc = reduce_level(h, l - 1, err))) return rc;
  return check_arena(h, l - 1, "rank reduction", -1, err);
}

static int finish_level(Handle& h, int l, std::string& err) {
  DevLevel& L = h.lv[l];
  int rc;
  dfree(h, L.d_recs);
  dfree(h, L.d_nbrs);
  L.d_recs = nullptr;
  L.d_nbrs = nullptr;
  if ((rc = upload(h, &L.d_recs, L.recs, err))) return rc;
  if ((rc = upload(h, &L.d_nbrs, L.nbrs, err))) return rc;
  dfree(h, L.d_st);
  L.d_st = nullptr;
  {
    std::vector<STask> all;
    all.reserve(L.st_w.size() + L.st_u.size() + L.st_b.size());
    all.insert(all.end(), L.st_w.begin(), L.st_w.end());
    all.insert(all.end(), L.st_u.begin(), L.st_u.end());
    all.insert(all.end(), L.st_b.begin(), L.st_b.end());
    if ((rc = upload(h, &L.d_st, all, err))) return rc;
  }
  dfree(h, L.d_sg);
  L.d_sg = nullptr;
  if (!L.sg.empty() && (rc = upload(h, &L.d_sg, L.sg, err))) return rc;
  // solve-vector offsets
  L.vx_off.resize(L.nn);
  L.vz_off.resize(L.nn);
  int64_t ox = 0, oz = 0;
  for (int32_t i = 0; i < L.nn; ++i) {
    L.vx_off[i] = ox;
    ox += L.n[i];
    L.vz_off[i] = oz;
    oz += L.r[i];
  }
  L.vx_total = ox;
  L.vz_total = oz;
  dfree(h, L.d_vx_off);
  dfree(h, L.d_vz_off);
  if ((rc = upload(h, &L.d_vx_off, L.vx_off, err))) return rc;
  if ((rc = upload(h, &L.d_vz_off, L.vz_off, err))) return rc;
  H2D(h, L.d_r, L.r.data(), L.nn * 4);
  return 0;
}

static void release_graph(Handle& h);
static void clear_factor(Handle& h) {
  release_graph(h);
  for (size_t l = 0; l < h.lv.size(); ++l) {
    release_level_work(h, (int)l);
    DevLevel& L = h.lv[l];
    void* ptrs[] = {L.d_recs, L.d_nbrs, L.d_vx_off, L.d_vz_off, L.d_n, L.d_r, L.d_parent, L.d_child_ptr, L.d_child,
                    L.d_st, L.d_sg};
    for (void* p : ptrs) dfree(h, p);
    L = DevLevel();
  }
  for (double* p : h.store_chunks) dfree(h, p);
  h.store_chunks.clear();
  h.store_used.clear();
  for (float* p : h.store32_chunks) dfree(h, (double*)p);
  h.store32_chunks.clear();
  h.store32_used.clear();
  h.store32_cur = nullptr;
  h.store32_left = 0;
  h.store_cur = nullptr;
  h.store_left = 0;
  h.store_bytes = 0;
  dfree(h, h.d_top);
  dfree(h, h.d_top_piv);
  dfree(h, h.d_top_inv);
  h.d_top = nullptr;
  h.d_top_piv = nullptr;
  h.d_top_inv = nullptr;
  h.factored = false;
}

int factor(Handle& h, std::string& err) {
  int rc;
  if (!h.dev_ready && (rc = device_init(h, err))) return rc;
  if (!h.d_model && !h.model_host.empty()) {  // the network named by options.rank_model
    HIPCHK(hipMalloc((void**)&h.d_model, h.model_host.size() * 4));
    HIPCHK(hipMemcpy(h.d_model, h.model_host.data(), h.model_host.size() * 4, hipMemcpyHostToDevice));
  }
  HIPCHK(hipSetDevice(h.device));
  clear_factor(h);
  h.lv.assign((size_t)h.tree.depth + 1, DevLevel());
  h.log = std::getenv("IFMM_LOG") != nullptr;
  h.poison = std::getenv("IFMM_POISON") != nullptr;
  h.check = std::getenv("IFMM_CHECK") != nullptr;
  {
    const char* ev = std::getenv("IFMM_EIG");
    h.eig_jacobi = ev && std::strcmp(ev, "jacobi") == 0;
  }
  h.prof = std::getenv("IFMM_PROF") != nullptr;
  h.il_tight = std::getenv("IFMM_IL_TIGHT") != nullptr;
  if (const char* e = std::getenv("IFMM_GRAPH")) h.graph_solve = std::atoi(e) != 0;
  if (const char* e = std::getenv("IFMM_BIG_D")) h.big_d = std::max(1, std::atoi(e));
  if (const char* e = std::getenv("IFMM_SKETCH")) h.sketch = std::atoi(e) != 0;
  if (const char* e = std::getenv("IFMM_PB_WAVE")) h.pb_wave = std::atoi(e) != 0;
  if (const char* e = std::getenv("IFMM_DEEP_N")) h.deep_n = std::max(1, std::atoi(e));
  if (const char* e = std::getenv("IFMM_F64_MFMA")) h.f64_mfma = std::atoi(e) != 0;
  tune_load(h);
  if (const char* e = std::getenv("IFMM_SOLVE_SPLIT")) h.solve_split = std::atoi(e) != 0;
  if (const char* e = std::getenv("IFMM_SCHUR_SPLIT")) h.schur_split = std::atoi(e) != 0;
  if (const char* e = std::getenv("IFMM_TRD_BIG")) h.trd_big = std::max(3, std::atoi(e));
  // IFMM_SOLVE32=1 (mixed form): the solve reads FP32 copies of L and G.  It
  // halves the store but ran slower than the FP64 blocks (the conversions
  // sit in the column loop), so it is off by default
  h.solve32 = false;
  if (const char* e = std::getenv("IFMM_SOLVE32")) h.solve32 = h.precision == 1 && std::atoi(e) != 0;
  h.prof_level = std::getenv("IFMM_PROF_LEVEL") != nullptr;
  if (const char* e = std::getenv("IFMM_SKETCH_MIN")) h.sketch_min = std::max(1, std::atoi(e));
  h.stat_sketch = h.stat_sketch_rejected = h.stat_sketch_narrow = 0;
  h.stat_full = h.stat_sketch_cols = 0;
  h.t_sync = 0;
  h.t_h2d = 0;
  h.rec_X.clear();
  h.rec_t.clear();
  h.stat_predicted = 0;
  h.kstat.clear();
  h.host_ms.clear();
  h.aux.clear();
  h.stat_far = 0;
  h.stat_changed = 0;
  h.stat_grown = 0;
  const double t0 = now_s();
  h.t_level_setup.assign((size_t)h.tree.depth + 1, 0.0);
  h.t_level_elim.assign((size_t)h.tree.depth + 1, 0.0);
  double ta = now_s();
  {
    HostLap lp(h);
    if ((rc = init_leaf_level(h, err))) return rc;
    lp.mark("level_setup");
  }
  h.t_level_setup[h.tree.depth] = now_s() - ta;
  for (int l = h.tree.depth; l >= 2; --l) {
    const Level& T = h.tree.levels[l];
    DevLevel& L = h.lv[l];
    L.col_ptr.assign(1, 0);
    L.cinv.clear();
    L.st_w.clear(); L.st_u.clear(); L.st_b.clear();
    L.stw_ptr.assign(1, 0); L.stu_ptr.assign(1, 0); L.stb_ptr.assign(1, 0);
    L.sg.clear();
    L.sg_ptr.assign(1, 0);
    L.part_slots = 0;
    ta = now_s();
    h.cur_level = l;
    for (int c = 0; c < T.ncolour; ++c)
      if ((rc = eliminate_colour(h, l, c, err))) return rc;
    HSYNC(h);
    prof_collect(h);
    tune_collect(h);
    {
      HostLap lp(h);
      if ((rc = finish_level(h, l, err))) return rc;
      lp.mark("finish_level");
    }
    h.t_level_elim[l] = now_s() - ta;
    if (h.log)
      std::fprintf(stderr, "[ifmm] level %d: %d nodes, %d colours eliminated in %.3f s (set-up %.3f s)\n", l, T.n,
                   T.ncolour, h.t_level_elim[l], h.t_level_setup[l]);
    ta = now_s();
    {
      HostLap lp(h);
      if (l > 2 && (rc = aggregate_level(h, l, err))) return rc;
      lp.mark("level_setup");
    }
    if (l > 2) h.t_level_setup[l - 1] = now_s() - ta;
  }
  h.cur_level = 0;
  ta = now_s();
  // top: dense LU of the level-2 system
  DevLevel& L2 = h.lv[2];
  h.top_off.assign(L2.nn + 1, 0);
  for (int32_t P = 0; P < L2.nn; ++P) h.top_off[P + 1] = h.top_off[P] + L2.r[P];
  h.top_n = (int32_t)h.top_off[L2.nn];
  if ((rc = dalloc(h, &h.d_top, std::max<int64_t>((int64_t)h.top_n * h.top_n, 1), err))) return rc;
  if ((rc = dalloc(h, &h.d_top_piv, std::max(h.top_n, 1), err))) return rc;
  int64_t* d_toff = nullptr;
  if ((rc = upload(h, &d_toff, h.top_off, err))) return rc;
  HIPCHK(hipMemsetAsync(h.d_top, 0, (size_t)std::max<int64_t>((int64_t)h.top_n * h.top_n, 1) * 8, h.stream));
  LevelView V2 = view_of(L2);
  int32_t* d_info = nullptr;
  if ((rc = dalloc(h, &d_info, 1, err))) return rc;
  if (h.top_n > 0) {
    const int n = h.top_n;
    HIPCHK(hipMemsetAsync(d_info, 0, 4, h.stream));
    hipLaunchKernelGGL(k_top_assemble, dim3(L2.nn), dim3(NT), 0, h.stream, V2, L2.nn, d_toff, h.d_top, n);
    // T^-1 from the blocked LU of [T | I] (Sec. 2.3: the top system is solved
    // densely): the pivots' machinery with one task, every step one launch
    // over many workgroups; T keeps its LU factors
    if ((rc = dalloc(h, &h.d_top_inv, (int64_t)n * n, err))) return rc;
    const unsigned nt = (unsigned)((n + 63) / 64);
    hipLaunchKernelGGL(k_eye, dim3(nt, nt), dim3(NT), 0, h.stream, h.d_top_inv, n);
    double* d_dinv = nullptr;
    const int64_t nsteps = (n + BLU_NB - 1) / BLU_NB;
    if ((rc = dalloc(h, &d_dinv, nsteps * 2 * 4096, err))) return rc;
    BluTask* d_bt = nullptr;
    if ((rc = dalloc(h, &d_bt, 1, err))) return rc;
    const BluTask bt{h.d_top, h.d_top_inv, h.d_top_piv, d_info, d_dinv, n, n};
    H2D(h, d_bt, held(h, std::vector<BluTask>{bt}), sizeof(BluTask));
    enqueue_blocked_lu(d_bt, 1, n, n, h.stream);
    HIPCHK(hipGetLastError());
    HSYNC(h);
    dfree(h, d_dinv);
    dfree(h, d_bt);
  }
  HIPCHK(hipGetLastError());
  // every stored factor block and the top inverse must be finite (an overflow
  // or a NaN anywhere in the elimination reaches one of them)
  int32_t* d_nf = nullptr;
  if ((rc = dalloc(h, &d_nf, 1, err))) return rc;
  HIPCHK(hipMemsetAsync(d_nf, 0, 4, h.stream));
  for (size_t q = 0; q < h.store_chunks.size(); ++q)
    if (h.store_used[q] > 0)
      hipLaunchKernelGGL(k_check_finite, dim3(2048), dim3(NT), 0, h.stream, h.store_chunks[q], h.store_used[q], d_nf);
  for (size_t q = 0; q < h.store32_chunks.size(); ++q)
    if (h.store32_used[q] > 0)
      hipLaunchKernelGGL(k_check_finite32, dim3(2048), dim3(NT), 0, h.stream, h.store32_chunks[q], h.store32_used[q],
                         d_nf);
  if (h.top_n > 0)
    hipLaunchKernelGGL(k_check_finite, dim3(256), dim3(NT), 0, h.stream, h.d_top_inv, (int64_t)h.top_n * h.top_n,
                       d_nf);
  HIPCHK(hipGetLastError());
  int32_t info = 0, nonfinite = 0;
  if (h.top_n > 0) HIPCHK(hipMemcpyAsync(&info, d_info, 4, hipMemcpyDeviceToHost, h.stream));
  HIPCHK(hipMemcpyAsync(&nonfinite, d_nf, 4, hipMemcpyDeviceToHost, h.stream));
  HSYNC(h);
  dfree(h, d_info);
  dfree(h, d_nf);
  h.d_top_off = d_toff;
  release_level_work(h, 2);
  if (info) {
    err = "singular top-level system (column " + std::to_string(info - 1) + ")";
    return -4;
  }
  if (nonfinite) {
    err = "non-finite or overflowing value in the factorisation";
    return -5;
  }
  h.t_top = now_s() - ta;
  h.t_factor = now_s() - t0;
  h.factored = true;
  return tune_save(h, err);
}

// ------------------------------------------------------------------ solve
// Fill kernel (graph-safe replacement of a memset)
__global__ void __launch_bounds__(NT) k_zero(double* p, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < n; e += (int64_t)gridDim.x * NT) p[e] = 0.0;
}

static void release_graph(Handle& h) {
  if (h.g_exec) (void)hipGraphExecDestroy(h.g_exec);
  if (h.g_graph) (void)hipGraphDestroy(h.g_graph);
  h.g_exec = nullptr;
  h.g_graph = nullptr;
  h.g_key_k = -1;
}

// Layout of the solve's work vector for k right-hand sides: per level X, Z,
// W and tmp, then the top system's two vectors (the part up to `zeroed` is
// cleared by every solve), then staging for host vectors.
struct SolvePlan {
  std::vector<int64_t> ox, oz, ow, ot;
  int64_t otop = 0, oio = 0, total = 0;  // doubles
};
static SolvePlan solve_plan(const Handle& h, int k, int64_t ld, bool staging) {
  const int D = h.tree.depth;
  SolvePlan P;
  P.ox.assign(D + 1, 0); P.oz.assign(D + 1, 0); P.ow.assign(D + 1, 0); P.ot.assign(D + 1, 0);
  int64_t tot = 0;
  for (int l = 2; l <= D; ++l) {
    const DevLevel& L = h.lv[l];
    P.ox[l] = tot; tot += L.vx_total * k + 32;
    P.oz[l] = tot; tot += L.vz_total * k + 32;
    P.ow[l] = tot; tot += L.wv_total * k + 32;
    P.ot[l] = tot; tot += (int64_t)L.part_slots * 64 * k + 32;  // partial sums of split backward tiles
  }
  P.otop = tot;
  tot += 2 * (int64_t)std::max(h.top_n, 1) * k + 32;
  P.oio = tot;
  if (staging) tot += 2 * ld * k + 32;
  P.total = tot;
  return P;
}

// One launch of a solve step over `ntask` row tiles, one workgroup each: the
// right-hand-side chunk width SK chosen for k (1, 4 or 8 columns at a time),
// the number of waves NW that split the tile's inner dimension (64-column
// chunks) for the colour's longest inner dimension.
static int solve_waves(int inner) { return inner <= 64 ? 1 : inner <= 256 ? 4 : 8; }
#define IFMM_SOLVE_LAUNCH(KERN, T, k, nw, ntask, st, ...)                                                        \
  do {                                                                                                         \
    const dim3 g_((unsigned)(ntask));                                                                          \
    const int sk_ = (k) == 1 ? 1 : (k) <= 4 ? 4 : 8;                                                           \
    if (sk_ == 1 && (nw) == 1) hipLaunchKernelGGL((KERN<1, 1, T>), g_, dim3(64), 0, st, __VA_ARGS__);        \
    else if (sk_ == 1 && (nw) == 4) hipLaunchKernelGGL((KERN<1, 4, T>), g_, dim3(256), 0, st, __VA_ARGS__);  \
    else if (sk_ == 1) hipLaunchKernelGGL((KERN<1, 8, T>), g_, dim3(512), 0, st, __VA_ARGS__);               \
    else if (sk_ == 4 && (nw) == 1) hipLaunchKernelGGL((KERN<4, 1, T>), g_, dim3(64), 0, st, __VA_ARGS__);   \
    else if (sk_ == 4 && (nw) == 4) hipLaunchKernelGGL((KERN<4, 4, T>), g_, dim3(256), 0, st, __VA_ARGS__);  \
    else if (sk_ == 4) hipLaunchKernelGGL((KERN<4, 8, T>), g_, dim3(512), 0, st, __VA_ARGS__);               \
    else if ((nw) == 1) hipLaunchKernelGGL((KERN<8, 1, T>), g_, dim3(64), 0, st, __VA_ARGS__);               \
    else if ((nw) == 4) hipLaunchKernelGGL((KERN<8, 4, T>), g_, dim3(256), 0, st, __VA_ARGS__);              \
    else hipLaunchKernelGGL((KERN<8, 8, T>), g_, dim3(512), 0, st, __VA_ARGS__);                             \
  } while (0)

// The substitution (Alg. 2) as one stream of launches on h.stream over the
// work vector B (layout P): clears B, then up the levels (colours ascending),
// the top solve, down the levels (colours descending).  Records hipEvent
// timings only when h.prof is set.
static void enqueue_solve(Handle& h, const SolvePlan& P, double* B, const double* d_rhs, double* d_x, int k,
                          int64_t ld) {
  const int D = h.tree.depth;
  auto sv = [&](int l) {
    SolveView S;
    S.X = B + P.ox[l]; S.Z = B + P.oz[l]; S.W = B + P.ow[l]; S.part = B + P.ot[l];
    S.xo = h.lv[l].d_vx_off; S.zo = h.lv[l].d_vz_off; S.k = k;
    return S;
  };
  hipLaunchKernelGGL(k_zero, dim3(1024), dim3(NT), 0, h.stream, B, P.otop);
  const Level& TL = h.tree.levels[D];
  const double es = h.solve32 ? 4.0 : 8.0;  // bytes per stored L / G entry
  const int sk = k == 1 ? 1 : k <= 4 ? 4 : 8;
  // waves per workgroup of a step at level l: forced while tuning, else the
  // autotuner's choice, else the rule (solve_waves)
  auto waves = [&](const char* step, int l, int rule) {
    if (h.solve_nw_force) return h.solve_nw_force;
    if (!h.tune.empty()) {
      const auto it = h.tune.find(solve_key(h, step, l, sk));
      if (it != h.tune.end()) return it->second;
    }
    return rule;
  };
  // while tuning, every launch of a step is timed under its key
  auto tstart = [&](hipEvent_t* a) {
    if (h.solve_tune_var < 0) return;
    *a = take_event(h);
    (void)hipEventRecord(*a, h.stream);
  };
  auto tstop = [&](hipEvent_t a, const char* step, int l) {
    if (h.solve_tune_var < 0) return;
    hipEvent_t b = take_event(h);
    (void)hipEventRecord(b, h.stream);
    h.tune_pending.push_back({a, b, solve_key(h, step, l, sk), h.solve_tune_var, h.solve_nw_force, 1.0});
  };
  hipLaunchKernelGGL(k_perm_in, dim3(TL.n), dim3(NT), 0, h.stream, d_rhs, ld, k, h.d_perm, h.d_pt_begin, h.lv[D].d_n,
                     sv(D));
  for (int l = D; l >= 2; --l) {
    const DevLevel& L = h.lv[l];
    SolveView S = sv(l);
    h.cur_level = l;  // profiler classes keyed per level (IFMM_PROF_LEVEL)
    const STask* st_w = L.d_st;
    const STask* st_u = L.d_st + L.st_w.size();
    for (size_t c = 0; c + 1 < L.col_ptr.size(); ++c) {
      const int a = L.col_ptr[c], b = L.col_ptr[c + 1];
      if (b <= a) continue;
      double by_w = 0, by_u = 0;
      if (h.prof)
        for (int e = a; e < b; ++e) {
          const ElimRec& R = L.recs[e];
          by_w += 8.0 * ((double)R.d * R.n + k * (2.0 * R.n + R.r));
          by_u += es * R.M * R.n + 8.0 * k * (R.n + 2.0 * R.M);
        }
      const int tw0 = L.stw_ptr[c], tw1 = L.stw_ptr[c + 1], tu0 = L.stu_ptr[c], tu1 = L.stu_ptr[c + 1];
      int nmx = 0;  // inner dimension of both forward steps: n
      for (int e = a; e < b; ++e) nmx = std::max(nmx, L.recs[e].n);
      if (tw1 > tw0) {
        ProfScope ps(h, "k_solve_fwd_w", 0, by_w);
        const int nw = waves("solve_fwd_w", l, solve_waves(nmx));
        hipEvent_t a = nullptr;
        tstart(&a);
        IFMM_SOLVE_LAUNCH(k_solve_fwd_w, double, k, nw, tw1 - tw0, h.stream, L.d_recs, st_w + tw0, S);
        tstop(a, "solve_fwd_w", l);
      }
      if (tu1 > tu0) {
        ProfScope ps(h, "k_solve_fwd_upd", 0, by_u);
        const int nw = waves("solve_fwd_upd", l, solve_waves(nmx));
        hipEvent_t a = nullptr;
        tstart(&a);
        if (h.solve32)
          IFMM_SOLVE_LAUNCH(k_solve_fwd_upd, float, k, nw, tu1 - tu0, h.stream, L.d_recs, L.d_nbrs, st_u + tu0, S);
        else
          IFMM_SOLVE_LAUNCH(k_solve_fwd_upd, double, k, nw, tu1 - tu0, h.stream, L.d_recs, L.d_nbrs, st_u + tu0, S);
        tstop(a, "solve_fwd_upd", l);
      }
    }
    if (l > 2) {
      const DevLevel& Pl = h.lv[l - 1];
      hipLaunchKernelGGL(k_vec_up, dim3(Pl.nn), dim3(NT), 0, h.stream, S, sv(l - 1), Pl.d_child_ptr, Pl.d_child, L.d_r,
                         Pl.d_n);
    }
  }
  if (h.top_n > 0) {
    const int n = h.top_n;
    double* f = B + P.otop;
    double* y = f + (int64_t)n * k;
    hipLaunchKernelGGL(k_top_gather, dim3(h.lv[2].nn), dim3(NT), 0, h.stream, sv(2), h.lv[2].nn, h.lv[2].d_r,
                       h.d_top_off, f, n);
    hipLaunchKernelGGL(k_gemm_tiles, dim3((n + 63) / 64, (k + 63) / 64), dim3(NT), 0, h.stream, n, k, n, 1.0,
                       h.d_top_inv, n, f, n, 0.0, y, n);
    hipLaunchKernelGGL(k_top_scatter, dim3(h.lv[2].nn), dim3(NT), 0, h.stream, sv(2), h.lv[2].nn, h.lv[2].d_r,
                       h.d_top_off, y, n);
  }
  for (int l = 2; l <= D; ++l) {
    const DevLevel& L = h.lv[l];
    SolveView S = sv(l);
    h.cur_level = l;
    if (l > 2) {
      const DevLevel& Pl = h.lv[l - 1];
      hipLaunchKernelGGL(k_vec_down, dim3(Pl.nn), dim3(NT), 0, h.stream, S, sv(l - 1), Pl.d_child_ptr, Pl.d_child,
                         L.d_r, Pl.d_n);
    }
    const STask* st_b = L.d_st + L.st_w.size() + L.st_u.size();
    for (int c = (int)L.col_ptr.size() - 2; c >= 0; --c) {
      const int a = L.col_ptr[c], b = L.col_ptr[c + 1];
      if (b <= a) continue;
      double by = 0;
      if (h.prof)
        for (int e = a; e < b; ++e) {
          const ElimRec& R = L.recs[e];
          by += es * R.n * R.M + 8.0 * ((double)R.n * R.r + k * (2.0 * R.n + R.M + R.r));
        }
      const int tb0 = L.stb_ptr[c], tb1 = L.stb_ptr[c + 1];
      if (tb1 <= tb0) continue;
      ProfScope ps(h, "k_solve_bwd", 0, by);
      int inner = 0;
      for (int e = a; e < b; ++e) inner = std::max(inner, L.recs[e].M + L.recs[e].r);
      const int nw = waves("solve_bwd", l, solve_waves(inner));
      hipEvent_t ev = nullptr;
      tstart(&ev);
      if (h.solve32)
        IFMM_SOLVE_LAUNCH(k_solve_bwd, float, k, nw, tb1 - tb0, h.stream, L.d_recs, L.d_nbrs, st_b + tb0, S);
      else
        IFMM_SOLVE_LAUNCH(k_solve_bwd, double, k, nw, tb1 - tb0, h.stream, L.d_recs, L.d_nbrs, st_b + tb0, S);
      const int sg0 = L.sg_ptr[c], sg1 = L.sg_ptr[c + 1];
      if (sg1 > sg0)  // split tiles: x = w - the partial sums, added in order
        hipLaunchKernelGGL(k_solve_bwd_sum, dim3((unsigned)(sg1 - sg0)), dim3(NT), 0, h.stream, L.d_recs,
                           L.d_sg + sg0, S);
      tstop(ev, "solve_bwd", l);
    }
  }
  h.cur_level = 0;
  hipLaunchKernelGGL(k_perm_out, dim3(TL.n), dim3(NT), 0, h.stream, d_x, ld, k, h.d_perm, h.d_pt_begin, h.lv[D].d_n,
                     sv(D));
}

int solve(Handle& h, const double* rhs, double* x, int k, int64_t ld, int on_device, std::string& err) {
  if (!h.factored) {
    err = "ifmm_solve called before ifmm_factor";
    return -6;
  }
  HIPCHK(hipSetDevice(h.device));
  const double t0 = now_s();
  const SolvePlan P = solve_plan(h, k, ld, true);
  int rc;
  double* before = h.svec;
  if ((rc = ensure(h, (void**)&h.svec, &h.svec_bytes, P.total * 8, err))) return rc;
  if (h.svec != before) release_graph(h);  // the captured graph refers to the old buffer
  double* B = h.svec;
  const double* d_rhs = rhs;
  double* d_x = x;
  if (!on_device) {
    double* io = B + P.oio;
    H2D(h, io, rhs, (size_t)ld * k * 8);
    d_rhs = io;
    d_x = io + ld * k;
  }
  if (!h.tune_cache.empty()) {
    // autotuner: a level / step / chunk width without an entry gets one timed
    // eager solve per wave count (1, 4, 8); the real solve follows
    const int sk = k == 1 ? 1 : k <= 4 ? 4 : 8;
    const std::string done = "solve " + form_name(h) + " d" + std::to_string(h.tree.depth) + " k" + std::to_string(sk);
    if (!h.tune.count(done)) {
      const int cand[3] = {1, 4, 8};
      for (int v = 0; v < 3; ++v) {
        h.solve_nw_force = cand[v];
        h.solve_tune_var = v;
        enqueue_solve(h, P, B, d_rhs, d_x, k, ld);
      }
      h.solve_nw_force = 0;
      h.solve_tune_var = -1;
      HIPCHK(hipStreamSynchronize(h.stream));
      prof_collect(h);
      tune_collect(h);
      h.tune[done] = 1;  // tuned (levels without a launch of a step keep the rule)
      h.tune_dirty = true;
      release_graph(h);
      if ((rc = tune_save(h, err))) return rc;
    }
  }
  if (const char* e = std::getenv("IFMM_GRAPH")) h.graph_solve = std::atoi(e) != 0;
  const bool use_graph = h.graph_solve;
  if (!use_graph) {
    enqueue_solve(h, P, B, d_rhs, d_x, k, ld);
  } else {
    const bool hit = h.g_exec && h.g_key_k == k && h.g_key_ld == ld && h.g_key_rhs == d_rhs && h.g_key_x == d_x;
    if (!hit) {
      release_graph(h);
      if (!h.cap_stream) HIPCHK(hipStreamCreateWithFlags(&h.cap_stream, hipStreamNonBlocking));
      HIPCHK(hipStreamSynchronize(h.stream));
      hipStream_t keep = h.stream;
      const bool prof = h.prof;
      h.stream = h.cap_stream;
      h.prof = false;  // no timing events inside the graph
      hipError_t e = hipStreamBeginCapture(h.stream, hipStreamCaptureModeThreadLocal);
      if (e == hipSuccess) {
        enqueue_solve(h, P, B, d_rhs, d_x, k, ld);
        e = hipStreamEndCapture(h.stream, &h.g_graph);
      }
      h.stream = keep;
      h.prof = prof;
      if (e == hipSuccess) e = hipGraphInstantiate(&h.g_exec, h.g_graph, nullptr, nullptr, 0);
      if (e != hipSuccess) {
        release_graph(h);
        err = std::string("capturing the solve into a HIP graph failed: ") + hipGetErrorString(e);
        return -3;
      }
      h.g_key_k = k;
      h.g_key_ld = ld;
      h.g_key_rhs = d_rhs;
      h.g_key_x = d_x;
    }
    {
      ProfScope ps(h, "group:solve_graph", 0, 0);
      HIPCHK(hipGraphLaunch(h.g_exec, h.stream));
    }
  }
  HIPCHK(hipGetLastError());
  if (!on_device) HIPCHK(hipMemcpyAsync(x, d_x, (size_t)ld * k * 8, hipMemcpyDeviceToHost, h.stream));
  HIPCHK(hipStreamSynchronize(h.stream));
  prof_collect(h);
  h.t_solve = now_s() - t0;
  return 0;
}

// ---- the solve without allocations: the work vector lives in a fixed
// device array of this library, one per device, shared by every handle and
// call on that device (so calls that overlap on one device race).
constexpr int64_t SOLVE_SCRATCH_DOUBLES = (int64_t)32 << 20;  // 256 MiB
static __device__ __align__(256) double scratch[SOLVE_SCRATCH_DOUBLES];
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[64] = {};  // device address of `scratch`, per device

int64_t solve_noalloc_limit_bytes() { return SOLVE_SCRATCH_DOUBLES * 8; }

int solve_noalloc(Handle& h, const double* rhs, double* x, int k, int64_t ld, std::string& err) {
  if (!h.factored) {
    err = "solve called before ifmm_factor";
    return -6;
  }
  if (h.device < 0 || h.device >= 64) {
    err = "device index out of range";
    return -3;
  }
  const SolvePlan P = solve_plan(h, k, ld, false);
  if (P.total > SOLVE_SCRATCH_DOUBLES) {
    err = "the solve needs " + std::to_string(P.total * 8) + " bytes of work space for " + std::to_string(k) +
          " right-hand sides, above the fixed " + std::to_string(SOLVE_SCRATCH_DOUBLES * 8) +
          " bytes of the allocation-free solve (use ifmm_solve, or fewer right-hand sides)";
    return -1;
  }
  double* B = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[h.device]) {
      int cur = -1;
      HIPCHK(hipGetDevice(&cur));
      HIPCHK(hipSetDevice(h.device));
      void* ptr = nullptr;
      const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
      (void)hipSetDevice(cur);
      if (e != hipSuccess || !ptr) {
        err = std::string("hipGetSymbolAddress of the solve scratch failed: ") + hipGetErrorString(e);
        return -3;
      }
      g_scratch_ptr[h.device] = (double*)ptr;
    }
    B = g_scratch_ptr[h.device];
  }
  HIPCHK(hipSetDevice(h.device));
  const bool prof = h.prof;
  h.prof = false;  // no timing events: the caller may be capturing this stream
  enqueue_solve(h, P, B, rhs, x, k, ld);
  h.prof = prof;
  HIPCHK(hipGetLastError());
  return 0;
}

// ------------------------------------------------------------------ BD preconditioner
#define BDCHK(x)                                                                    \
  do {                                                                              \
    hipError_t e_ = (x);                                                            \
    if (e_ != hipSuccess) {                                                         \
      err = std::string(#x) + " failed: " + hipGetErrorString(e_);                  \
      return -3;                                                                    \
    }                                                                               \
  } while (0)

int bd_setup(BdHandle& h, const double* pts, int64_t n, const double* w, const double* diag, double diag_scalar,
             int level, int leaf_max, std::string& err) {
  const double t0 = now_s();
  err = h.tree.build(pts, n, leaf_max, 3, level, 2, 0);
  if (!err.empty()) return -1;
  err = h.tree.coincident(pts);
  if (!err.empty()) return -1;
  const Level& Lf = h.tree.levels[h.tree.depth];
  h.N = n;
  h.nbox = Lf.n;
  std::vector<int64_t> begin((size_t)Lf.n + 1, 0), off((size_t)Lf.n, 0);
  int64_t tot = 0;
  for (int32_t b = 0; b < Lf.n; ++b) {
    const int nb = (int)(Lf.pt_end[b] - Lf.pt_begin[b]);
    begin[b] = Lf.pt_begin[b];
    off[b] = tot;
    tot += (int64_t)nb * nb;
    h.nmax = std::max(h.nmax, nb);
  }
  begin[Lf.n] = n;
  if (h.nmax > BD_MAXN) {
    err = "a box of level " + std::to_string(h.tree.depth) + " holds " + std::to_string(h.nmax) +
          " points, above the supported " + std::to_string(BD_MAXN) + " (choose a finer level)";
    return -1;
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
    err = "no HIP device";
    return -3;
  }
  BDCHK(hipGetDevice(&h.device));
  if (!h.stream) {
    BDCHK(hipStreamCreate(&h.stream));
    h.own_stream = true;
  }
  std::vector<double> P(3 * n), W(n), Dg(n);
  for (int64_t t = 0; t < n; ++t) {
    const int64_t p = h.tree.perm[t];
    for (int e = 0; e < 3; ++e) P[3 * t + e] = pts[3 * p + e];
    W[t] = w ? w[p] : 1.0;
    Dg[t] = diag ? diag[p] : diag_scalar;
    if (!std::isfinite(W[t]) || !std::isfinite(Dg[t])) {
      err = "non-finite weight or diagonal entry";
      return -5;
    }
  }
  auto up = [&](auto** d, const auto& v) -> int {
    BDCHK(hipMalloc((void**)d, std::max<size_t>(v.size(), 1) * sizeof(v[0])));
    if (!v.empty()) BDCHK(hipMemcpy(*d, v.data(), v.size() * sizeof(v[0]), hipMemcpyHostToDevice));
    return 0;
  };
  int rc;
  if ((rc = up(&h.d_pts, P)) || (rc = up(&h.d_w, W)) || (rc = up(&h.d_diag, Dg)) || (rc = up(&h.d_perm, h.tree.perm)) ||
      (rc = up(&h.d_pt_begin, begin)))
    return rc;
  // per box: D (overwritten by its LU), X (becomes D^-1), panel inverses
  int64_t dinv = 0;
  std::vector<int64_t> doff((size_t)Lf.n);
  for (int32_t b = 0; b < Lf.n; ++b) {
    const int nb = (int)(begin[b + 1] - begin[b]);
    doff[b] = dinv;
    dinv += (int64_t)((nb + BLU_NB - 1) / BLU_NB) * 2 * 4096;
  }
  h.block_doubles = tot;
  BDCHK(hipMalloc((void**)&h.d_mem, (size_t)std::max<int64_t>(2 * tot, 1) * 8));
  BDCHK(hipMalloc((void**)&h.d_dinv, (size_t)std::max<int64_t>(dinv, 1) * 8));
  BDCHK(hipMalloc((void**)&h.d_piv, (size_t)std::max<int64_t>(n, 1) * 4));
  BDCHK(hipMalloc((void**)&h.d_info, (size_t)std::max(Lf.n, 1) * 4));
  std::vector<BluTask> tasks((size_t)Lf.n);
  for (int32_t b = 0; b < Lf.n; ++b) {
    const int nb = (int)(begin[b + 1] - begin[b]);
    tasks[b] = {h.d_mem + off[b], h.d_mem + tot + off[b], h.d_piv + begin[b], h.d_info + b, h.d_dinv + doff[b], nb, nb};
  }
  if ((rc = up((BluTask**)&h.d_tasks, tasks))) return rc;
  if (Lf.n > 0) {
    const BluTask* dt = (const BluTask*)h.d_tasks;
    hipLaunchKernelGGL(k_bd_assemble, dim3((unsigned)((h.nmax + 63) / 64), (unsigned)Lf.n), dim3(NT), 0, h.stream,
                       h.d_pts, h.d_w, h.d_diag, h.d_pt_begin, dt);
    enqueue_blocked_lu(dt, (unsigned)Lf.n, h.nmax, h.nmax, h.stream);
  }
  BDCHK(hipGetLastError());
  std::vector<int32_t> info((size_t)std::max(Lf.n, 1), 0);
  if (Lf.n > 0) BDCHK(hipMemcpyAsync(info.data(), h.d_info, (size_t)Lf.n * 4, hipMemcpyDeviceToHost, h.stream));
  BDCHK(hipStreamSynchronize(h.stream));
  for (int32_t b = 0; b < Lf.n; ++b)
    if (info[b]) {
      err = "singular diagonal block of box " + std::to_string(b);
      return -4;
    }
  // the LU factors and panel inverses are no longer needed
  (void)hipFree(h.d_dinv);
  h.d_dinv = nullptr;
  h.t_build = now_s() - t0;
  return 0;
}

int bd_apply(BdHandle& h, const double* r, double* z, std::string& err) {
  if (h.nbox > 0)
    hipLaunchKernelGGL(k_bd_apply, dim3((unsigned)h.nbox), dim3(NT), 0, h.stream, (const BluTask*)h.d_tasks,
                       h.d_pt_begin, h.d_perm, r, z);
  BDCHK(hipGetLastError());
  BDCHK(hipStreamSynchronize(h.stream));
  return 0;
}

void bd_release(BdHandle& h) {
  void* ptrs[] = {h.d_pts, h.d_w, h.d_diag, h.d_mem, h.d_dinv, h.d_perm, h.d_pt_begin, h.d_piv, h.d_info, h.d_tasks};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (h.own_stream && h.stream) (void)hipStreamDestroy(h.stream);
  h.stream = nullptr;
}

// ------------------------------------------------------------------ init / release
int device_init(Handle& h, std::string& err) {
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev < 1) {
    err = "no HIP device available";
    return -3;
  }
  HIPCHK(hipGetDevice(&h.device));
  hipDeviceProp_t prop;
  HIPCHK(hipGetDeviceProperties(&prop, h.device));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
    err = std::string("device is ") + prop.gcnArchName + ", this library is built for gfx950";
    return -3;
  }
  const double t0 = now_s();
  const int K = h.K;
  const int64_t N = h.N;
  h.poison = std::getenv("IFMM_POISON") != nullptr;
  int rc;
  std::vector<double> pts(h.pts), lo(h.tree.lo, h.tree.lo + 3);
  if ((rc = upload(h, &h.d_pts, pts, err))) return rc;
  if ((rc = upload(h, &h.d_w, h.w, err))) return rc;
  if ((rc = upload(h, &h.d_diag, h.diag, err))) return rc;
  if ((rc = upload(h, &h.d_perm, h.tree.perm, err))) return rc;
  if ((rc = upload(h, &h.d_pt_begin, h.tree.levels[h.tree.depth].pt_begin, err))) return rc;
  if ((rc = upload(h, &h.d_lo, lo, err))) return rc;
  (void)N;
  if ((rc = dalloc(h, &h.d_unit, 343LL * K * K, err))) return rc;
  if ((rc = dalloc(h, &h.d_uus, 343LL * K * K, err))) return rc;
  if ((rc = dalloc(h, &h.d_m2m8, 8LL * K * K, err))) return rc;
  hipLaunchKernelGGL(k_unit_m2l, dim3(343), dim3(NT), 0, h.stream, h.nc, h.d_unit);
  hipLaunchKernelGGL(k_unit_gram, dim3(343), dim3(NT), 0, h.stream, K, h.d_unit, h.d_uus);
  hipLaunchKernelGGL(k_m2m8, dim3(8), dim3(NT), 0, h.stream, h.nc, h.d_m2m8);
  HIPCHK(hipGetLastError());
  // far-field weights, top-down
  h.weights_G.assign((size_t)h.tree.depth + 1, nullptr);
  for (int l = 2; l <= h.tree.depth; ++l) {
    const Level& T = h.tree.levels[l];
    int32_t *d_coord = nullptr, *d_ilp = nullptr, *d_il = nullptr, *d_par = nullptr;
    if ((rc = upload(h, &d_coord, T.coord, err))) return rc;
    if ((rc = upload(h, &d_ilp, T.il_ptr, err))) return rc;
    if ((rc = upload(h, &d_il, T.il, err))) return rc;
    if ((rc = upload(h, &d_par, T.parent, err))) return rc;
    if ((rc = dalloc(h, &h.weights_G[l], std::max<int64_t>((int64_t)T.n * K * K, 1), err))) return rc;
    double* tmp = nullptr;
    if ((rc = dalloc(h, &tmp, std::max<int64_t>((int64_t)T.n * K * K, 1), err))) return rc;
    const double side = 2.0 * h.tree.H / (double)(1LL << l);
    if (T.n > 0)
      hipLaunchKernelGGL(k_weights, dim3(T.n), dim3(NT), 0, h.stream, K, T.n, d_coord, d_ilp, d_il, d_par, h.d_uus,
                         h.d_m2m8, 1.0 / (side * side), l > 2 ? h.weights_G[l - 1] : nullptr, h.weights_G[l], tmp);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(h.stream));
    dfree(h, tmp);
    dfree(h, d_coord);
    dfree(h, d_ilp);
    dfree(h, d_il);
    dfree(h, d_par);
  }
  h.dev_ready = true;
  h.t_init = now_s() - t0;
  return 0;
}

void release(Handle& h) {
  if (!h.dev_ready) return;
  (void)hipSetDevice(h.device);
  (void)hipStreamSynchronize(h.stream);
  clear_factor(h);
  for (auto& a : h.allocs) (void)hipFree(a.first);
  h.allocs.clear();
  if (h.d_flag) (void)hipFree(h.d_flag);
  h.d_flag = nullptr;
  for (auto& p : h.pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  h.pending.clear();
  for (hipEvent_t e : h.event_pool) (void)hipEventDestroy(e);
  h.event_pool.clear();
  if (h.cap_stream) (void)hipStreamDestroy(h.cap_stream);
  h.cap_stream = nullptr;
  if (h.side_stream) (void)hipStreamDestroy(h.side_stream);
  h.side_stream = nullptr;
  if (h.ev_fork) (void)hipEventDestroy(h.ev_fork);
  if (h.ev_join) (void)hipEventDestroy(h.ev_join);
  h.ev_fork = h.ev_join = nullptr;
  if (h.batch_stream) {
    if (h.stream == h.batch_stream) h.stream = nullptr;
    (void)hipStreamDestroy(h.batch_stream);
  }
  h.batch_stream = nullptr;
  h.dev_bytes = 0;
  h.dev_ready = false;
}

}  // namespace ifmm

// Internal test hook (not part of the public header): eigen-decomposition of
// `count` symmetric n x n matrices (host, column-major, back to back) with the
// device solver; lam (count x n, descending) and the k leading vectors
// (count x n x k).  Returns 0 or a negative status.
extern "C" int ifmm_internal_syev(const double* A, int count, int n, int k, double* lam, double* V, int jacobi) {
  using namespace ifmm;
  if (count < 1 || n < 1 || n > TRD_MAXN || k < 0 || k > n) return -1;
  const int64_t nn = (int64_t)n * n;
  double *dA = nullptr, *dV = nullptr, *dW = nullptr, *dL = nullptr, *dI = nullptr;
  EigTask* dT = nullptr;
  int32_t* dC = nullptr;
  const int64_t wsz = jacobi ? nn : 3LL * n;
  if (hipMalloc((void**)&dA, count * nn * 8) != hipSuccess) return -3;
  (void)hipMalloc((void**)&dV, count * nn * 8);
  (void)hipMalloc((void**)&dW, count * wsz * 8);
  (void)hipMalloc((void**)&dL, count * (int64_t)n * 8);
  (void)hipMalloc((void**)&dI, count * (5LL * n * std::max(k, 1)) * 8);
  (void)hipMalloc((void**)&dT, count * sizeof(EigTask));
  (void)hipMalloc((void**)&dC, count * 4);
  std::vector<EigTask> t(count);
  for (int c = 0; c < count; ++c)
    t[c] = {dA + c * nn, dV + c * nn, dW + c * wsz, dL + (int64_t)c * n, dI + c * (5LL * n * std::max(k, 1)), n, k};
  (void)hipMemcpy(dA, A, count * nn * 8, hipMemcpyHostToDevice);
  (void)hipMemcpy(dT, t.data(), count * sizeof(EigTask), hipMemcpyHostToDevice);
  int rc = 0;
  if (jacobi) {
    hipLaunchKernelGGL(k_eig_jacobi, dim3(count), dim3(NT), 0, nullptr, dT, 0.0, dC);
  } else {
    // the factorisation's routing: one workgroup below the threshold, the
    // multi-workgroup reduction from there on
    Handle hh;
    std::string err;
    rc = eig_values(hh, t, dT, 0.0, dC, nullptr, err);
    if (rc == 0) eig_vectors(hh, t, dT, nullptr);
    if (hipDeviceSynchronize() != hipSuccess) rc = -3;
    for (auto& a : hh.allocs) (void)hipFree(a.first);
  }
  if (hipDeviceSynchronize() != hipSuccess) rc = -3;
  (void)hipMemcpy(lam, dL, count * (int64_t)n * 8, hipMemcpyDeviceToHost);
  for (int c = 0; c < count; ++c)
    (void)hipMemcpy(V + c * (int64_t)n * k, dV + c * nn, (int64_t)n * k * 8, hipMemcpyDeviceToHost);
  (void)hipFree(dA); (void)hipFree(dV); (void)hipFree(dW); (void)hipFree(dL); (void)hipFree(dI);
  (void)hipFree(dT); (void)hipFree(dC);
  return rc;
}

namespace ifmm {
__global__ void __launch_bounds__(NT) k_internal_gemm(int m, int n, int k, double alpha, const double* A, int lda, int tA, const double* B,
                                int ldb, int tB, double beta, double* C, int ldc, int f32) {
  const int i0 = blockIdx.x * 64, j0 = blockIdx.y * 64;
  const int mm = min(64, m - i0), nn = min(64, n - j0);
  if (mm <= 0 || nn <= 0) return;
  const double* Ab = tA ? A + (int64_t)i0 * lda : A + i0;
  const double* Bb = tB ? B + j0 : B + (int64_t)j0 * ldb;
  if (f32 == 2) wg_gemm_f32_deep(mm, nn, k, alpha, Ab, lda, tA != 0, Bb, ldb, tB != 0, beta, C + i0 + (int64_t)j0 * ldc, ldc);
  else if (f32 == 3 && !tA && !tB) wg_gemm_f64m(mm, nn, k, alpha, Ab, lda, Bb, ldb, beta, C + i0 + (int64_t)j0 * ldc, ldc);
  else if (f32 == 3) wg_gemm(mm, nn, k, alpha, Ab, lda, tA != 0, Bb, ldb, tB != 0, beta, C + i0 + (int64_t)j0 * ldc, ldc);
  else wg_gemm_p(f32 != 0, mm, nn, k, alpha, Ab, lda, tA != 0, Bb, ldb, tB != 0, beta, C + i0 + (int64_t)j0 * ldc, ldc);
}
}  // namespace ifmm

// Test hook (not declared in the public header): X = D^-1 B for `count`
// matrices of order d with W right-hand columns through the blocked LU path.
extern "C" int ifmm_internal_blocked_solve(const double* D, int count, int d, const double* B, int W, double* X,
                                           int32_t* info) {
  using namespace ifmm;
  if (count < 1 || d < 1 || W < 1) return -1;
  const int64_t dd = (int64_t)d * d, dw = (int64_t)d * W, nblk = (d + BLU_NB - 1) / BLU_NB;
  double *dD = nullptr, *dX = nullptr, *dI = nullptr;
  int32_t *dP = nullptr, *dInfo = nullptr;
  BluTask* dT = nullptr;
  if (hipMalloc((void**)&dD, count * dd * 8) != hipSuccess) return -3;
  (void)hipMalloc((void**)&dX, count * dw * 8);
  (void)hipMalloc((void**)&dI, count * nblk * 2 * 4096 * 8);
  (void)hipMalloc((void**)&dP, count * (int64_t)d * 4);
  (void)hipMalloc((void**)&dInfo, count * 4);
  (void)hipMalloc((void**)&dT, count * sizeof(BluTask));
  std::vector<BluTask> t(count);
  for (int c = 0; c < count; ++c)
    t[c] = {dD + c * dd, dX + c * dw, dP + (int64_t)c * d, dInfo + c, dI + c * nblk * 2 * 4096, d, W};
  (void)hipMemcpy(dD, D, count * dd * 8, hipMemcpyHostToDevice);
  (void)hipMemcpy(dX, B, count * dw * 8, hipMemcpyHostToDevice);
  (void)hipMemset(dInfo, 0, count * 4);
  (void)hipMemcpy(dT, t.data(), count * sizeof(BluTask), hipMemcpyHostToDevice);
  enqueue_blocked_lu(dT, (unsigned)count, d, W, nullptr);
  int rc = hipDeviceSynchronize() == hipSuccess ? 0 : -3;
  (void)hipMemcpy(X, dX, count * dw * 8, hipMemcpyDeviceToHost);
  (void)hipMemcpy(info, dInfo, count * 4, hipMemcpyDeviceToHost);
  (void)hipFree(dD); (void)hipFree(dX); (void)hipFree(dI); (void)hipFree(dP); (void)hipFree(dInfo); (void)hipFree(dT);
  return rc;
}

// Test hook (not part of the declared ABI): C = alpha op(A) op(B) + beta C on
// host arrays (column-major, tight leading dimensions) with the FP64 (f32 = 0)
// or FP32 matrix-core workgroup product (f32 = 1: the lite tile; f32 = 2: the
// double-buffered tile from inner dimension 96 on), or the FP64 matrix-core
// product (f32 = 3, untransposed operands), one workgroup per 64 x 64 tile.
extern "C" int ifmm_internal_gemm(int m, int n, int k, double alpha, const double* A, int tA, const double* B, int tB,
                                  double beta, double* C, int f32) {
  using namespace ifmm;
  if (m < 1 || n < 1 || k < 0) return -1;
  const int lda = tA ? std::max(k, 1) : m, ldb = tB ? n : std::max(k, 1);
  const int64_t sa = (int64_t)m * k, sb = (int64_t)k * n, sc = (int64_t)m * n;
  double *dA = nullptr, *dB = nullptr, *dC = nullptr;
  if (hipMalloc((void**)&dA, std::max<int64_t>(sa, 1) * 8) != hipSuccess) return -3;
  if (hipMalloc((void**)&dB, std::max<int64_t>(sb, 1) * 8) != hipSuccess) return -3;
  if (hipMalloc((void**)&dC, sc * 8) != hipSuccess) return -3;
  if (sa) (void)hipMemcpy(dA, A, sa * 8, hipMemcpyHostToDevice);
  if (sb) (void)hipMemcpy(dB, B, sb * 8, hipMemcpyHostToDevice);
  (void)hipMemcpy(dC, C, sc * 8, hipMemcpyHostToDevice);
  hipLaunchKernelGGL(k_internal_gemm, dim3((m + 63) / 64, (n + 63) / 64), dim3(NT), 0, nullptr, m, n, k, alpha, dA, lda,
                     tA, dB, ldb, tB, beta, dC, m, f32);
  int rc = hipDeviceSynchronize() == hipSuccess ? 0 : -3;
  (void)hipMemcpy(C, dC, sc * 8, hipMemcpyDeviceToHost);
  (void)hipFree(dA); (void)hipFree(dB); (void)hipFree(dC);
  return rc;
}
