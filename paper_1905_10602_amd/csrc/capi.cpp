// C ABI of the library (declared in include/ifmm.h).  Argument checking,
// error reporting and handle life-time; the work is in engine.hip / tree.cpp.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <atomic>
#include <functional>
#include <thread>
#include <vector>

#include "../../include/ifmm.h"
#include "engine.hpp"
#include "fmm.hpp"

struct ifmm_handle {
  ifmm::Handle h;
};

struct fmm_handle {
  ifmm::FmmHandle h;
};

struct bd_handle {
  ifmm::BdHandle h;
};

namespace ifmm {
static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }
const char* get_error() { return g_err.c_str(); }

int build_host(Handle& h, const double* pts, int64_t n, const double* w, const double* diag, double diag_scalar,
               std::string& err) {
  err = h.tree.build(pts, n, h.leaf_max, h.sigma, h.bottom_level > 0 ? h.bottom_level : 0, h.top_tau, h.colouring);
  if (!err.empty()) return IFMM_EINVAL;
  if (h.bottom_level == -1) {  // the depth the cost model prefers (a coarser leaf level, or the same)
    const int l = h.tree.cost_depth(h.K, &h.depth_costs);
    if (l != h.tree.depth) {
      err = h.tree.build(pts, n, h.leaf_max, h.sigma, l, h.top_tau, h.colouring);
      if (!err.empty()) return IFMM_EINVAL;
    }
  }
  err = h.tree.coincident(pts);
  if (!err.empty()) return IFMM_EINVAL;
  h.N = n;
  h.symmetric = (w == nullptr);
  // points inside every node's box (leaf ranges summed up the tree)
  const int D = h.tree.depth;
  h.pt_count.assign((size_t)D + 1, {});
  for (int l = D; l >= 2; --l) {
    const Level& L = h.tree.levels[l];
    h.pt_count[l].assign((size_t)L.n, 0);
    for (int i = 0; i < L.n; ++i) {
      if (l == D) {
        h.pt_count[l][i] = L.pt_end[i] - L.pt_begin[i];
      } else {
        for (int e = L.child_ptr[i]; e < L.child_ptr[i + 1]; ++e) h.pt_count[l][i] += h.pt_count[l + 1][L.child[e]];
      }
    }
  }
  h.pts.resize((size_t)(3 * n));
  h.w.resize((size_t)n);
  h.diag.resize((size_t)n);
  for (int64_t t = 0; t < n; ++t) {
    const int64_t p = h.tree.perm[t];
    for (int e = 0; e < 3; ++e) h.pts[3 * t + e] = pts[3 * p + e];
    h.w[t] = w ? w[p] : 1.0;
    h.diag[t] = diag ? diag[p] : diag_scalar;
    if (!std::isfinite(h.w[t]) || !std::isfinite(h.diag[t])) {
      err = "non-finite weight or diagonal entry";
      return IFMM_ENONFINITE;
    }
  }
  return IFMM_OK;
}
}  // namespace ifmm

static ifmm_status fail(int code, const std::string& msg) {
  ifmm::set_error(msg);
  return (ifmm_status)code;
}

extern "C" {

void ifmm_default_options(ifmm_options* opt) {
  if (!opt) return;
  opt->leaf_max = 64;
  opt->cheb_order = 4;
  opt->precision = IFMM_PREC_FP64;
  opt->top_tau = 2;
  opt->rank_model = nullptr;
  opt->tune_cache = nullptr;
  opt->max_device_bytes = 0;
  opt->deterministic = 1;
  opt->bottom_level = 0;
  opt->rank_cap = 0;
  opt->colouring = 0;
  opt->stream = nullptr;
}

ifmm_status ifmm_build(const double* points, int64_t n, const double* weights, const double* diag, double diag_scalar,
                       int32_t kernel, double eps, int32_t sigma, const ifmm_options* opt, ifmm_handle** out) {
  ifmm::set_error("");
  if (!out) return fail(IFMM_EINVAL, "out is NULL");
  *out = nullptr;
  if (!points) return fail(IFMM_EINVAL, "points is NULL");
  if (n < 1) return fail(IFMM_EINVAL, "n must be >= 1");
  if (kernel != IFMM_KERNEL_LAPLACE3D) return fail(IFMM_EINVAL, "unsupported kernel");
  if (!(eps > 0.0 && eps < 1.0)) return fail(IFMM_EINVAL, "eps must lie in (0, 1)");
  if (sigma < 3) return fail(IFMM_EINVAL, "sigma must be >= 3 (sigma <= 2 serialises every node)");
  if (!diag && !std::isfinite(diag_scalar)) return fail(IFMM_ENONFINITE, "non-finite diag_scalar");
  ifmm_options o;
  ifmm_default_options(&o);
  if (opt) o = *opt;
  if (o.leaf_max < 1) return fail(IFMM_EINVAL, "leaf_max must be >= 1");
  if (o.cheb_order < 2 || o.cheb_order > 6) return fail(IFMM_EINVAL, "cheb_order must lie in [2, 6]");
  if (o.precision != IFMM_PREC_FP64 && o.precision != IFMM_PREC_MIXED) return fail(IFMM_EINVAL, "unknown precision mode");
  if (o.rank_cap < 0) return fail(IFMM_EINVAL, "rank_cap must be >= 0");
  if (o.top_tau < 2) return fail(IFMM_EINVAL, "top_tau must be >= 2");
  if (o.bottom_level < -1 || o.bottom_level == 1 || o.bottom_level > 10)
    return fail(IFMM_EINVAL, "bottom_level must be 0 (from leaf_max), -1 (cost model) or in [2, 10]");
  if (o.deterministic != 0 && o.deterministic != 1) return fail(IFMM_EINVAL, "deterministic must be 0 or 1");
  if (o.colouring != 0 && o.colouring != 1) return fail(IFMM_EINVAL, "colouring must be 0 (Alg. 3) or 1 (look-back)");
  ifmm_handle* H = new (std::nothrow) ifmm_handle();
  if (!H) return fail(IFMM_ENOMEM, "host allocation failed");
  ifmm::Handle& h = H->h;
  h.eps = eps;
  h.sigma = sigma;
  h.leaf_max = o.leaf_max;
  h.nc = o.cheb_order;
  h.K = o.cheb_order * o.cheb_order * o.cheb_order;
  h.precision = o.precision;
  h.rank_cap = o.rank_cap;
  h.max_bytes = o.max_device_bytes;
  h.stream = (hipStream_t)o.stream;
  h.top_tau = o.top_tau;
  h.bottom_level = o.bottom_level;
  h.colouring = o.colouring;
  if (o.tune_cache) h.tune_cache = o.tune_cache;
  if (o.rank_model) {
    const int64_t np = ifmm_rank_model_params(IFMM_RANK_FEATURES);
    FILE* f = std::fopen(o.rank_model, "rb");
    if (!f) {
      delete H;
      return fail(IFMM_EINVAL, std::string("cannot open rank_model file ") + o.rank_model);
    }
    h.model_host.assign((size_t)np, 0.f);
    const size_t got = std::fread(h.model_host.data(), 4, (size_t)np, f);
    const bool extra = std::fgetc(f) != EOF;
    std::fclose(f);
    if (got != (size_t)np || extra) {
      delete H;
      return fail(IFMM_EINVAL, "rank_model file must hold exactly " + std::to_string(np) + " FP32 values");
    }
    for (float v : h.model_host)
      if (!std::isfinite(v)) {
        delete H;
        return fail(IFMM_ENONFINITE, "non-finite value in the rank_model file");
      }
  }
  std::string err;
  int rc;
  try {
    rc = ifmm::build_host(h, points, n, weights, diag, diag_scalar, err);
  } catch (const std::bad_alloc&) {
    rc = IFMM_ENOMEM;
    err = "host allocation failed";
  }
  if (rc) {
    delete H;
    return fail(rc, err);
  }
  *out = H;
  return IFMM_OK;
}

ifmm_status ifmm_factor(ifmm_handle* H) {
  ifmm::set_error("");
  if (!H) return fail(IFMM_EINVAL, "handle is NULL");
  std::string err;
  int rc;
  try {
    rc = ifmm::factor(H->h, err);
  } catch (const std::bad_alloc&) {
    rc = IFMM_ENOMEM;
    err = "host allocation failed";
  }
  if (rc) return fail(rc, err);
  return IFMM_OK;
}

ifmm_status ifmm_solve(ifmm_handle* H, const double* rhs, double* x, int32_t nrhs, int64_t ld, int32_t on_device) {
  ifmm::set_error("");
  if (!H) return fail(IFMM_EINVAL, "handle is NULL");
  if (!H->h.factored) return fail(IFMM_ESTATE, "ifmm_solve called before ifmm_factor");
  if (!rhs || !x) return fail(IFMM_EINVAL, "rhs / x is NULL");
  if (nrhs < 1) return fail(IFMM_EINVAL, "nrhs must be >= 1");
  if (ld < H->h.N) return fail(IFMM_EINVAL, "ld must be >= N");
  std::string err;
  int rc = ifmm::solve(H->h, rhs, x, nrhs, ld, on_device ? 1 : 0, err);
  if (rc) return fail(rc, err);
  return IFMM_OK;
}

ifmm_status ifmm_solve_noalloc(ifmm_handle* H, const double* rhs, double* x, int32_t nrhs, int64_t ld) {
  ifmm::set_error("");
  if (!H) return fail(IFMM_EINVAL, "handle is NULL");
  if (!H->h.factored) return fail(IFMM_ESTATE, "ifmm_solve_noalloc called before ifmm_factor");
  if (!rhs || !x) return fail(IFMM_EINVAL, "rhs / x is NULL");
  if (nrhs < 1) return fail(IFMM_EINVAL, "nrhs must be >= 1");
  if (ld < H->h.N) return fail(IFMM_EINVAL, "ld must be >= N");
  std::string err;
  int rc = ifmm::solve_noalloc(H->h, rhs, x, nrhs, ld, err);
  if (rc) return fail(rc, err);
  return IFMM_OK;
}

int64_t ifmm_solve_noalloc_max_bytes(void) { return ifmm::solve_noalloc_limit_bytes(); }

ifmm_status ifmm_stats(const ifmm_handle* H, char* json, int64_t cap) {
  if (!H || !json || cap < 1) return fail(IFMM_EINVAL, "bad arguments");
  const ifmm::Handle& h = H->h;
  std::string s = "{\"N\":" + std::to_string(h.N) + ",\"depth\":" + std::to_string(h.tree.depth) +
                  ",\"sigma\":" + std::to_string(h.sigma) + ",\"eps\":" + std::to_string(h.eps) +
                  ",\"t_init\":" + std::to_string(h.t_init) + ",\"t_factor\":" + std::to_string(h.t_factor) +
                  ",\"t_solve\":" + std::to_string(h.t_solve) + ",\"device_bytes\":" + std::to_string(h.dev_bytes) +
                  ",\"store_bytes\":" + std::to_string(h.store_bytes) + ",\"top_n\":" + std::to_string(h.top_n) +
                  ",\"t_top\":" + std::to_string(h.t_top) + ",\"far_pairs\":" + std::to_string(h.stat_far) + ",\"changed\":" + std::to_string(h.stat_changed) + ",\"grown\":" + std::to_string(h.stat_grown) +
                  ",\"sketches\":" + std::to_string(h.stat_sketch) +
                  ",\"sketches_rejected\":" + std::to_string(h.stat_sketch_rejected) +
                  ",\"sketches_narrow\":" + std::to_string(h.stat_sketch_narrow) +
                  ",\"full_decompositions\":" + std::to_string(h.stat_full) +
                  ",\"sketch_columns\":" + std::to_string(h.stat_sketch_cols) +
                  ",\"rank_predictions\":" + std::to_string(h.stat_predicted) +
                  ",\"t_sync\":" + std::to_string(h.t_sync) +
                  ",\"top_tau\":" + std::to_string(h.top_tau) + ",\"colouring\":" + std::to_string(h.colouring) +
                  ",\"bottom_level\":" + std::to_string(h.bottom_level) + ",\"depth_costs\":[" +
                  [&] {
                    std::string c;
                    for (size_t q = 0; q < h.depth_costs.size(); ++q) {
                      char b[40];
                      std::snprintf(b, sizeof b, "%s%.6e", q ? "," : "", h.depth_costs[q]);
                      c += b;
                    }
                    return c;
                  }() + "]" +
                  ",\"t_h2d\":" + std::to_string(h.t_h2d) +
                  ",\"levels\":[";
  for (int l = 2; l <= h.tree.depth; ++l) {
    const ifmm::Level& T = h.tree.levels[l];
    long long rs = 0, rm = 0, ns = 0, nm = 0, sg = 0, st = 0;
    if ((int)h.lv.size() > l) {
      const ifmm::DevLevel& L = h.lv[l];
      for (size_t i = 0; i < L.r.size(); ++i) { rs += L.r[i]; rm = std::max<long long>(rm, L.r[i]); }
      for (size_t i = 0; i < L.n.size(); ++i) { ns += L.n[i]; nm = std::max<long long>(nm, L.n[i]); }
      sg = (long long)L.sg.size();
      st = (long long)L.st_b.size();
    }
    s += std::string(l > 2 ? "," : "") + "{\"level\":" + std::to_string(l) + ",\"nodes\":" + std::to_string(T.n) +
         ",\"colours\":" + std::to_string(T.ncolour) + ",\"rank_sum\":" + std::to_string(rs) +
         ",\"rank_max\":" + std::to_string(rm) + ",\"n_sum\":" + std::to_string(ns) + ",\"n_max\":" + std::to_string(nm) +
         ",\"solve_bwd_tasks\":" + std::to_string(st) + ",\"solve_split_tiles\":" + std::to_string(sg) +
         ",\"t_setup\":" + std::to_string((int)h.t_level_setup.size() > l ? h.t_level_setup[l] : 0.0) +
         ",\"t_elim\":" + std::to_string((int)h.t_level_elim.size() > l ? h.t_level_elim[l] : 0.0) + "}";
  }
  s += "],\"kernels\":{";
  bool first = true;
  for (const auto& kv : h.kstat) {
    char buf[256];
    std::snprintf(buf, sizeof buf, "%s\"%s\":{\"launches\":%lld,\"ms\":%.6f,\"flops\":%.6e,\"bytes\":%.6e}",
                  first ? "" : ",", kv.first.c_str(), (long long)kv.second.launches, kv.second.ms, kv.second.flops,
                  kv.second.bytes);
    s += buf;
    first = false;
  }
  s += "},\"aux\":{";
  first = true;
  for (const auto& kv : h.aux) {
    char buf[160];
    std::snprintf(buf, sizeof buf, "%s\"%s\":%.6e", first ? "" : ",", kv.first.c_str(), kv.second);
    s += buf;
    first = false;
  }
  s += "},\"host_ms\":{";
  first = true;
  for (const auto& kv : h.host_ms) {
    char buf[160];
    std::snprintf(buf, sizeof buf, "%s\"%s\":%.3f", first ? "" : ",", kv.first.c_str(), kv.second);
    s += buf;
    first = false;
  }
  s += "}}";
  std::snprintf(json, (size_t)cap, "%s", s.c_str());
  return IFMM_OK;
}

ifmm_status ifmm_tree_depth(const ifmm_handle* H, int32_t* depth) {
  if (!H || !depth) return fail(IFMM_EINVAL, "bad arguments");
  *depth = H->h.tree.depth;
  return IFMM_OK;
}

ifmm_status ifmm_tree_perm(const ifmm_handle* H, int64_t* perm) {
  if (!H || !perm) return fail(IFMM_EINVAL, "bad arguments");
  std::memcpy(perm, H->h.tree.perm.data(), H->h.tree.perm.size() * sizeof(int64_t));
  return IFMM_OK;
}

ifmm_status ifmm_tree_level(const ifmm_handle* H, int32_t level, int32_t* nnodes, int32_t* coords, int32_t* parent,
                            int32_t* colour, int32_t* ncolour) {
  if (!H || !nnodes) return fail(IFMM_EINVAL, "bad arguments");
  const ifmm::Tree& T = H->h.tree;
  if (level < 2 || level > T.depth) return fail(IFMM_EINVAL, "level out of range");
  const ifmm::Level& L = T.levels[level];
  *nnodes = L.n;
  if (coords) std::memcpy(coords, L.coord.data(), L.coord.size() * 4);
  if (parent) std::memcpy(parent, L.parent.data(), L.parent.size() * 4);
  if (colour) std::memcpy(colour, L.colour.data(), L.colour.size() * 4);
  if (ncolour) *ncolour = L.ncolour;
  return IFMM_OK;
}

ifmm_status ifmm_tree_lists(const ifmm_handle* H, int32_t level, int32_t which, int32_t* ptr, int32_t* idx) {
  if (!H || !ptr || (which != 0 && which != 1)) return fail(IFMM_EINVAL, "bad arguments");
  const ifmm::Tree& T = H->h.tree;
  if (level < 2 || level > T.depth) return fail(IFMM_EINVAL, "level out of range");
  const ifmm::Level& L = T.levels[level];
  const std::vector<int32_t>& p = which ? L.il_ptr : L.nbr_ptr;
  const std::vector<int32_t>& v = which ? L.il : L.nbr;
  std::memcpy(ptr, p.data(), p.size() * 4);
  if (idx) std::memcpy(idx, v.data(), v.size() * 4);
  return IFMM_OK;
}

ifmm_status ifmm_ranks(const ifmm_handle* H, int32_t level, int32_t* ranks) {
  if (!H || !ranks) return fail(IFMM_EINVAL, "bad arguments");
  const ifmm::Handle& h = H->h;
  if (!h.factored) return fail(IFMM_ESTATE, "no factorisation");
  if (level < 2 || level > h.tree.depth) return fail(IFMM_EINVAL, "level out of range");
  std::memcpy(ranks, h.lv[level].r.data(), h.lv[level].r.size() * 4);
  return IFMM_OK;
}

// Many independent handles at once: each gets a stream of its own (a
// library-owned one if it has none) and a host thread drives its
// colour-by-colour schedule, so the small per-colour launches of different
// geometries overlap on the device.
static ifmm_status run_batch(ifmm_handle** hs, int32_t count, int32_t threads,
                             const std::function<int(ifmm_handle*, int32_t, std::string&)>& work, int32_t* failed) {
  ifmm::set_error("");
  if (!hs || count < 1) return fail(IFMM_EINVAL, "bad arguments");
  for (int32_t g = 0; g < count; ++g) {
    if (!hs[g]) return fail(IFMM_EINVAL, "NULL handle in the batch");
    for (int32_t q = 0; q < g; ++q)
      if (hs[q] == hs[g]) return fail(IFMM_EINVAL, "a handle appears twice in the batch");
  }
  for (int32_t g = 0; g < count; ++g) {
    ifmm::Handle& h = hs[g]->h;
    if (!h.stream && !h.batch_stream) {
      if (hipStreamCreateWithFlags(&h.batch_stream, hipStreamNonBlocking) != hipSuccess)
        return fail(IFMM_EDEVICE, "stream creation failed");
    }
    if (!h.stream) h.stream = h.batch_stream;
  }
  const int nt = std::max(1, std::min<int>(threads > 0 ? threads : 8, count));
  std::vector<int> rcs(count, 0);
  std::vector<std::string> errs(count);
  std::vector<std::thread> pool;
  std::atomic<int> next{0};
  for (int t = 0; t < nt; ++t)
    pool.emplace_back([&]() {
      for (int g = next++; g < count; g = next++) {
        try {
          rcs[g] = work(hs[g], g, errs[g]);
        } catch (const std::bad_alloc&) {
          rcs[g] = IFMM_ENOMEM;
          errs[g] = "host allocation failed";
        }
      }
    });
  for (auto& th : pool) th.join();
  for (int32_t g = 0; g < count; ++g)
    if (rcs[g]) {
      if (failed) *failed = g;
      return fail(rcs[g], "geometry " + std::to_string(g) + ": " + errs[g]);
    }
  if (failed) *failed = -1;
  return IFMM_OK;
}

ifmm_status ifmm_factor_batch(ifmm_handle** hs, int32_t count, int32_t threads, int32_t* failed) {
  return run_batch(hs, count, threads, [](ifmm_handle* H, int32_t, std::string& e) { return ifmm::factor(H->h, e); },
                   failed);
}

ifmm_status ifmm_solve_batch(ifmm_handle** hs, int32_t count, const double* const* rhs, double* const* x,
                             int32_t nrhs, const int64_t* ld, int32_t on_device, int32_t threads, int32_t* failed) {
  if (!hs || !rhs || !x || !ld || nrhs < 1 || count < 1) return fail(IFMM_EINVAL, "bad arguments");
  for (int32_t g = 0; g < count; ++g) {
    if (!hs[g] || !hs[g]->h.factored) return fail(IFMM_ESTATE, "a handle of the batch is not factored");
    if (!rhs[g] || !x[g] || ld[g] < hs[g]->h.N) return fail(IFMM_EINVAL, "bad vectors in the batch");
  }
  return run_batch(
      hs, count, threads,
      [&](ifmm_handle* H, int32_t g, std::string& e) {
        return ifmm::solve(H->h, rhs[g], x[g], nrhs, ld[g], on_device ? 1 : 0, e);
      },
      failed);
}

ifmm_status ifmm_set_rank_model(ifmm_handle* H, const float* theta, int32_t nfeat) {
  ifmm::set_error("");
  if (!H) return fail(IFMM_EINVAL, "handle is NULL");
  ifmm::Handle& h = H->h;
  h.model_host.clear();  // an explicit model (or none) replaces options.rank_model
  if (h.d_model) {
    (void)hipFree(h.d_model);
    h.d_model = nullptr;
  }
  if (!theta) return IFMM_OK;
  if (nfeat != IFMM_RANK_FEATURES) return fail(IFMM_EINVAL, "the rank model takes IFMM_RANK_FEATURES inputs");
  const int64_t np = ifmm_rank_model_params(nfeat);
  for (int64_t i = 0; i < np; ++i)
    if (!std::isfinite(theta[i])) return fail(IFMM_ENONFINITE, "non-finite model parameter");
  if (hipMalloc((void**)&h.d_model, (size_t)np * 4) != hipSuccess) return fail(IFMM_EDEVICE, "device allocation failed");
  if (hipMemcpy(h.d_model, theta, (size_t)np * 4, hipMemcpyHostToDevice) != hipSuccess)
    return fail(IFMM_EDEVICE, "copy failed");
  return IFMM_OK;
}

ifmm_status ifmm_record_ranks(ifmm_handle* H, int32_t on) {
  if (!H) return fail(IFMM_EINVAL, "handle is NULL");
  H->h.record_ranks = on != 0;
  return IFMM_OK;
}

ifmm_status ifmm_rank_records(const ifmm_handle* H, float* X, float* t, int64_t cap, int64_t* count) {
  if (!H || !count) return fail(IFMM_EINVAL, "bad arguments");
  const ifmm::Handle& h = H->h;
  const int64_t m = (int64_t)h.rec_t.size();
  *count = m;
  if (!X || !t) return IFMM_OK;
  const int64_t k = std::min(m, cap);
  std::memcpy(X, h.rec_X.data(), (size_t)k * IFMM_RANK_FEATURES * 4);
  std::memcpy(t, h.rec_t.data(), (size_t)k * 4);
  return IFMM_OK;
}

const char* ifmm_last_error(void) { return ifmm::get_error(); }

void ifmm_destroy(ifmm_handle* H) {
  if (!H) return;
  if (H->h.d_model) (void)hipFree(H->h.d_model);
  H->h.d_model = nullptr;
  ifmm::release(H->h);
  delete H;
}

ifmm_status fmm_build(const double* points, int64_t n, const double* weights, const double* diag, double diag_scalar,
                      int32_t cheb_order, int32_t leaf_max, void* stream, fmm_handle** out) {
  ifmm::set_error("");
  if (!out) return fail(IFMM_EINVAL, "out is NULL");
  *out = nullptr;
  if (!points) return fail(IFMM_EINVAL, "points is NULL");
  if (n < 1) return fail(IFMM_EINVAL, "n must be >= 1");
  if (cheb_order < 2 || cheb_order > 6) return fail(IFMM_EINVAL, "cheb_order must lie in [2, 6]");
  if (leaf_max < 1) return fail(IFMM_EINVAL, "leaf_max must be >= 1");
  if (!diag && !std::isfinite(diag_scalar)) return fail(IFMM_ENONFINITE, "non-finite diag_scalar");
  fmm_handle* F = new (std::nothrow) fmm_handle();
  if (!F) return fail(IFMM_ENOMEM, "host allocation failed");
  F->h.nc = cheb_order;
  F->h.leaf_max = leaf_max;
  F->h.stream = (hipStream_t)stream;
  std::string err;
  int rc;
  try {
    rc = ifmm::fmm_setup(F->h, points, n, weights, diag, diag_scalar, err);
  } catch (const std::bad_alloc&) {
    rc = IFMM_ENOMEM;
    err = "host allocation failed";
  }
  if (rc) {
    ifmm::fmm_release(F->h);
    delete F;
    return fail(rc, err);
  }
  *out = F;
  return IFMM_OK;
}

// host <-> device staging for the vector calls
struct Staged {
  double* d = nullptr;
  ~Staged() {
    if (d) (void)hipFree(d);
  }
};

ifmm_status fmm_matvec(fmm_handle* F, const double* x, double* y, int32_t on_device) {
  ifmm::set_error("");
  if (!F || !x || !y) return fail(IFMM_EINVAL, "bad arguments");
  ifmm::FmmHandle& h = F->h;
  std::string err;
  int rc;
  if (on_device) {
    rc = ifmm::fmm_apply(h, x, y, err);
  } else {
    Staged st;
    if (hipMalloc((void**)&st.d, (size_t)(2 * h.N) * 8) != hipSuccess) return fail(IFMM_ENOMEM, "device allocation failed");
    if (hipMemcpy(st.d, x, (size_t)h.N * 8, hipMemcpyHostToDevice) != hipSuccess) return fail(IFMM_EDEVICE, "copy failed");
    rc = ifmm::fmm_apply(h, st.d, st.d + h.N, err);
    if (!rc && hipMemcpy(y, st.d + h.N, (size_t)h.N * 8, hipMemcpyDeviceToHost) != hipSuccess)
      return fail(IFMM_EDEVICE, "copy failed");
  }
  if (rc) return fail(rc, err);
  return IFMM_OK;
}

ifmm_status fmm_gmres(fmm_handle* F, const double* b, ifmm_handle* P, double tol, int32_t restart, int32_t maxit,
                      double* x, int32_t on_device, int32_t* iters, double* relres) {
  ifmm::set_error("");
  if (!F || !b || !x || !iters || !relres) return fail(IFMM_EINVAL, "bad arguments");
  if (restart < 1 || restart > 1000) return fail(IFMM_EINVAL, "restart must lie in [1, 1000]");
  if (maxit < 0) return fail(IFMM_EINVAL, "maxit must be >= 0");
  if (!(tol > 0.0)) return fail(IFMM_EINVAL, "tol must be > 0");
  if (b == x) return fail(IFMM_EINVAL, "b and x may not alias");
  ifmm::FmmHandle& h = F->h;
  if (P) {
    if (!P->h.factored) return fail(IFMM_ESTATE, "preconditioner is not factored");
    if (P->h.N != h.N) return fail(IFMM_EINVAL, "preconditioner size differs from the FMM's");
  }
  std::string err;
  int rc;
  if (on_device) {
    rc = ifmm::fmm_gmres(h, P ? &P->h : nullptr, b, x, tol, restart, maxit, iters, relres, err);
  } else {
    Staged st;
    if (hipMalloc((void**)&st.d, (size_t)(2 * h.N) * 8) != hipSuccess) return fail(IFMM_ENOMEM, "device allocation failed");
    if (hipMemcpy(st.d, b, (size_t)h.N * 8, hipMemcpyHostToDevice) != hipSuccess) return fail(IFMM_EDEVICE, "copy failed");
    rc = ifmm::fmm_gmres(h, P ? &P->h : nullptr, st.d, st.d + h.N, tol, restart, maxit, iters, relres, err);
    if (!rc && hipMemcpy(x, st.d + h.N, (size_t)h.N * 8, hipMemcpyDeviceToHost) != hipSuccess)
      return fail(IFMM_EDEVICE, "copy failed");
  }
  if (rc) return fail(rc, err);
  if (!(*relres <= tol)) return fail(IFMM_ENOCONV, "GMRES did not reach the tolerance");
  return IFMM_OK;
}

ifmm_status bd_build(const double* points, int64_t n, const double* weights, const double* diag, double diag_scalar,
                     int32_t level, int32_t leaf_max, void* stream, bd_handle** out) {
  ifmm::set_error("");
  if (!out) return fail(IFMM_EINVAL, "out is NULL");
  *out = nullptr;
  if (!points) return fail(IFMM_EINVAL, "points is NULL");
  if (n < 1) return fail(IFMM_EINVAL, "n must be >= 1");
  if (level != 0 && (level < 2 || level > 10)) return fail(IFMM_EINVAL, "level must be 0 (from leaf_max) or in [2, 10]");
  if (leaf_max < 1) return fail(IFMM_EINVAL, "leaf_max must be >= 1");
  if (!diag && !std::isfinite(diag_scalar)) return fail(IFMM_ENONFINITE, "non-finite diag_scalar");
  bd_handle* B = new (std::nothrow) bd_handle();
  if (!B) return fail(IFMM_ENOMEM, "host allocation failed");
  B->h.stream = (hipStream_t)stream;
  std::string err;
  int rc;
  try {
    rc = ifmm::bd_setup(B->h, points, n, weights, diag, diag_scalar, level, leaf_max, err);
  } catch (const std::bad_alloc&) {
    rc = IFMM_ENOMEM;
    err = "host allocation failed";
  }
  if (rc) {
    ifmm::bd_release(B->h);
    delete B;
    return fail(rc, err);
  }
  *out = B;
  return IFMM_OK;
}

ifmm_status bd_apply(bd_handle* B, const double* r, double* z, int32_t on_device) {
  ifmm::set_error("");
  if (!B || !r || !z) return fail(IFMM_EINVAL, "bad arguments");
  if (r == z) return fail(IFMM_EINVAL, "r and z may not alias");
  ifmm::BdHandle& h = B->h;
  std::string err;
  int rc;
  if (on_device) {
    rc = ifmm::bd_apply(h, r, z, err);
  } else {
    Staged st;
    if (hipMalloc((void**)&st.d, (size_t)(2 * h.N) * 8) != hipSuccess) return fail(IFMM_ENOMEM, "device allocation failed");
    if (hipMemcpy(st.d, r, (size_t)h.N * 8, hipMemcpyHostToDevice) != hipSuccess) return fail(IFMM_EDEVICE, "copy failed");
    rc = ifmm::bd_apply(h, st.d, st.d + h.N, err);
    if (!rc && hipMemcpy(z, st.d + h.N, (size_t)h.N * 8, hipMemcpyDeviceToHost) != hipSuccess)
      return fail(IFMM_EDEVICE, "copy failed");
  }
  if (rc) return fail(rc, err);
  return IFMM_OK;
}

ifmm_status fmm_gmres_bd(fmm_handle* F, const double* b, bd_handle* B, double tol, int32_t restart, int32_t maxit,
                         double* x, int32_t on_device, int32_t* iters, double* relres) {
  ifmm::set_error("");
  if (!F || !B || !b || !x || !iters || !relres) return fail(IFMM_EINVAL, "bad arguments");
  if (restart < 1 || restart > 1000) return fail(IFMM_EINVAL, "restart must lie in [1, 1000]");
  if (maxit < 0) return fail(IFMM_EINVAL, "maxit must be >= 0");
  if (!(tol > 0.0)) return fail(IFMM_EINVAL, "tol must be > 0");
  if (b == x) return fail(IFMM_EINVAL, "b and x may not alias");
  ifmm::FmmHandle& h = F->h;
  if (B->h.N != h.N) return fail(IFMM_EINVAL, "preconditioner size differs from the FMM's");
  std::string err;
  int rc;
  if (on_device) {
    rc = ifmm::fmm_gmres(h, nullptr, b, x, tol, restart, maxit, iters, relres, err, &B->h);
  } else {
    Staged st;
    if (hipMalloc((void**)&st.d, (size_t)(2 * h.N) * 8) != hipSuccess) return fail(IFMM_ENOMEM, "device allocation failed");
    if (hipMemcpy(st.d, b, (size_t)h.N * 8, hipMemcpyHostToDevice) != hipSuccess) return fail(IFMM_EDEVICE, "copy failed");
    rc = ifmm::fmm_gmres(h, nullptr, st.d, st.d + h.N, tol, restart, maxit, iters, relres, err, &B->h);
    if (!rc && hipMemcpy(x, st.d + h.N, (size_t)h.N * 8, hipMemcpyDeviceToHost) != hipSuccess)
      return fail(IFMM_EDEVICE, "copy failed");
  }
  if (rc) return fail(rc, err);
  if (!(*relres <= tol)) return fail(IFMM_ENOCONV, "GMRES did not reach the tolerance");
  return IFMM_OK;
}

ifmm_status bd_stats(const bd_handle* B, char* json, int64_t cap) {
  if (!B || !json || cap < 1) return fail(IFMM_EINVAL, "bad arguments");
  const ifmm::BdHandle& h = B->h;
  std::snprintf(json, (size_t)cap, "{\"N\":%lld,\"level\":%d,\"boxes\":%d,\"largest_box\":%d,\"block_bytes\":%lld,\"t_build\":%.6f}",
                (long long)h.N, h.tree.depth, h.nbox, h.nmax, (long long)(h.block_doubles * 8), h.t_build);
  return IFMM_OK;
}

void bd_destroy(bd_handle* B) {
  if (!B) return;
  ifmm::bd_release(B->h);
  delete B;
}

ifmm_status fmm_stats(const fmm_handle* F, char* json, int64_t cap) {
  if (!F || !json || cap < 1) return fail(IFMM_EINVAL, "bad arguments");
  const ifmm::FmmHandle& h = F->h;
  char buf[512];
  std::snprintf(buf, sizeof buf,
                "{\"N\":%lld,\"depth\":%d,\"K\":%d,\"m2l_pairs\":%lld,\"m2l_flops\":%.6e,\"matvecs\":%lld,"
                "\"t_matvec\":%.6f}",
                (long long)h.N, h.tree.depth, h.K, (long long)h.npairs, h.flops_m2l, (long long)h.matvecs, h.t_matvec);
  std::snprintf(json, (size_t)cap, "%s", buf);
  return IFMM_OK;
}

void fmm_destroy(fmm_handle* F) {
  if (!F) return;
  ifmm::fmm_release(F->h);
  delete F;
}

ifmm_status fmbem_gmres(const double* centroids, const double* areas, const double* self_terms, int64_t n,
                        const double* f, ifmm_handle* P, int32_t fmm_cheb_order, double tol, int32_t restart,
                        int32_t maxit, double* sol, int32_t* iters, double* relres) {
  if (!centroids || !areas || !self_terms || !f || !sol) return fail(IFMM_EINVAL, "bad arguments");
  fmm_handle* F = nullptr;
  ifmm_status st = fmm_build(centroids, n, areas, self_terms, 0.0, fmm_cheb_order, 64, nullptr, &F);
  if (st != IFMM_OK) return st;
  st = fmm_gmres(F, f, P, tol, restart, maxit, sol, 0, iters, relres);
  const std::string msg = ifmm::get_error();
  fmm_destroy(F);
  if (st != IFMM_OK) ifmm::set_error(msg);
  return st;
}

}  // extern "C"
