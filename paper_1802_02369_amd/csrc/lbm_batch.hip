// C ABI for batches of lattices, hipGraph capture of batched runs, and the
// autotuner (with its JSON cache) of both the single-lattice and the batched
// blocked kernels.  Declared in include/lbm.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/lbm.h"
#include "lbm_internal.hpp"

using namespace lbm;

namespace {

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

namespace {

// Workspace layout (byte offsets) of a batch for a tile count.
struct Layout {
  size_t state2, consts, offs, tiles, diag, backup, total;
};

Layout layout(const lbm_batch* b, int64_t ntiles, bool backup) {
  Layout L{};
  size_t o = 0;
  L.state2 = o;
  o = align256(o + sizeof(double) * 6 * (size_t)b->n_total);
  L.consts = o;
  o = align256(o + sizeof(Consts) * (size_t)b->n_inst);
  L.offs = o;
  o = align256(o + sizeof(int64_t) * (size_t)(b->n_inst + 1));
  L.tiles = o;
  o = align256(o + sizeof(TileRef) * (size_t)std::max<int64_t>(ntiles, 1));
  L.diag = o;
  o = align256(o + sizeof(double) * 8 * (size_t)b->n_inst);
  L.backup = o;
  if (backup) o = align256(o + sizeof(double) * 6 * (size_t)b->n_total);
  L.total = o;
  return L;
}

template <class T>
T* at(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

int check_batch_ws(const lbm_batch* b, const void* ws, size_t ws_bytes) {
  if (!b || !ws) return set_err(LBM_EINVAL, "NULL argument");
  if (b->prep_ws != ws || !same_tuning(b->prep_tune, b->tune))
    return set_err(LBM_EINVAL,
                   "workspace not prepared for this tuning: call "
                   "lbm_batch_prepare");
  if (ws_bytes < layout(b, b->prep_tiles, false).total)
    return set_err(LBM_EWORKSPACE, "workspace too small");
  return LBM_OK;
}

// Launch sequence of a batched run on stream s.
int enqueue_batch(lbm_batch* b, double* f, void* ws, int64_t nsteps,
                  hipStream_t s) {
  const Layout L = layout(b, b->prep_tiles, false);
  const Consts* cs = at<Consts>(ws, L.consts);
  const int64_t* offs = at<int64_t>(ws, L.offs);
  const TileRef* tiles = at<TileRef>(ws, L.tiles);
  double* a = f;
  double* w = at<double>(ws, L.state2);
  const int H = 2 * b->tune.steps_per_launch;
  int64_t launches = 0;
  for (int k : split_steps(nsteps, b->tune.steps_per_launch)) {
    int rc = launch_batch_tile(cs, offs, tiles, b->prep_tiles, a, w,
                               b->n_total, b->tune.nodes_per_lane, H, k,
                               b->tune.waves_per_group, b->eq_class(), s);
    if (rc) return rc;
    std::swap(a, w);
    ++launches;
  }
  if (launches & 1)
    return hip_check(hipMemcpyAsync(f, at<double>(ws, L.state2),
                                    sizeof(double) * 6 * b->n_total,
                                    hipMemcpyDeviceToDevice, s),
                     "hipMemcpyAsync");
  return LBM_OK;
}

}  // namespace

namespace lbm {
void drop_adjoint_graph(lbm_batch* b);
}

namespace {

void drop_graph(lbm_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  b->exec = nullptr;
  b->g_f = nullptr;
  b->g_ws = nullptr;
  b->g_nsteps = -1;
}

// --------------------------------------------------------- tuning cache --

std::map<std::string, lbm_tuning> read_cache(const char* path) {
  std::map<std::string, lbm_tuning> m;
  FILE* fp = path ? std::fopen(path, "r") : nullptr;
  if (!fp) return m;
  std::string text;
  char buf[4096];
  size_t r;
  while ((r = std::fread(buf, 1, sizeof buf, fp)) > 0) text.append(buf, r);
  std::fclose(fp);
  // entries: "key": {"kernel": a, "P": b, "K": c, "W": d}
  size_t pos = 0;
  while ((pos = text.find('"', pos)) != std::string::npos) {
    const size_t end = text.find('"', pos + 1);
    if (end == std::string::npos) break;
    const std::string key = text.substr(pos + 1, end - pos - 1);
    const size_t brace = text.find('{', end);
    const size_t close = text.find('}', end);
    if (brace == std::string::npos || close == std::string::npos ||
        brace > close) {
      pos = end + 1;
      continue;
    }
    lbm_tuning t{};
    const std::string body = text.substr(brace, close - brace + 1);
    if (std::sscanf(body.c_str(),
                    "{ \"kernel\" : %d , \"P\" : %d , \"K\" : %d , \"W\" : %d }",
                    &t.kernel, &t.nodes_per_lane, &t.steps_per_launch,
                    &t.waves_per_group) == 4 &&
        check_tuning(&t) == LBM_OK)
      m[key] = t;
    pos = close + 1;
  }
  return m;
}

}  // namespace

namespace lbm {

bool tune_cache_get(const char* path, const std::string& key, lbm_tuning* t) {
  auto m = read_cache(path);
  auto it = m.find(key);
  if (it == m.end()) return false;
  *t = it->second;
  return true;
}

void tune_cache_put(const char* path, const std::string& key,
                    const lbm_tuning& t) {
  if (!path) return;
  auto m = read_cache(path);
  m[key] = t;
  const std::string tmp = std::string(path) + ".tmp";
  FILE* fp = std::fopen(tmp.c_str(), "w");
  if (!fp) return;
  std::fprintf(fp, "{\n");
  size_t i = 0;
  for (const auto& kv : m) {
    std::fprintf(fp, "  \"%s\": {\"kernel\": %d, \"P\": %d, \"K\": %d, \"W\": %d}%s\n",
                 kv.first.c_str(), kv.second.kernel, kv.second.nodes_per_lane,
                 kv.second.steps_per_launch, kv.second.waves_per_group,
                 ++i < m.size() ? "," : "");
  }
  std::fprintf(fp, "}\n");
  std::fclose(fp);
  std::rename(tmp.c_str(), path);
}

std::string gpu_arch_name() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return "unknown";
  std::string a = prop.gcnArchName;
  const size_t colon = a.find(':');
  return colon == std::string::npos ? a : a.substr(0, colon);
}

}  // namespace lbm

namespace {

int log2_class(double x) { return x > 1 ? (int)std::lround(std::log2(x)) : 0; }

// Generation of the tile kernels, the last component of every tuning-cache
// key: entries measured on kernels of another generation are not reused.
constexpr const char* kKernelGeneration = "/k3";

// Times `run(t)` for each candidate on the state f, restoring f from
// `backup` before each run and at the end; returns the fastest.
template <class Prepare, class Run>
int autotune_impl(hipStream_t s, double* f, double* backup, size_t bytes,
                  int64_t probe, const std::vector<lbm_tuning>& cands,
                  Prepare prepare, Run run, lbm_tuning* best) {
  int rc = hip_check(hipMemcpyAsync(backup, f, bytes, hipMemcpyDeviceToDevice, s),
                     "hipMemcpyAsync");
  if (rc) return rc;
  hipEvent_t e0, e1;
  if ((rc = hip_check(hipEventCreate(&e0), "hipEventCreate"))) return rc;
  if ((rc = hip_check(hipEventCreate(&e1), "hipEventCreate"))) {
    (void)hipEventDestroy(e0);
    return rc;
  }
  float best_ms = INFINITY;
  for (const lbm_tuning& t : cands) {
    if ((rc = prepare(t))) break;
    if ((rc = run(t, probe))) break;  // warm-up
    if ((rc = hip_check(hipMemcpyAsync(f, backup, bytes,
                                       hipMemcpyDeviceToDevice, s),
                        "hipMemcpyAsync")))
      break;
    (void)hipEventRecord(e0, s);
    if ((rc = run(t, probe))) break;
    (void)hipEventRecord(e1, s);
    if ((rc = hip_check(hipEventSynchronize(e1), "hipEventSynchronize")))
      break;
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (ms < best_ms) {
      best_ms = ms;
      *best = t;
    }
    if ((rc = hip_check(hipMemcpyAsync(f, backup, bytes,
                                       hipMemcpyDeviceToDevice, s),
                        "hipMemcpyAsync")))
      break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) {
    (void)hipMemcpyAsync(f, backup, bytes, hipMemcpyDeviceToDevice, s);
    return rc;
  }
  return hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
}

}  // namespace

extern "C" {

int lbm_autotune(lbm_handle* h, double* f, void* ws, size_t ws_bytes,
                 int64_t probe_steps, const char* cache_path, lbm_tuning* out) {
  if (!h || !f || !ws) return set_err(LBM_EINVAL, "NULL argument");
  if (probe_steps < 1) return set_err(LBM_EINVAL, "probe_steps must be >= 1");
  if (ws_bytes < lbm_workspace_bytes(h, LBM_WS_TUNE))
    return set_err(LBM_EWORKSPACE, "autotune needs LBM_WS_TUNE workspace");
  const size_t sbytes = sizeof(double) * 6 * (size_t)h->n;
  if (overlaps(f, sbytes, ws, ws_bytes))
    return set_err(LBM_EINVAL, "f and ws overlap");
  const std::string key =
      gpu_arch_name() + "/single/n" + std::to_string(log2_class((double)h->n)) +
      kKernelGeneration;
  lbm_tuning best{};
  if (!tune_cache_get(cache_path, key, &best)) {
    std::vector<lbm_tuning> cands = tuning_candidates();
    cands.push_back(lbm_tuning{LBM_KERNEL_PLAIN, 0, 1, 1});
    double* backup = static_cast<double*>(ws) + 6 * h->n + diag_ws_doubles();
    const size_t step_ws = lbm_workspace_bytes(h, LBM_WS_STEP);
    int rc = autotune_impl(
        h->stream, f, backup, sbytes, probe_steps, cands,
        [&](const lbm_tuning& t) { h->tune = t; return LBM_OK; },
        [&](const lbm_tuning&, int64_t k) {
          return lbm_step(h, f, ws, step_ws, k);
        },
        &best);
    if (rc) return rc;
    tune_cache_put(cache_path, key, best);
  }
  h->tune = best;
  if (out) *out = best;
  return LBM_OK;
}

int lbm_batch_init(lbm_batch** b, int64_t n_inst, const int64_t* offsets,
                   const lbm_params* params, void* stream) {
  if (!b) return set_err(LBM_EINVAL, "batch pointer is NULL");
  *b = nullptr;
  if (n_inst < 1 || n_inst > (int64_t(1) << 30) || !offsets || !params)
    return set_err(LBM_EINVAL, "need n_inst >= 1 and host offsets/params");
  if (offsets[0] != 0) return set_err(LBM_EINVAL, "offsets[0] must be 0");
  for (int64_t i = 0; i < n_inst; ++i)
    if (offsets[i + 1] - offsets[i] < 3)
      return set_err(LBM_EINVAL,
                     "lattice %lld has length %lld (offsets must increase by "
                     ">= 3)",
                     (long long)i, (long long)(offsets[i + 1] - offsets[i]));
  if (offsets[n_inst] > kMaxNodes)
    return set_err(LBM_EINVAL, "batch of %lld nodes exceeds 2^36",
                   (long long)offsets[n_inst]);
  lbm_batch* x = new lbm_batch;
  x->n_inst = n_inst;
  x->n_total = offsets[n_inst];
  x->offsets.assign(offsets, offsets + n_inst + 1);
  x->params.assign(params, params + n_inst);
  x->consts.resize(n_inst);
  for (int64_t i = 0; i < n_inst; ++i) {
    int rc = make_consts(&params[i], &x->consts[i]);
    if (rc) {
      delete x;
      return set_err(rc, "lattice %lld: %s", (long long)i, g_err.c_str());
    }
  }
  x->stream = (hipStream_t)stream;
  x->tune = default_tuning(x->n_total / n_inst, x->n_total);
  *b = x;
  return LBM_OK;
}

void lbm_batch_destroy(lbm_batch* b) {
  if (!b) return;
  drop_graph(b);
  lbm::drop_adjoint_graph(b);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  delete b;
}

int lbm_batch_set_stream(lbm_batch* b, void* stream) {
  if (!b) return set_err(LBM_EINVAL, "batch is NULL");
  b->stream = (hipStream_t)stream;
  return LBM_OK;
}

int lbm_batch_set_tuning(lbm_batch* b, const lbm_tuning* t) {
  if (!b) return set_err(LBM_EINVAL, "batch is NULL");
  int rc = check_tuning(t);
  if (rc) return rc;
  if (t->kernel == LBM_KERNEL_PLAIN)
    return set_err(LBM_EINVAL, "batches run the blocked kernel only");
  b->tune = *t;
  b->tune.kernel = LBM_KERNEL_BLOCKED;
  return LBM_OK;
}

int lbm_batch_get_tuning(const lbm_batch* b, lbm_tuning* t) {
  if (!b || !t) return set_err(LBM_EINVAL, "NULL argument");
  *t = b->tune;
  return LBM_OK;
}

int64_t lbm_batch_total_nodes(const lbm_batch* b) { return b ? b->n_total : 0; }

size_t lbm_batch_workspace_bytes(const lbm_batch* b, int kind) {
  if (!b) return 0;
  if (kind == LBM_WS_STEP) return layout(b, b->count_tiles(b->tune), false).total;
  if (kind == LBM_WS_TUNE) {
    int64_t mx = b->count_tiles(b->tune);
    for (const lbm_tuning& t : tuning_candidates())
      mx = std::max(mx, b->count_tiles(t));
    return layout(b, mx, true).total;
  }
  return 0;
}

int lbm_batch_prepare(lbm_batch* b, void* ws, size_t ws_bytes) {
  if (!b || !ws) return set_err(LBM_EINVAL, "NULL argument");
  const int64_t ntiles = b->count_tiles(b->tune);
  const Layout L = layout(b, ntiles, false);
  if (ws_bytes < L.total)
    return set_err(LBM_EWORKSPACE, "workspace of %zu bytes, need %zu", ws_bytes,
                   L.total);
  std::vector<TileRef> tiles;
  tiles.reserve(ntiles);
  const int64_t out = tile_width(b->tune) - 4 * (int64_t)b->tune.steps_per_launch;
  for (int64_t i = 0; i < b->n_inst; ++i) {
    const int64_t n = b->offsets[i + 1] - b->offsets[i];
    for (int64_t t = 0; t * out < n; ++t)
      tiles.push_back(TileRef{(int32_t)i, (int32_t)t});
  }
  int rc = hip_check(hipMemcpyAsync(at<char>(ws, L.consts), b->consts.data(),
                                    sizeof(Consts) * b->n_inst,
                                    hipMemcpyHostToDevice, b->stream),
                     "hipMemcpyAsync");
  if (!rc)
    rc = hip_check(hipMemcpyAsync(at<char>(ws, L.offs), b->offsets.data(),
                                  sizeof(int64_t) * (b->n_inst + 1),
                                  hipMemcpyHostToDevice, b->stream),
                   "hipMemcpyAsync");
  if (!rc)
    rc = hip_check(hipMemcpyAsync(at<char>(ws, L.tiles), tiles.data(),
                                  sizeof(TileRef) * tiles.size(),
                                  hipMemcpyHostToDevice, b->stream),
                   "hipMemcpyAsync");
  if (!rc) rc = hip_check(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
  if (rc) return rc;
  b->prep_ws = ws;
  b->prep_tune = b->tune;
  b->prep_tiles = (int64_t)tiles.size();
  return LBM_OK;
}

int lbm_batch_set_equilibrium(lbm_batch* b, const double* rho, const double* J,
                              const double* zeta, double* f, void* ws,
                              size_t ws_bytes) {
  if (!rho || !J || !zeta || !f) return set_err(LBM_EINVAL, "NULL argument");
  int rc = check_batch_ws(b, ws, ws_bytes);
  if (rc) return rc;
  const Layout L = layout(b, b->prep_tiles, false);
  return launch_batch_equilibrium(at<Consts>(ws, L.consts),
                                  at<int64_t>(ws, L.offs), b->n_inst, rho, J,
                                  zeta, f, b->n_total, b->stream);
}

int lbm_batch_run(lbm_batch* b, double* f, void* ws, size_t ws_bytes,
                  int64_t nsteps, int use_graph) {
  int rc = check_batch_ws(b, ws, ws_bytes);
  if (rc) return rc;
  if (!f) return set_err(LBM_EINVAL, "f is NULL");
  if (nsteps < 0) return set_err(LBM_EINVAL, "nsteps must be >= 0");
  if (overlaps(f, sizeof(double) * 6 * b->n_total, ws, ws_bytes))
    return set_err(LBM_EINVAL, "f and ws overlap");
  if (((uintptr_t)f | (uintptr_t)ws) & 7)
    return set_err(LBM_EINVAL, "f and ws must be 8-byte aligned");
  if (nsteps == 0) return LBM_OK;
  if (!use_graph) return enqueue_batch(b, f, ws, nsteps, b->stream);
  if (!(b->exec && b->g_f == f && b->g_ws == ws && b->g_nsteps == nsteps &&
        same_tuning(b->g_tune, b->tune))) {
    drop_graph(b);
    if (!b->cap &&
        (rc = hip_check(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking),
                        "hipStreamCreate")))
      return rc;
    if ((rc = hip_check(hipStreamBeginCapture(b->cap,
                                              hipStreamCaptureModeThreadLocal),
                        "hipStreamBeginCapture")))
      return rc;
    const int rc_enq = enqueue_batch(b, f, ws, nsteps, b->cap);
    hipGraph_t graph = nullptr;
    rc = hip_check(hipStreamEndCapture(b->cap, &graph), "hipStreamEndCapture");
    if (rc_enq) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc_enq;
    }
    if (rc) return rc;
    rc = hip_check(hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0),
                   "hipGraphInstantiate");
    (void)hipGraphDestroy(graph);
    if (rc) {
      b->exec = nullptr;
      return rc;
    }
    b->g_f = f;
    b->g_ws = ws;
    b->g_nsteps = nsteps;
    b->g_tune = b->tune;
  }
  return hip_check(hipGraphLaunch(b->exec, b->stream), "hipGraphLaunch");
}

int lbm_batch_moments(lbm_batch* b, const double* f, double* m, void* ws,
                      size_t ws_bytes) {
  int rc = check_batch_ws(b, ws, ws_bytes);
  if (rc) return rc;
  if (!f || !m) return set_err(LBM_EINVAL, "NULL argument");
  if (overlaps(f, sizeof(double) * 6 * b->n_total, m, sizeof(double) * 6 * b->n_total))
    return set_err(LBM_EINVAL, "f and m overlap");
  const Layout L = layout(b, b->prep_tiles, false);
  return launch_batch_moments(at<Consts>(ws, L.consts), at<int64_t>(ws, L.offs),
                              b->n_inst, f, m, b->n_total, b->stream);
}

int lbm_batch_diagnostics(lbm_batch* b, const double* f, void* ws,
                          size_t ws_bytes, double* out) {
  int rc = check_batch_ws(b, ws, ws_bytes);
  if (rc) return rc;
  if (!f || !out) return set_err(LBM_EINVAL, "NULL argument");
  const Layout L = layout(b, b->prep_tiles, false);
  double* d = at<double>(ws, L.diag);
  rc = launch_batch_diag(at<Consts>(ws, L.consts), at<int64_t>(ws, L.offs),
                         b->n_inst, f, b->n_total, d, b->stream);
  if (!rc)
    rc = hip_check(hipMemcpyAsync(out, d, sizeof(double) * 8 * b->n_inst,
                                  hipMemcpyDeviceToHost, b->stream),
                   "hipMemcpyAsync");
  if (!rc) rc = hip_check(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
  if (rc) return rc;
  for (int64_t i = 0; i < b->n_inst; ++i)
    if (out[8 * i + 6] > 0 || out[8 * i + 7] > 0)
      return set_err(LBM_ENONFINITE, "lattice %lld is non-finite or non-physical",
                     (long long)i);
  return LBM_OK;
}

int lbm_batch_autotune(lbm_batch* b, double* f, void* ws, size_t ws_bytes,
                       int64_t probe_steps, const char* cache_path,
                       lbm_tuning* out) {
  if (!b || !f || !ws) return set_err(LBM_EINVAL, "NULL argument");
  if (probe_steps < 1) return set_err(LBM_EINVAL, "probe_steps must be >= 1");
  if (ws_bytes < lbm_batch_workspace_bytes(b, LBM_WS_TUNE))
    return set_err(LBM_EWORKSPACE, "autotune needs LBM_WS_TUNE workspace");
  const double mean_len = (double)b->n_total / (double)b->n_inst;
  const std::string key = gpu_arch_name() + "/batch/N" +
                          std::to_string(log2_class((double)b->n_total)) + "/L" +
                          std::to_string(log2_class(mean_len)) + kKernelGeneration;
  lbm_tuning best = b->tune;
  if (!tune_cache_get(cache_path, key, &best)) {
    int64_t mx = 0;
    for (const lbm_tuning& t : tuning_candidates())
      mx = std::max(mx, b->count_tiles(t));
    double* backup = at<double>(ws, layout(b, mx, true).backup);
    const size_t sbytes = sizeof(double) * 6 * (size_t)b->n_total;
    int rc = autotune_impl(
        b->stream, f, backup, sbytes, probe_steps, tuning_candidates(),
        [&](const lbm_tuning& t) {
          b->tune = t;
          return lbm_batch_prepare(b, ws, ws_bytes);
        },
        [&](const lbm_tuning&, int64_t k) {
          return lbm_batch_run(b, f, ws, ws_bytes, k, 0);
        },
        &best);
    if (rc) return rc;
    tune_cache_put(cache_path, key, best);
  }
  b->tune = best;
  int rc = lbm_batch_prepare(b, ws, ws_bytes);
  if (rc) return rc;
  if (out) *out = best;
  return LBM_OK;
}

}  // extern "C"
