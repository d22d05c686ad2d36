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

static_assert(kResidentMin == LBM_RESIDENT_MIN && kResidentMax == LBM_RESIDENT_MAX,
              "resident lattice bounds of the header");

namespace {

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

namespace {

// Workspace layout (byte offsets) of a batch for a tile count.
struct Layout {
  size_t state2, consts, offs, tiles, res_items, res_first, diag, rec, backup,
      total;
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
  L.res_items = o;  // resident lattices and their workgroups
  o = align256(o + sizeof(ResidentItem) * (size_t)b->n_inst);
  L.res_first = o;
  o = align256(o + sizeof(int32_t) * (size_t)(b->n_inst + 1));
  L.diag = o;
  o = align256(o + sizeof(double) * 8 * (size_t)b->n_inst);
  L.rec = o;  // failure record of LBM_CHECK_FINITE
  o = align256(o + sizeof(unsigned long long));
  L.backup = o;
  if (backup) o = align256(o + sizeof(double) * 6 * (size_t)b->n_total);
  L.total = o;
  return L;
}

template <class T>
T* at(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

// With LBM_CHECK_FINITE on some lattice: waits for the run and turns the
// failure record into LBM_ENONFINITE.
int batch_check_result(lbm_batch* b, void* ws) {
  if (!b->check_finite()) return LBM_OK;
  unsigned long long key = 0;
  const Layout L = layout(b, b->run_tiles(), false);
  int rc = read_check_record(at<unsigned long long>(ws, L.rec), b->stream, &key);
  if (rc || key == ~0ull) return rc;
  const long long steps = (long long)(key >> 31);
  return set_err(LBM_ENONFINITE,
                 "non-finite or non-physical state (rho <= 0 or T <= 0) after "
                 "%lld%s time steps: first failing lattice %lld",
                 steps, steps == kCheckMaxStepsB ? " or more" : "",
                 (long long)(key & ((1ull << 31) - 1)));
}

int check_batch_ws(const lbm_batch* b, const void* ws, size_t ws_bytes) {
  if (!b || !ws) return set_err(LBM_EINVAL, "NULL argument");
  if (b->prep_ws != ws || !same_tuning(b->prep_tune, b->tune) ||
      !same_tunings(b->prep_group_tune, b->group_tune) ||
      b->prep_group_of != b->group_of ||
      b->prep_resident_mode != b->resident_mode)
    return set_err(LBM_EINVAL,
                   "workspace not prepared for this tuning: call "
                   "lbm_batch_prepare");
  if (ws_bytes < layout(b, b->run_tiles(), false).total)
    return set_err(LBM_EWORKSPACE, "workspace too small");
  return LBM_OK;
}

// Launches of nsteps steps of the tiles [first, first + ntiles) of the table
// with tuning t on stream s (ping-pong between f and the workspace state).
// An odd number of launches (nsteps = 1, or K = 1 and nsteps odd) leaves
// the result in the workspace state: a copy of those tiles' nodes brings it
// into f.
int enqueue_tiles(lbm_batch* b, const Layout& L, void* ws, double* f,
                  int64_t nsteps, const lbm_tuning& t, int64_t first,
                  int64_t ntiles, hipStream_t s) {
  const Consts* cs = at<Consts>(ws, L.consts);
  const int64_t* offs = at<int64_t>(ws, L.offs);
  const TileRef* tiles = at<TileRef>(ws, L.tiles) + first;
  double* a = f;
  double* w = at<double>(ws, L.state2);
  const int H = 2 * t.steps_per_launch;
  const bool check = b->check_finite();
  const int out = (int)(tile_width(t) - 2 * H);
  int64_t done = 0, launches = 0;
  for (int k : split_steps(nsteps, t.steps_per_launch)) {
    int rc = launch_batch_tile(cs, offs, tiles, ntiles, a, w, b->n_total,
                               t.nodes_per_lane, H, k, t.waves_per_group,
                               b->eq_class(), s);
    done += k;
    if (!rc && check)
      rc = launch_batch_check(cs, offs, tiles, ntiles, w, b->n_total, out,
                              done, at<unsigned long long>(ws, L.rec), s);
    if (rc) return rc;
    std::swap(a, w);
    ++launches;
  }
  if (launches & 1)
    return launch_batch_copy_tiles(offs, tiles, ntiles, out, a, f, b->n_total, s);
  return LBM_OK;
}

// Launch sequence of a batched run on stream s.  With shape groups, group 0
// runs on s and group g > 0 on its own stream, forked from s and joined back
// to it (inside a graph capture the side streams join the capture).  Every
// sequence leaves its lattices' result in f.
int enqueue_batch(lbm_batch* b, double* f, void* ws, int64_t nsteps,
                  hipStream_t s) {
  const Layout L = layout(b, b->run_tiles(), false);
  int rc = b->check_finite()
               ? launch_check_reset(at<unsigned long long>(ws, L.rec), s)
               : LBM_OK;
  if (rc) return rc;
  // Resident lattices: one launch for all the steps, in place in f, on a
  // side stream forked from s and joined back before the end (also inside a
  // graph); no tile reads or writes their nodes.
  const int64_t nres = (int64_t)b->prep_res_items.size();
  const int64_t nwg = nres ? (int64_t)b->prep_res_first.size() - 1 : 0;
  if (nres) {
    rc = hip_check(hipEventRecord(b->res_events[0], s), "hipEventRecord");
    if (!rc)
      rc = hip_check(hipStreamWaitEvent(b->res_stream, b->res_events[0], 0),
                     "hipStreamWaitEvent");
    if (rc) return rc;
    const Consts* cs = at<Consts>(ws, L.consts);
    const int64_t* offs = at<int64_t>(ws, L.offs);
    const ResidentItem* items = at<ResidentItem>(ws, L.res_items);
    // at most kResidentMaxSteps steps per launch, so that no launch holds
    // the chip for long; each chunk is checked when asked
    for (int64_t done = 0; done < nsteps && !rc;) {
      const int64_t T = std::min<int64_t>(kResidentMaxSteps, nsteps - done);
      rc = launch_batch_resident(cs, offs, items, at<int32_t>(ws, L.res_first),
                                 nwg, f, f, b->n_total, T, b->eq_class(),
                                 b->res_stream);
      done += T;
      if (!rc && b->check_finite())
        rc = launch_batch_check_lattices(cs, offs, items, nres, f, b->n_total,
                                         done, at<unsigned long long>(ws, L.rec),
                                         b->res_stream);
    }
    // join even after a failure, so that a capture ends
    const int r1 = hip_check(hipEventRecord(b->res_events[1], b->res_stream),
                             "hipEventRecord");
    if (!rc) rc = r1;
    if (rc) {
      (void)hipStreamWaitEvent(s, b->res_events[1], 0);
      return rc;
    }
  }
  if (b->prep_tiles == 0) {
    // every lattice is resident
  } else if (b->prep_group_tune.empty()) {
    rc = enqueue_tiles(b, L, ws, f, nsteps, b->tune, 0, b->prep_tiles, s);
  } else {
    const size_t ng = b->prep_group_tune.size();
    rc = hip_check(hipEventRecord(b->gevents[0], s), "hipEventRecord");
    for (size_t g = 1; g < ng && !rc; ++g)
      rc = hip_check(hipStreamWaitEvent(b->gstreams[g - 1], b->gevents[0], 0),
                     "hipStreamWaitEvent");
    for (size_t g = 0; g < ng && !rc; ++g) {
      const hipStream_t sg = g == 0 ? s : b->gstreams[g - 1];
      const int64_t first = b->prep_group_first[g];
      rc = enqueue_tiles(b, L, ws, f, nsteps, b->prep_group_tune[g], first,
                         b->prep_group_first[g + 1] - first, sg);
    }
    // join every side stream even after a failure, so that a capture ends
    for (size_t g = 1; g < ng; ++g) {
      const int r1 = hip_check(hipEventRecord(b->gevents[g], b->gstreams[g - 1]),
                               "hipEventRecord");
      const int r2 = hip_check(hipStreamWaitEvent(s, b->gevents[g], 0),
                               "hipStreamWaitEvent");
      if (!rc) rc = r1 ? r1 : r2;
    }
  }
  if (nres) {
    const int r = hip_check(hipStreamWaitEvent(s, b->res_events[1], 0),
                            "hipStreamWaitEvent");
    if (!rc) rc = r;
  }
  return rc;
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
  b->g_group_tune.clear();
  b->g_group_of.clear();
}

// --------------------------------------------------------- tuning cache --

// A tuning-cache entry: the shape and, for batches, optional shape groups
// with their measured time per computed node-update.
struct CacheEntry {
  lbm_tuning t{};
  std::vector<lbm_tuning> gshape;
  std::vector<double> gcost;
  int resident = -1;  // batch entries: the resident mode the search kept
};

std::map<std::string, CacheEntry> read_cache(const char* path) {
  std::map<std::string, CacheEntry> m;
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
    CacheEntry e;
    lbm_tuning& t = e.t;
    const std::string body = text.substr(brace, close - brace + 1);
    if (std::sscanf(body.c_str(),
                    "{ \"kernel\" : %d , \"P\" : %d , \"K\" : %d , \"W\" : %d",
                    &t.kernel, &t.nodes_per_lane, &t.steps_per_launch,
                    &t.waves_per_group) == 4 &&
        check_tuning(&t) == LBM_OK) {
      // optional "groups": [[P, K, W, seconds per node-update], ...]
      const size_t gp = body.find("\"groups\"");
      size_t q = gp == std::string::npos ? gp : body.find('[', gp);
      if (q != std::string::npos) {
        for (++q;;) {
          const size_t o = body.find('[', q);
          const size_t c = o == std::string::npos ? o : body.find(']', o);
          if (c == std::string::npos) break;
          lbm_tuning g{LBM_KERNEL_BLOCKED, 0, 0, 0};
          double cost = 0;
          if (std::sscanf(body.c_str() + o, "[ %d , %d , %d , %lf ]",
                          &g.nodes_per_lane, &g.steps_per_launch,
                          &g.waves_per_group, &cost) == 4 &&
              check_tuning(&g) == LBM_OK && cost > 0) {
            e.gshape.push_back(g);
            e.gcost.push_back(cost);
          }
          q = c + 1;
        }
        if (e.gshape.size() < 2 || e.gshape.size() > LBM_MAX_GROUPS) {
          e.gshape.clear();
          e.gcost.clear();
        }
      }
      // optional "resident": 0 or 1
      const size_t rp = body.find("\"resident\"");
      int r = -1;
      if (rp != std::string::npos &&
          std::sscanf(body.c_str() + rp, "\"resident\" : %d", &r) == 1 &&
          (r == 0 || r == 1))
        e.resident = r;
      m[key] = e;
    }
    pos = close + 1;
  }
  return m;
}

}  // namespace

namespace lbm {

bool tune_cache_get(const char* path, const std::string& key, lbm_tuning* t,
                    std::vector<lbm_tuning>* gshape, std::vector<double>* gcost,
                    int* resident) {
  auto m = read_cache(path);
  auto it = m.find(key);
  if (it == m.end()) return false;
  *t = it->second.t;
  if (gshape) *gshape = it->second.gshape;
  if (gcost) *gcost = it->second.gcost;
  if (resident && it->second.resident >= 0) *resident = it->second.resident;
  return true;
}

void tune_cache_put(const char* path, const std::string& key,
                    const lbm_tuning& t, const std::vector<lbm_tuning>* gshape,
                    const std::vector<double>* gcost, int resident) {
  if (!path) return;
  auto m = read_cache(path);
  CacheEntry e;
  e.t = t;
  if (gshape && gcost) {
    e.gshape = *gshape;
    e.gcost = *gcost;
  }
  e.resident = resident;
  m[key] = e;
  const std::string tmp = std::string(path) + ".tmp";
  FILE* fp = std::fopen(tmp.c_str(), "w");
  if (!fp) return;
  std::fprintf(fp, "{\n");
  size_t i = 0;
  for (const auto& kv : m) {
    const CacheEntry& x = kv.second;
    std::fprintf(fp, "  \"%s\": {\"kernel\": %d, \"P\": %d, \"K\": %d, \"W\": %d",
                 kv.first.c_str(), x.t.kernel, x.t.nodes_per_lane,
                 x.t.steps_per_launch, x.t.waves_per_group);
    if (!x.gshape.empty()) {
      std::fprintf(fp, ", \"groups\": [");
      for (size_t g = 0; g < x.gshape.size(); ++g)
        std::fprintf(fp, "%s[%d, %d, %d, %.9e]", g ? ", " : "",
                     x.gshape[g].nodes_per_lane, x.gshape[g].steps_per_launch,
                     x.gshape[g].waves_per_group, x.gcost[g]);
      std::fprintf(fp, "]");
    }
    if (x.resident >= 0) std::fprintf(fp, ", \"resident\": %d", x.resident);
    std::fprintf(fp, "}%s\n", ++i < m.size() ? "," : "");
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

// The batch autotuner's shapes: the throughput candidates and the batch's
// default shape (one wavefront, or one node per lane, on small problems).
std::vector<lbm_tuning> batch_candidates(const lbm_batch* b) {
  std::vector<lbm_tuning> v = tuning_candidates();
  const lbm_tuning d =
      default_tuning(b->n_total / b->n_inst, b->n_total, b->eq_class());
  if (std::none_of(v.begin(), v.end(),
                   [&](const lbm_tuning& c) { return same_tuning(c, d); }))
    v.push_back(d);
  return v;
}

// Tile-table size the autotuner may need: any grouping of the candidates,
// i.e. each lattice at its largest tile count, and the current settings.
int64_t tune_tiles(const lbm_batch* b) {
  int64_t mx = 0;
  const std::vector<lbm_tuning> cands = batch_candidates(b);
  for (int64_t i = 0; i < b->n_inst; ++i) {
    int64_t m = 0;
    for (const lbm_tuning& t : cands) m = std::max(m, b->lattice_tiles(i, t));
    mx += m;
  }
  return std::max(mx, std::max(b->run_tiles(), b->count_tiles(b->tune)));
}

// Modelled time of a grouping: lattice i costs work_i(s) * c_s on shape s,
// work_i(s) its lane-nodes per step and c_s a measured time per computed
// node-update; each lattice takes its cheapest shape (written to *of).
// Returns the total.
double assign_groups(const lbm_batch* b, const std::vector<lbm_tuning>& shapes,
                     const std::vector<double>& cost, std::vector<int32_t>* of) {
  double total = 0;
  if (of) of->assign(b->n_inst, 0);
  for (int64_t i = 0; i < b->n_inst; ++i) {
    if (b->resident(i)) continue;  // runs in the resident launch
    double best = INFINITY;
    for (size_t g = 0; g < shapes.size(); ++g) {
      const double c = (double)b->lattice_work(i, shapes[g]) * cost[g];
      if (c < best) {
        best = c;
        if (of) (*of)[i] = (int32_t)g;
      }
    }
    total += best;
  }
  return total;
}

}  // namespace

extern "C" int lbm_batch_set_groups(lbm_batch* b, int32_t n_groups,
                                    const lbm_tuning* shapes,
                                    const int32_t* group_of);

namespace {

// Groups of the shapes gshape with costs gcost for this batch: each lattice on
// its cheapest shape, unused shapes dropped.  Sets them on b.
int apply_groups(lbm_batch* b, const std::vector<lbm_tuning>& gshape,
                 const std::vector<double>& gcost) {
  std::vector<int32_t> of;
  assign_groups(b, gshape, gcost, &of);
  std::vector<int32_t> remap(gshape.size(), -1);
  std::vector<lbm_tuning> used;
  for (int32_t& g : of) {
    if (remap[g] < 0) {
      remap[g] = (int32_t)used.size();
      used.push_back(gshape[g]);
    }
    g = remap[g];
  }
  if (used.size() < 2) return lbm_batch_set_groups(b, 0, nullptr, nullptr);
  return lbm_batch_set_groups(b, (int32_t)used.size(), used.data(), of.data());
}


// Generation of the tile kernels, the last component of every tuning-cache
// key: entries measured on kernels of another generation are not reused.
constexpr const char* kKernelGeneration = "/k6";

// Times `run(t)` for each candidate on the state f, restoring f from
// `backup` before each run and at the end; returns the fastest, and every
// candidate's milliseconds in *times (when not NULL).
template <class Prepare, class Run>
int autotune_impl(hipStream_t s, double* f, double* backup, size_t bytes,
                  int64_t probe, const std::vector<lbm_tuning>& cands,
                  Prepare prepare, Run run, lbm_tuning* best,
                  std::vector<float>* times = nullptr) {
  if (times) times->assign(cands.size(), INFINITY);
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
  for (size_t ci = 0; ci < cands.size(); ++ci) {
    const lbm_tuning& t = cands[ci];
    // a blocked shape runs whole pairs of its own K (a shorter run would be
    // split into shorter launches), at least `probe` steps; times are
    // compared per step, scaled to `probe` steps
    int64_t steps = probe;
    if (t.kernel == LBM_KERNEL_BLOCKED) {
      const int64_t k2 = 2 * (int64_t)t.steps_per_launch;
      steps = (std::max(probe, k2) + k2 - 1) / k2 * k2;
    }
    if ((rc = prepare(t))) break;
    if ((rc = run(t, steps))) break;  // warm-up
    if ((rc = hip_check(hipMemcpyAsync(f, backup, bytes,
                                       hipMemcpyDeviceToDevice, s),
                        "hipMemcpyAsync")))
      break;
    (void)hipEventRecord(e0, s);
    if ((rc = run(t, steps))) break;
    (void)hipEventRecord(e1, s);
    if ((rc = hip_check(hipEventSynchronize(e1), "hipEventSynchronize")))
      break;
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    ms = ms * (float)probe / (float)steps;
    if (times) (*times)[ci] = ms;
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
      (h->p.eq_kind == 0 ? "/eq8" : "/eqsel") + kKernelGeneration;
  lbm_tuning best{};
  if (!tune_cache_get(cache_path, key, &best)) {
    std::vector<lbm_tuning> cands = tuning_candidates();
    cands.push_back(lbm_tuning{LBM_KERNEL_PLAIN, 0, 1, 1});
    // the default shape (one wavefront, or one node per lane, on small
    // lattices) is not among the throughput candidates
    const lbm_tuning d = default_tuning(h->n, h->n, h->p.eq_kind == 0 ? 0 : -1);
    if (std::none_of(cands.begin(), cands.end(),
                     [&](const lbm_tuning& c) { return same_tuning(c, d); }))
      cands.push_back(d);
    double* backup = static_cast<double*>(ws) + 6 * h->n + diag_ws_doubles();
    const size_t step_ws = lbm_workspace_bytes(h, LBM_WS_STEP);
    const lbm_tuning prev = h->tune;
    int rc = autotune_impl(
        h->stream, f, backup, sbytes, probe_steps, cands,
        [&](const lbm_tuning& t) { h->tune = t; return LBM_OK; },
        [&](const lbm_tuning&, int64_t k) {
          return lbm_step(h, f, ws, step_ws, k);
        },
        &best);
    if (rc) {
      h->tune = prev;  // a failed search leaves the tuning as it was
      return rc;
    }
    tune_cache_put(cache_path, key, best);
  }
  h->tune = best;
  h->tune_default = false;
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
  x->eq_cls = std::all_of(params, params + n_inst,
                          [](const lbm_params& q) { return q.eq_kind == 0; })
                  ? 0
                  : -1;
  x->consts.resize(n_inst);
  for (int64_t i = 0; i < n_inst; ++i) {
    int rc = make_consts(&params[i], &x->consts[i]);
    if (rc) {
      delete x;
      return set_err(rc, "lattice %lld: %s", (long long)i, g_err.c_str());
    }
  }
  x->stream = (hipStream_t)stream;
  x->tune = default_tuning(x->n_total / n_inst, x->n_total, x->eq_class());
  *b = x;
  return LBM_OK;
}

void lbm_batch_destroy(lbm_batch* b) {
  if (!b) return;
  drop_graph(b);
  lbm::drop_adjoint_graph(b);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  if (b->rstream) (void)hipStreamDestroy(b->rstream);
  for (hipEvent_t ev : b->revents)
    if (ev) (void)hipEventDestroy(ev);
  for (hipStream_t st : b->gstreams) (void)hipStreamDestroy(st);
  for (hipEvent_t ev : b->gevents) (void)hipEventDestroy(ev);
  if (b->res_stream) (void)hipStreamDestroy(b->res_stream);
  for (hipEvent_t ev : b->res_events)
    if (ev) (void)hipEventDestroy(ev);
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
  b->group_tune.clear();
  b->group_of.clear();
  return LBM_OK;
}

int lbm_batch_get_tuning(const lbm_batch* b, lbm_tuning* t) {
  if (!b || !t) return set_err(LBM_EINVAL, "NULL argument");
  *t = b->tune;
  return LBM_OK;
}

int lbm_batch_set_groups(lbm_batch* b, int32_t n_groups,
                         const lbm_tuning* shapes, const int32_t* group_of) {
  if (!b) return set_err(LBM_EINVAL, "batch is NULL");
  if (n_groups == 0) {
    b->group_tune.clear();
    b->group_of.clear();
    return LBM_OK;
  }
  if (n_groups < 0 || n_groups > LBM_MAX_GROUPS)
    return set_err(LBM_EINVAL, "n_groups must lie in 0 .. %d", LBM_MAX_GROUPS);
  if (!shapes || !group_of) return set_err(LBM_EINVAL, "NULL argument");
  std::vector<lbm_tuning> gt(shapes, shapes + n_groups);
  for (lbm_tuning& t : gt) {
    const int rc = check_tuning(&t);
    if (rc) return rc;
    if (t.kernel == LBM_KERNEL_PLAIN)
      return set_err(LBM_EINVAL, "batches run the blocked kernel only");
    t.kernel = LBM_KERNEL_BLOCKED;
  }
  std::vector<int32_t> go(group_of, group_of + b->n_inst);
  for (int64_t i = 0; i < b->n_inst; ++i)
    if (go[i] < 0 || go[i] >= n_groups)
      return set_err(LBM_EINVAL, "group_of[%lld] = %d is not a group",
                     (long long)i, (int)go[i]);
  // side streams (default priority) and fork/join events, created once
  while ((int32_t)b->gstreams.size() < n_groups - 1) {
    hipStream_t st;
    const int rc = hip_check(hipStreamCreateWithFlags(&st, hipStreamNonBlocking),
                             "hipStreamCreate");
    if (rc) return rc;
    b->gstreams.push_back(st);
  }
  while ((int32_t)b->gevents.size() < n_groups) {
    hipEvent_t ev;
    const int rc = hip_check(hipEventCreateWithFlags(&ev, hipEventDisableTiming),
                             "hipEventCreate");
    if (rc) return rc;
    b->gevents.push_back(ev);
  }
  b->group_tune = gt;
  b->group_of = go;
  return LBM_OK;
}

int lbm_batch_get_groups(const lbm_batch* b, int32_t* n_groups,
                         lbm_tuning* shapes, int32_t* group_of) {
  if (!b || !n_groups) return set_err(LBM_EINVAL, "NULL argument");
  *n_groups = (int32_t)b->group_tune.size();
  if (shapes)
    std::copy(b->group_tune.begin(), b->group_tune.end(), shapes);
  if (group_of)
    std::copy(b->group_of.begin(), b->group_of.end(), group_of);
  return LBM_OK;
}

int64_t lbm_batch_total_nodes(const lbm_batch* b) { return b ? b->n_total : 0; }

int lbm_batch_set_resident(lbm_batch* b, int mode) {
  if (!b) return set_err(LBM_EINVAL, "batch is NULL");
  if (mode != 0 && mode != 1)
    return set_err(LBM_EINVAL, "resident mode must be 0 or 1, not %d", mode);
  b->resident_mode = mode;
  return LBM_OK;
}

int64_t lbm_batch_resident_lattices(const lbm_batch* b) {
  if (!b) return 0;
  int64_t c = 0;
  for (int64_t i = 0; i < b->n_inst; ++i) c += b->resident(i) ? 1 : 0;
  return c;
}

size_t lbm_batch_workspace_bytes(const lbm_batch* b, int kind) {
  if (!b) return 0;
  if (kind == LBM_WS_STEP) return layout(b, b->run_tiles(), false).total;
  if (kind == LBM_WS_TUNE) return layout(b, tune_tiles(b), true).total;
  return 0;
}

int lbm_batch_prepare(lbm_batch* b, void* ws, size_t ws_bytes) {
  if (!b || !ws) return set_err(LBM_EINVAL, "NULL argument");
  const int64_t ntiles = b->run_tiles();
  const Layout L = layout(b, ntiles, false);
  if (ws_bytes < L.total)
    return set_err(LBM_EWORKSPACE, "workspace of %zu bytes, need %zu", ws_bytes,
                   L.total);
  // one table per group (a single group: tune), concatenated
  const bool grouped = !b->group_tune.empty();
  const size_t ng = grouped ? b->group_tune.size() : 1;
  std::vector<TileRef> tiles;
  tiles.reserve(ntiles);
  std::vector<int64_t> first(ng + 1, 0);
  for (size_t g = 0; g < ng; ++g) {
    first[g] = (int64_t)tiles.size();
    const lbm_tuning& t = grouped ? b->group_tune[g] : b->tune;
    const int64_t out = tile_width(t) - 4 * (int64_t)t.steps_per_launch;
    for (int64_t i = 0; i < b->n_inst; ++i) {
      if ((grouped && b->group_of[i] != (int32_t)g) || b->resident(i)) continue;
      const int64_t n = b->offsets[i + 1] - b->offsets[i];
      for (int64_t k = 0; k * out < n; ++k)
        tiles.push_back(TileRef{(int32_t)i, (int32_t)k});
    }
  }
  first[ng] = (int64_t)tiles.size();
  // Resident lattices packed into workgroups of kResidentWaves wavefronts,
  // longest first, each into the first workgroup with room for its
  // ceil(L / 62P) wavefronts.
  std::vector<ResidentItem> items;
  std::vector<int32_t> res_first;
  {
    std::vector<int64_t> order;
    for (int64_t i = 0; i < b->n_inst; ++i)
      if (b->resident(i)) order.push_back(i);
    auto waves = [&](int64_t i) {
      const int64_t L = b->offsets[i + 1] - b->offsets[i];
      return (int32_t)((L + 62 * kResP - 1) / (62 * kResP));
    };
    std::stable_sort(order.begin(), order.end(),
                     [&](int64_t x, int64_t y) { return waves(x) > waves(y); });
    std::vector<int32_t> used;                     // wavefronts used per workgroup
    std::vector<std::vector<ResidentItem>> bins;
    for (int64_t i : order) {
      const int32_t w = waves(i);
      size_t g = 0;
      while (g < used.size() && used[g] + w > kResidentWaves) ++g;
      if (g == used.size()) {
        used.push_back(0);
        bins.emplace_back();
      }
      bins[g].push_back(ResidentItem{(int32_t)i, used[g], w, 0});
      used[g] += w;
    }
    for (const auto& bin : bins) {
      res_first.push_back((int32_t)items.size());
      items.insert(items.end(), bin.begin(), bin.end());
    }
    res_first.push_back((int32_t)items.size());
  }
  if (!items.empty()) {
    // the resident launch's side stream (default priority) and events,
    // created once, outside any capture
    if (!b->res_stream) {
      const int r = hip_check(hipStreamCreateWithFlags(&b->res_stream,
                                                       hipStreamNonBlocking),
                              "hipStreamCreate");
      if (r) return r;
    }
    for (hipEvent_t& ev : b->res_events)
      if (!ev) {
        const int r = hip_check(hipEventCreateWithFlags(&ev, hipEventDisableTiming),
                                "hipEventCreate");
        if (r) return r;
      }
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
  if (!rc && !tiles.empty())
    rc = hip_check(hipMemcpyAsync(at<char>(ws, L.tiles), tiles.data(),
                                  sizeof(TileRef) * tiles.size(),
                                  hipMemcpyHostToDevice, b->stream),
                   "hipMemcpyAsync");
  if (!rc && !items.empty())
    rc = hip_check(hipMemcpyAsync(at<char>(ws, L.res_items), items.data(),
                                  sizeof(ResidentItem) * items.size(),
                                  hipMemcpyHostToDevice, b->stream),
                   "hipMemcpyAsync");
  if (!rc && !items.empty())
    rc = hip_check(hipMemcpyAsync(at<char>(ws, L.res_first), res_first.data(),
                                  sizeof(int32_t) * res_first.size(),
                                  hipMemcpyHostToDevice, b->stream),
                   "hipMemcpyAsync");
  if (!rc) rc = hip_check(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
  if (rc) return rc;
  b->prep_ws = ws;
  b->prep_tune = b->tune;
  b->prep_tiles = (int64_t)tiles.size();
  b->prep_group_tune = b->group_tune;
  b->prep_group_of = b->group_of;
  b->prep_group_first = grouped ? first : std::vector<int64_t>();
  b->prep_resident_mode = b->resident_mode;
  b->prep_res_items = items;
  b->prep_res_first = items.empty() ? std::vector<int32_t>() : res_first;
  return LBM_OK;
}

int lbm_batch_set_equilibrium(lbm_batch* b, const double* rho, const double* J,
                              const double* zeta, double* f, void* ws,
                              size_t ws_bytes) {
  if (!rho || !J || !zeta || !f) return set_err(LBM_EINVAL, "NULL argument");
  int rc = check_batch_ws(b, ws, ws_bytes);
  if (rc) return rc;
  const Layout L = layout(b, b->run_tiles(), false);
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
  if (!use_graph) {
    rc = enqueue_batch(b, f, ws, nsteps, b->stream);
    return rc ? rc : batch_check_result(b, ws);
  }
  if (!(b->exec && b->g_f == f && b->g_ws == ws && b->g_nsteps == nsteps &&
        same_tuning(b->g_tune, b->tune) &&
        same_tunings(b->g_group_tune, b->group_tune) &&
        b->g_group_of == b->group_of && b->g_resident_mode == b->resident_mode)) {
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
    b->g_group_tune = b->group_tune;
    b->g_group_of = b->group_of;
    b->g_resident_mode = b->resident_mode;
  }
  rc = hip_check(hipGraphLaunch(b->exec, b->stream), "hipGraphLaunch");
  return rc ? rc : batch_check_result(b, ws);
}

int lbm_batch_moments(lbm_batch* b, const double* f, double* m, void* ws,
                      size_t ws_bytes) {
  int rc = check_batch_ws(b, ws, ws_bytes);
  if (rc) return rc;
  if (!f || !m) return set_err(LBM_EINVAL, "NULL argument");
  if (overlaps(f, sizeof(double) * 6 * b->n_total, m, sizeof(double) * 6 * b->n_total))
    return set_err(LBM_EINVAL, "f and m overlap");
  const Layout L = layout(b, b->run_tiles(), false);
  return launch_batch_moments(at<Consts>(ws, L.consts), at<int64_t>(ws, L.offs),
                              b->n_inst, f, m, b->n_total, b->stream);
}

int lbm_batch_diagnostics(lbm_batch* b, const double* f, void* ws,
                          size_t ws_bytes, double* out) {
  int rc = check_batch_ws(b, ws, ws_bytes);
  if (rc) return rc;
  if (!f || !out) return set_err(LBM_EINVAL, "NULL argument");
  const Layout L = layout(b, b->run_tiles(), false);
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
                          std::to_string(log2_class(mean_len)) +
                          (b->eq_class() == 0 ? "/eq8" : "/eqsel") +
                          (b->resident_mode ? "/res" : "") + kKernelGeneration;
  lbm_tuning best = b->tune;
  std::vector<lbm_tuning> gshape;
  std::vector<double> gcost;
  int resident = b->resident_mode;
  if (!tune_cache_get(cache_path, key, &best, &gshape, &gcost, &resident)) {
    double* backup = at<double>(ws, layout(b, tune_tiles(b), true).backup);
    const size_t sbytes = sizeof(double) * 6 * (size_t)b->n_total;
    // a failed search leaves the tuning, the groups and the mode as they were
    const lbm_tuning prev = b->tune;
    const std::vector<lbm_tuning> prev_gt = b->group_tune;
    const std::vector<int32_t> prev_go = b->group_of;
    const int32_t prev_mode = b->resident_mode;
    auto fail = [&](int code) {
      b->tune = prev;
      b->group_tune = prev_gt;
      b->group_of = prev_go;
      b->resident_mode = prev_mode;
      return code;
    };
    auto run = [&](const lbm_tuning&, int64_t k) {
      return lbm_batch_run(b, f, ws, ws_bytes, k, 0);
    };
    // One search for the current resident mode: the tile shape of the tiled
    // lattices, then shape groups (*ms: the kept setting's time for
    // probe_steps steps).  With every lattice resident there are no tiles
    // to tune, and the run is timed as it is.
    auto search = [&](lbm_tuning* best_out, std::vector<lbm_tuning>* gs,
                      std::vector<double>* gc, float* ms) -> int {
      b->tune = prev;
      b->group_tune.clear();
      b->group_of.clear();
      gs->clear();
      gc->clear();
      std::vector<float> times;
      if (b->count_work(b->tune) == 0) {
        *best_out = b->tune;
        lbm_tuning unused = b->tune;
        const int r = autotune_impl(
            b->stream, f, backup, sbytes, probe_steps, {b->tune},
            [&](const lbm_tuning&) { return lbm_batch_prepare(b, ws, ws_bytes); },
            run, &unused, &times);
        *ms = r ? INFINITY : times[0];
        return r;
      }
      const std::vector<lbm_tuning> cands = batch_candidates(b);
      int rc = autotune_impl(
          b->stream, f, backup, sbytes, probe_steps, cands,
          [&](const lbm_tuning& t) {
            b->tune = t;
            return lbm_batch_prepare(b, ws, ws_bytes);
          },
          run, best_out, &times);
      if (rc) return rc;
      // Shape groups: the measured time per computed node-update of each
      // shape models a grouping; the best set of two or three among the
      // eight fastest shapes is timed and kept if it beats the best single
      // shape.
      std::vector<double> cost(cands.size());
      std::vector<size_t> order(cands.size());
      size_t ib = 0;
      for (size_t c = 0; c < cands.size(); ++c) {
        cost[c] = (double)times[c] * 1e-3 /
                  ((double)b->count_work(cands[c]) * (double)probe_steps);
        order[c] = c;
        if (same_tuning(cands[c], *best_out)) ib = c;
      }
      *ms = times[ib];
      std::sort(order.begin(), order.end(),
                [&](size_t x, size_t y) { return times[x] < times[y]; });
      const size_t top = std::min<size_t>(8, order.size());
      const double single = assign_groups(b, {cands[ib]}, {cost[ib]}, nullptr);
      double best_model = single;
      std::vector<size_t> pick;
      auto consider = [&](const std::vector<size_t>& set) {
        std::vector<lbm_tuning> sh;
        std::vector<double> co;
        for (size_t c : set) {
          sh.push_back(cands[c]);
          co.push_back(cost[c]);
        }
        const double m = assign_groups(b, sh, co, nullptr);
        if (m < best_model) {
          best_model = m;
          pick = set;
        }
      };
      for (size_t x = 0; x < top; ++x)
        for (size_t y = x + 1; y < top; ++y) {
          consider({order[x], order[y]});
          for (size_t z = y + 1; z < top; ++z) consider({order[x], order[y], order[z]});
        }
      if (!pick.empty() && best_model < 0.97 * single) {
        std::vector<lbm_tuning> sh;
        std::vector<double> co;
        for (size_t c : pick) {
          sh.push_back(cands[c]);
          co.push_back(cost[c]);
        }
        b->tune = *best_out;
        std::vector<float> gt;
        lbm_tuning unused = *best_out;
        rc = autotune_impl(
            b->stream, f, backup, sbytes, probe_steps, {*best_out},
            [&](const lbm_tuning&) {
              const int r = apply_groups(b, sh, co);
              return r ? r : lbm_batch_prepare(b, ws, ws_bytes);
            },
            run, &unused, &gt);
        if (rc) return rc;
        if (gt[0] < times[ib]) {
          *gs = sh;
          *gc = co;
          *ms = gt[0];
        }
      }
      return LBM_OK;
    };
    float ms = INFINITY;
    int rc = search(&best, &gshape, &gcost, &ms);
    if (rc) return fail(rc);
    // Resident lattices on: the search is repeated with every lattice on
    // tiles, and the faster of the two modes is kept.
    if (prev_mode == 1 && lbm_batch_resident_lattices(b) > 0) {
      b->resident_mode = 0;
      lbm_tuning best0 = prev;
      std::vector<lbm_tuning> gshape0;
      std::vector<double> gcost0;
      float ms0 = INFINITY;
      rc = search(&best0, &gshape0, &gcost0, &ms0);
      if (rc) return fail(rc);
      // the two settings compared over a longer run: a short probe
      // under-weighs the resident launch, which loads and stores its
      // lattices once per run
      auto time_setting = [&](int mode, const lbm_tuning& t,
                              const std::vector<lbm_tuning>& gs,
                              const std::vector<double>& gc, float* out_ms) {
        b->resident_mode = mode;
        b->tune = t;
        std::vector<float> tm;
        lbm_tuning unused = t;
        const int r = autotune_impl(
            b->stream, f, backup, sbytes, std::max<int64_t>(8 * probe_steps, 1024),
            {t},
            [&](const lbm_tuning&) {
              const int r2 = gs.empty() ? lbm_batch_set_groups(b, 0, nullptr, nullptr)
                                        : apply_groups(b, gs, gc);
              return r2 ? r2 : lbm_batch_prepare(b, ws, ws_bytes);
            },
            run, &unused, &tm);
        *out_ms = r ? INFINITY : tm[0];
        return r;
      };
      if ((rc = time_setting(1, best, gshape, gcost, &ms))) return fail(rc);
      if ((rc = time_setting(0, best0, gshape0, gcost0, &ms0))) return fail(rc);
      if (ms0 < ms) {
        best = best0;
        gshape = gshape0;
        gcost = gcost0;
        resident = 0;
      } else {
        resident = 1;
      }
    }
    tune_cache_put(cache_path, key, best, &gshape, &gcost, resident);
  }
  b->resident_mode = resident;
  b->tune = best;
  int rc = gshape.empty() ? lbm_batch_set_groups(b, 0, nullptr, nullptr)
                          : apply_groups(b, gshape, gcost);
  if (!rc) rc = lbm_batch_prepare(b, ws, ws_bytes);
  if (rc) return rc;
  if (out) *out = best;
  return LBM_OK;
}

}  // extern "C"
