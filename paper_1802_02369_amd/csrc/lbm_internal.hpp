// Host-side declarations shared by the translation units of the library.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>
#include <map>

#include "../../include/lbm.h"
#include "lbm_device.hpp"

namespace lbm {

extern thread_local std::string g_err;
int set_err(int code, const char* fmt, ...);
int hip_check(hipError_t e, const char* what);
int make_consts(const lbm_params* p, Consts* c);

int64_t tile_out(int P, int K, int wg);
size_t diag_ws_doubles();

// Failure detection (LBM_CHECK_FINITE).  The record is one 64-bit word in
// the workspace: ~0 when nothing failed, else the smallest key
// (steps << 36) | node (single lattice; steps saturate at kCheckMaxSteps1)
// or (steps << 31) | lattice (batch; steps saturate at kCheckMaxStepsB).
constexpr int64_t kCheckMaxSteps1 = (int64_t(1) << 28) - 1;
constexpr int64_t kCheckMaxStepsB = (int64_t(1) << 32) - 1;
// offset in doubles of the single-lattice record inside the diagnostics
// scratch (which follows the second state in the step workspace)
size_t check_record_double();
int launch_check_reset(unsigned long long* rec, hipStream_t s);
int launch_check_state(const Consts& c, const double* f, int64_t n,
                       int64_t steps, unsigned long long* rec, hipStream_t s);
int launch_batch_check(const Consts* cs, const int64_t* offs,
                       const TileRef* tiles, int64_t ntiles, const double* f,
                       int64_t S, int OUT, int64_t steps,
                       unsigned long long* rec, hipStream_t s);
// copies the record to the host and synchronises the stream
int read_check_record(const unsigned long long* rec, hipStream_t s,
                      unsigned long long* out);

// Resident lattices of a batch (k_batch_resident): P nodes per lane,
// workgroups of kResidentWaves wavefronts, lattices of 2P to
// 62 P kResidentWaves nodes.  Twelve wavefronts at three per SIMD (168
// VGPRs) measured 278 GLUPS on the 4096-lattice batch (lengths 512 ..
// 16384) against 272 for eight at two per SIMD and 265 on tiles alone.
constexpr int kResP = 8;
constexpr int kResidentWaves = 12;
constexpr int64_t kResidentMin = 2 * kResP;
constexpr int64_t kResidentMax = (int64_t)62 * kResP * kResidentWaves;
// steps of one resident launch (about 2 s on the 4096-lattice batch)
constexpr int64_t kResidentMaxSteps = int64_t(1) << 16;
// Copies the output nodes of the tiles [0, ntiles) of a table (OUT per
// tile) from src to dst.
int launch_batch_copy_tiles(const int64_t* offs, const TileRef* tiles,
                            int64_t ntiles, int OUT, const double* src,
                            double* dst, int64_t S, hipStream_t s);
int launch_batch_resident(const Consts* cs, const int64_t* offs,
                          const ResidentItem* items, const int32_t* wg_first,
                          int64_t nwg, const double* fin, double* fout,
                          int64_t S, int64_t T, int eq, hipStream_t s);
int launch_batch_check_lattices(const Consts* cs, const int64_t* offs,
                                const ResidentItem* items, int64_t nitems,
                                const double* f, int64_t S, int64_t steps,
                                unsigned long long* rec, hipStream_t s);

int launch_equilibrium(const Consts& c, const double* rho, const double* J,
                       const double* zeta, double* f, int64_t n, hipStream_t s);
int launch_step_plain(const Consts& c, const double* fin, double* fout,
                      int64_t n, hipStream_t s);
int launch_step_tile(const Consts& c, const double* fin, double* fout,
                     int64_t n, int P, int K, int wpg, hipStream_t s);
int launch_diagnostics(const Consts& c, const double* f, int64_t n,
                       double* scratch, hipStream_t s);
int launch_moments(const Consts& c, const double* f, double* m, int64_t n,
                   hipStream_t s);

// state_stride > 0: fin is state `first` of a checkpoint segment, and of
// the states first+1 .. first+K the launch reaches, state i is stored into
// fout + ((i-1)/every)*state_stride when i is a multiple of `every`.  eq = 0
// when every lattice of the table has the equilibria of section 8
// (eq_kind 0), else -1.
int launch_batch_tile(const Consts* cs, const int64_t* offs,
                      const TileRef* tiles, int64_t ntiles, const double* fin,
                      double* fout, int64_t S, int P, int H, int K, int wg,
                      int eq, hipStream_t s, int64_t state_stride = 0,
                      int first = 0, int every = 1);
int launch_batch_equilibrium(const Consts* cs, const int64_t* offs,
                             int64_t n_inst, const double* rho, const double* J,
                             const double* zeta, double* f, int64_t S,
                             hipStream_t s);
int launch_batch_moments(const Consts* cs, const int64_t* offs, int64_t n_inst,
                         const double* f, double* m, int64_t S, hipStream_t s);
int launch_batch_diag(const Consts* cs, const int64_t* offs, int64_t n_inst,
                      const double* f, int64_t S, double* out, hipStream_t s);

// Largest lattice (or batch) in nodes: keeps every grid dimension and tile
// index of every kernel within 32 bits (3.3 TB per state, beyond any device).
constexpr int64_t kMaxNodes = int64_t(1) << 36;

// Splits nsteps into launches of at most K steps, an even number of them
// when nsteps >= 2 (so that ping-pong buffering ends in the caller's state).
// The sizes are described, not stored: a run of any length costs O(1) host
// memory; iterate with a range-for.
struct StepSplit {
  int64_t count = 0, base = 0, extra = 0;
  struct It {
    const StepSplit* s;
    int64_t i;
    int operator*() const { return (int)(s->base + (i < s->extra ? 1 : 0)); }
    It& operator++() {
      ++i;
      return *this;
    }
    bool operator!=(const It& o) const { return i != o.i; }
  };
  It begin() const { return It{this, 0}; }
  It end() const { return It{this, count}; }
};
StepSplit split_steps(int64_t nsteps, int K);

// Tile shape used until lbm_set_tuning / lbm_autotune: the widest tile at
// most a quarter of the (mean) lattice length len that still leaves >= 1024
// tiles in total (four workgroups per compute unit), else the narrowest.
// Default tile shape for lattices of (mean) length len, total nodes total,
// equilibrium class eq (0: every lattice has eq_kind 0, else -1).
lbm_tuning default_tuning(int64_t len, int64_t total, int eq);

// Tile shapes the autotuner tries (P, K, waves per tile).
std::vector<lbm_tuning> tuning_candidates();

bool overlaps(const void* a, size_t na, const void* b, size_t nb);

// Tuning cache: "<arch>/<kind>/<class>" -> shape, in a small JSON file.
// Batch entries may carry shape groups with their measured time per computed
// node-update (gshape, gcost; absent groups read back empty) and the
// resident mode (-1: none stored, *resident left as it is).
bool tune_cache_get(const char* path, const std::string& key, lbm_tuning* t,
                    std::vector<lbm_tuning>* gshape = nullptr,
                    std::vector<double>* gcost = nullptr,
                    int* resident = nullptr);
void tune_cache_put(const char* path, const std::string& key,
                    const lbm_tuning& t,
                    const std::vector<lbm_tuning>* gshape = nullptr,
                    const std::vector<double>* gcost = nullptr,
                    int resident = -1);
std::string gpu_arch_name();

// Validates a tuning record for a lattice (or batch) of minimum length nmin.
int check_tuning(const lbm_tuning* t);

}  // namespace lbm

namespace lbm {
inline bool same_tuning(const lbm_tuning& a, const lbm_tuning& b) {
  return a.kernel == b.kernel && a.nodes_per_lane == b.nodes_per_lane &&
         a.steps_per_launch == b.steps_per_launch &&
         a.waves_per_group == b.waves_per_group;
}

inline bool same_tunings(const std::vector<lbm_tuning>& a,
                         const std::vector<lbm_tuning>& b) {
  if (a.size() != b.size()) return false;
  for (size_t i = 0; i < a.size(); ++i)
    if (!same_tuning(a[i], b[i])) return false;
  return true;
}

// Nodes spanned by a register tile of wg wavefronts of P nodes per lane:
// neighbouring wavefronts share two lanes (one mirror lane each).
__host__ __device__ constexpr int tile_nodes(int P, int wg) {
  return P * (62 * wg + 2);
}

inline int64_t tile_width(const lbm_tuning& t) {
  return tile_nodes(t.nodes_per_lane, t.waves_per_group);
}

// Lane-nodes a lattice of L nodes computes per step with tuning t: its
// ceil(L/OUT) tiles, each running the wavefronts it needs (the device's
// active-wave rule: the fewest whose span covers the tile's stored nodes
// and both halos of 2K), 64 P per wavefront.
inline int64_t lattice_lane_nodes(int64_t L, const lbm_tuning& t) {
  const int64_t P = t.nodes_per_lane, W = t.waves_per_group,
                H = 2 * (int64_t)t.steps_per_launch;
  const int64_t out = tile_width(t) - 2 * H;
  int64_t s = 0;
  for (int64_t first = 0; first < L; first += out) {
    const int64_t need = (L - first) + 2 * H - 2 * P;
    int64_t nw = (need + 62 * P - 1) / (62 * P);
    nw = nw < 1 ? 1 : (nw > W ? W : nw);
    s += 64 * P * nw;
  }
  return s;
}
}  // namespace lbm

struct lbm_handle {
  int64_t n;
  lbm_params p;
  lbm::Consts c;
  hipStream_t stream;
  lbm_tuning tune;
  bool tune_default = true;  // tune is the default for n and the equilibria
  int32_t adj_kernel = LBM_KERNEL_AUTO;  // reverse-sweep kernel
  int32_t rec_stride = 0;  // stride of the stored segment states (0: auto)
  lbm_batch* one = nullptr;  // batch of this one lattice, for the adjoint
};

struct lbm_batch {
  int64_t n_inst = 0, n_total = 0;
  std::vector<int64_t> offsets;
  std::vector<lbm_params> params;
  std::vector<lbm::Consts> consts;
  hipStream_t stream = nullptr;
  hipStream_t cap = nullptr;  // private stream used only for graph capture
  // side stream and events of the pipelined reverse sweep (the recompute
  // of one checkpoint segment overlaps the reverse steps of the next)
  hipStream_t rstream = nullptr;
  hipEvent_t revents[6] = {};
  lbm_tuning tune{};
  // what lbm_batch_prepare uploaded
  const void* prep_ws = nullptr;
  lbm_tuning prep_tune{};
  int64_t prep_tiles = 0;
  // Resident lattices (lbm_batch_set_resident): 1 (default) runs every
  // lattice of kResidentMin .. kResidentMax nodes in one launch for the
  // whole call (k_batch_resident), the others on tiles; 0 puts every
  // lattice on tiles.  What lbm_batch_prepare built: the resident items and
  // their workgroups.
  int32_t resident_mode = 1;
  int32_t prep_resident_mode = -1;
  hipStream_t res_stream = nullptr;  // side stream of the resident launch
  hipEvent_t res_events[2] = {};     // fork, join
  std::vector<lbm::ResidentItem> prep_res_items;
  std::vector<int32_t> prep_res_first;
  // Shape groups of lbm_batch_run (lbm_batch_set_groups): lattice i runs with
  // group_tune[group_of[i]], each group as its own launch sequence on its own
  // stream.  Empty: every lattice runs with tune.
  std::vector<lbm_tuning> group_tune;
  std::vector<int32_t> group_of;
  std::vector<hipStream_t> gstreams;  // groups 1.. (group 0: the run's stream)
  std::vector<hipEvent_t> gevents;    // [0] fork, [g] end of group g
  // the groups lbm_batch_prepare built the table for; the table holds each
  // group's tiles from prep_group_first[g] to prep_group_first[g + 1]
  std::vector<lbm_tuning> prep_group_tune;
  std::vector<int32_t> prep_group_of;
  std::vector<int64_t> prep_group_first;
  // captured graph of the last lbm_batch_run(use_graph = 1)
  hipGraphExec_t exec = nullptr;
  const double* g_f = nullptr;
  const void* g_ws = nullptr;
  int64_t g_nsteps = -1;
  lbm_tuning g_tune{};
  std::vector<lbm_tuning> g_group_tune;
  std::vector<int32_t> g_group_of;
  int32_t g_resident_mode = -1;
  // adjoint workspace uploaded by lbm_batch_forward_ckpt
  const void* adj_ws = nullptr;
  int64_t adj_nsteps = -1, adj_ckpt = -1;
  lbm_tuning adj_tune{};
  int32_t adj_kernel = LBM_KERNEL_AUTO;  // requested reverse-sweep kernel
  // the kernel lbm_batch_forward_ckpt resolved it to: one reverse step per
  // launch (else K per launch)
  bool adj_plain = false;
  bool adj_plain_up = false;  // the value the uploaded tables were built for
  // requested stride of the segment states the reverse sweep stores (0:
  // automatic), what lbm_batch_forward_ckpt resolved it to, and the value
  // the uploaded tables were built for
  int32_t rec_stride = 0;
  int32_t adj_every = 1, adj_every_up = 1;
  // captured graph of the last lbm_batch_adjoint(use_graph = 1)
  hipGraphExec_t adj_exec = nullptr;
  const double* ag_fbar = nullptr;
  const double* ag_rbar = nullptr;

  // whether some lattice asks for LBM_CHECK_FINITE
  bool check_finite() const {
    for (const lbm_params& q : params)
      if (q.flags & LBM_CHECK_FINITE) return true;
    return false;
  }

  // equilibrium class of the tile kernels: 0 if every lattice has eq_kind 0
  // (set by lbm_batch_init; the constants do not change afterwards)
  int32_t eq_cls = 0;
  int eq_class() const { return eq_cls; }

  // whether lattice i runs resident with the current settings: only in
  // batches of section-8 lattices (the kernel that selects the equilibria
  // per lattice needs more registers than three wavefronts per SIMD leave)
  bool resident(int64_t i) const {
    const int64_t L = offsets[i + 1] - offsets[i];
    return resident_mode == 1 && eq_cls == 0 && L >= lbm::kResidentMin &&
           L <= lbm::kResidentMax;
  }

  // tiles of lattice i for a tuning: ceil(L_i / OUT)
  int64_t lattice_tiles(int64_t i, const lbm_tuning& t) const {
    const int64_t out = lbm::tile_width(t) - 4 * (int64_t)t.steps_per_launch;
    return (offsets[i + 1] - offsets[i] + out - 1) / out;
  }

  // lane-nodes lattice i computes per step with tuning t
  int64_t lattice_work(int64_t i, const lbm_tuning& t) const {
    return lbm::lattice_lane_nodes(offsets[i + 1] - offsets[i], t);
  }

  // lane-nodes of the tiled lattices of the batch per step with tuning t
  int64_t count_work(const lbm_tuning& t) const {
    int64_t s = 0;
    for (int64_t i = 0; i < n_inst; ++i)
      if (!resident(i)) s += lattice_work(i, t);
    return s;
  }

  // tiles of the table for one tuning: sum of ceil(L_i / OUT)
  int64_t count_tiles(const lbm_tuning& t) const {
    int64_t s = 0;
    for (int64_t i = 0; i < n_inst; ++i) s += lattice_tiles(i, t);
    return s;
  }

  // tiles of the run's table: the groups' shapes, else tune
  int64_t run_tiles() const {
    if (group_tune.empty()) return count_tiles(tune);
    int64_t s = 0;
    for (int64_t i = 0; i < n_inst; ++i)
      s += lattice_tiles(i, group_tune[group_of[i]]);
    return s;
  }
};



