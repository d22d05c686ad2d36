// Host-side declarations shared by the translation units of the library.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/lbm.h"
#include "lbm_device.hpp"

namespace lbm {

extern thread_local std::string g_err;
int set_err(int code, const char* fmt, ...);
int hip_check(hipError_t e, const char* what);
int make_consts(const lbm_params* p, Consts* c);

int64_t tile_out(int P, int K, int wg);
size_t diag_ws_doubles();

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

int launch_batch_tile(const Consts* cs, const int64_t* offs,
                      const TileRef* tiles, int64_t ntiles, const double* fin,
                      double* fout, int64_t S, int P, int H, int K, int wg,
                      hipStream_t s);
int launch_batch_equilibrium(const Consts* cs, const int64_t* offs,
                             int64_t n_inst, const double* rho, const double* J,
                             const double* zeta, double* f, int64_t S,
                             hipStream_t s);
int launch_batch_diag(const Consts* cs, const int64_t* offs, int64_t n_inst,
                      const double* f, int64_t S, double* out, hipStream_t s);

// Splits nsteps into launches of at most K steps, an even number of them
// when nsteps >= 2 (so that ping-pong buffering ends in the caller's state).
std::vector<int> split_steps(int64_t nsteps, int K);

// Tile shapes the autotuner tries (P, K, waves per tile).
std::vector<lbm_tuning> tuning_candidates();

bool overlaps(const void* a, size_t na, const void* b, size_t nb);

// Tuning cache: "<arch>/<kind>/<class>" -> shape, in a small JSON file.
bool tune_cache_get(const char* path, const std::string& key, lbm_tuning* t);
void tune_cache_put(const char* path, const std::string& key,
                    const lbm_tuning& t);
std::string gpu_arch_name();

// Validates a tuning record for a lattice (or batch) of minimum length nmin.
int check_tuning(const lbm_tuning* t);

}  // namespace lbm

struct lbm_handle {
  int64_t n;
  lbm_params p;
  lbm::Consts c;
  hipStream_t stream;
  lbm_tuning tune;
};
