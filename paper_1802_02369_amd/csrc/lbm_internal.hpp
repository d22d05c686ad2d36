// Host-side declarations shared by the translation units of the library.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "../../include/lbm.h"
#include "lbm_device.hpp"

namespace lbm {

extern thread_local std::string g_err;
int set_err(int code, const char* fmt, ...);
int hip_check(hipError_t e, const char* what);
int make_consts(const lbm_params* p, Consts* c);

int64_t tile_out(int P, int K);
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

// Validates a tuning record for a lattice (or batch) of minimum length nmin.
int check_tuning(const lbm_tuning* t);

}  // namespace lbm
