// Concurrent execution of independent work: several solves, or several HMC
// trajectories (independent Markov chains), each on its own stream, driven
// from one host thread per item.  A single system at moderate size leaves
// most compute units idle between its dependent launches (its kernels are
// bound by latency, not bandwidth), so independent items interleave on the
// GPU's hardware queues.  Every item keeps its own handle, workspace and
// stream; results are those of the same calls made one after the other.
#include <hip/hip_runtime.h>

#include <thread>
#include <vector>

#include "../../include/holstein_hmc.h"
#include "fph_internal.h"

namespace {

template <typename F>
int run_threads(int n, F&& body) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fph::record_hip_error(e);
  std::vector<int> rc(n, FPH_OK);
  std::vector<std::thread> th;
  th.reserve(n);
  for (int k = 0; k < n; ++k)
    th.emplace_back([&, k]() {
      const hipError_t es = hipSetDevice(dev);
      rc[k] = (es == hipSuccess) ? body(k) : fph::record_hip_error(es);
    });
  for (auto& t : th) t.join();
  for (int k = 0; k < n; ++k)
    if (rc[k] != FPH_OK) return rc[k];
  return FPH_OK;
}

bool distinct_streams(int n, void* const* streams) {
  for (int a = 0; a < n; ++a) {
    if (streams[a] == nullptr) return false;
    for (int b = a + 1; b < n; ++b)
      if (streams[a] == streams[b]) return false;
  }
  return true;
}

}  // namespace

extern "C" {

int pcg_solve_concurrent(int32_t n, fph_handle_t const* h, const int32_t* nrhs, const double* const* b_dev,
                         double* const* u_dev, const fph_pcg_opts_t* opts, fph_pcg_stats_t* const* stats_host,
                         void* const* streams) {
  if (n < 1 || n > 64) return FPH_E_ARG;
  if (h == nullptr || nrhs == nullptr || b_dev == nullptr || u_dev == nullptr || opts == nullptr ||
      streams == nullptr)
    return FPH_E_NULL;
  for (int k = 0; k < n; ++k) {
    if (h[k] == nullptr || b_dev[k] == nullptr || u_dev[k] == nullptr) return FPH_E_NULL;
    for (int j = 0; j < k; ++j)
      if (h[j] == h[k]) return FPH_E_ARG;  // a handle serves one stream at a time
  }
  if (!distinct_streams(n, streams)) return FPH_E_ARG;
  return run_threads(n, [&](int k) {
    return pcg_solve(h[k], nrhs[k], b_dev[k], u_dev[k], &opts[k], stats_host ? stats_host[k] : nullptr,
                     streams[k]);
  });
}

int hmc_trajectory_concurrent(int32_t n, fph_hmc_t const* hh, double* const* x_dev,
                              const double* const* R_fields_dev, const double* const* R_mom_dev,
                              const double* r_uniform, double* const* p_out_dev, fph_hmc_stats_t* stats_host,
                              void* const* streams) {
  if (n < 1 || n > 64) return FPH_E_ARG;
  if (hh == nullptr || x_dev == nullptr || R_fields_dev == nullptr || R_mom_dev == nullptr ||
      r_uniform == nullptr || streams == nullptr)
    return FPH_E_NULL;
  for (int k = 0; k < n; ++k) {
    if (hh[k] == nullptr) return FPH_E_NULL;
    // distinct contexts on distinct operators; no Holstein handle used twice,
    // also as the preconditioner of an SSH context
    const void* ok_ = fph::hmc_operator(hh[k]);
    const void* ak = fph::hmc_aux(hh[k]);
    for (int j = 0; j < k; ++j) {
      const void* oj = fph::hmc_operator(hh[j]);
      const void* aj = fph::hmc_aux(hh[j]);
      if (hh[j] == hh[k] || oj == ok_ || (aj && (aj == ak || aj == ok_)) || (ak && ak == oj))
        return FPH_E_ARG;
    }
  }
  if (!distinct_streams(n, streams)) return FPH_E_ARG;
  return run_threads(n, [&](int k) {
    return hmc_trajectory(hh[k], x_dev[k], R_fields_dev[k], R_mom_dev[k], r_uniform[k],
                          p_out_dev ? p_out_dev[k] : nullptr, stats_host ? &stats_host[k] : nullptr,
                          streams[k]);
  });
}

}  // extern "C"
