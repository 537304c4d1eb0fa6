// C ABI of the gfx950 fermion solver (declared in include/holstein_hmc.h).
//
// One translation unit: kernels come from the fph_*.h headers; this file
// owns the handle, workspace, launch configuration and the host side of
// the conjugate-gradient loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/holstein_hmc.h"
#include "fph_blas.h"
#include "fph_common.h"
#include "fph_matvec.h"
#include "fph_precond.h"

using namespace fph;

#define FPH_CHECK(call)                          \
  do {                                           \
    hipError_t e_ = (call);                      \
    if (e_ != hipSuccess) return fail_hip(e_);   \
  } while (0)

namespace {

thread_local char g_last_hip_error[256] = "";

int fail_hip(hipError_t e) {
  std::snprintf(g_last_hip_error, sizeof(g_last_hip_error), "%s", hipGetErrorString(e));
  return FPH_E_HIP;
}

}  // namespace

struct fph_handle_s {
  fph_lattice_t lat;
  Geom g;
  int max_rhs;
  int device;
  double ch, sh;  // cosh(dtau t), sinh(dtau t)
  bool have_field;
  double a1, a2;
  // field
  double* E64;
  float* E32;
  double* dbar64;
  float* dbar32;
  // CG workspace, max_rhs right-hand sides each
  double *r64, *pa64, *pb64, *Ap64;
  float *u32, *r32, *pa32, *pb32, *Ap32, *z32;
  double* z64;
  // reductions and state
  RhsState* st;
  RhsState* st_host;  // pinned mirror
  double* partial;
  long partial_len;
  unsigned* counter;
  double* tmp64;      // max_rhs doubles
  double* tmp_host;   // pinned, max_rhs doubles
  // preconditioner
  PcTables pc;
};

namespace {

size_t vbytes(const fph_handle_s* h, size_t elem) { return (size_t)h->g.d * h->max_rhs * elem; }

int elem_blocks(long d) {
  long nb = (d + 2047) / 2048;
  return (int)std::max(1L, std::min(nb, 1024L));
}

// ------------------------------------------------ operator launch helpers

template <typename T, int NT, int MS, class In, class Epi>
hipError_t launch_mtm_cfg(const fph_handle_s* h, int nrhs, int Tch, In in, Epi epi,
                          RhsState* st, hipStream_t s) {
  const Geom& g = h->g;
  const int S = (g.Q <= NT) ? NT / g.Q : 1;
  const int nchunks = (g.Ltau + Tch - 1) / Tch;
  const int nblk = (nchunks + S - 1) / S;
  const size_t lds = 2 * (size_t)S * g.N * sizeof(T);
  auto kern = k_mtm<T, NT, MS, In, Epi>;
  if (lds > 48 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(kern, dim3(nblk, nrhs), dim3(NT), lds, s, g, (const T*)(sizeof(T) == 8 ? (const void*)h->E64 : (const void*)h->E32),
                     (T)h->ch, (T)h->sh, Tch, in, epi, st, h->partial, h->counter);
  return hipGetLastError();
}

// Slices per chunk of the fused operator: enough blocks to cover the chip.
int pick_chunk(const fph_handle_s* h, int nrhs, int NT) {
  const Geom& g = h->g;
  const int S = (g.Q <= NT) ? NT / g.Q : 1;
  int best = 1;
  for (int T = 16; T >= 1; T >>= 1) {
    const long nblk = (long)((g.Ltau + T - 1) / T + S - 1) / S * nrhs;
    if (nblk >= 1024) {
      best = T;
      break;
    }
  }
  return best;
}

template <typename T, class In, class Epi>
hipError_t launch_mtm(const fph_handle_s* h, int nrhs, In in, Epi epi, RhsState* st,
                      hipStream_t s) {
  const int Q = h->g.Q;
  if (Q <= 64) return launch_mtm_cfg<T, 64, 1>(h, nrhs, pick_chunk(h, nrhs, 64), in, epi, st, s);
  if (Q <= 256) return launch_mtm_cfg<T, 256, 1>(h, nrhs, pick_chunk(h, nrhs, 256), in, epi, st, s);
  if (Q <= 512) return launch_mtm_cfg<T, 256, 2>(h, nrhs, pick_chunk(h, nrhs, 256), in, epi, st, s);
  return launch_mtm_cfg<T, 256, 4>(h, nrhs, pick_chunk(h, nrhs, 256), in, epi, st, s);
}

template <typename T, int NT, int MS, int MODE>
hipError_t launch_M_cfg(const fph_handle_s* h, int nrhs, const T* v, T* out, double coef,
                        hipStream_t s) {
  const Geom& g = h->g;
  const int S = (g.Q <= NT) ? NT / g.Q : 1;
  const int nblk = (g.Ltau + S - 1) / S;
  const size_t lds = (size_t)S * g.N * sizeof(T);
  auto kern = k_apply_M<T, NT, MS, MODE>;
  if (lds > 48 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  const T* E = (const T*)(sizeof(T) == 8 ? (const void*)h->E64 : (const void*)h->E32);
  hipLaunchKernelGGL(kern, dim3(nblk, MODE == 0 ? nrhs : 1), dim3(NT), lds, s, g, E,
                     (T)h->ch, (T)h->sh, 1, nrhs, v, out, coef);
  return hipGetLastError();
}

template <typename T, int MODE>
hipError_t launch_M(const fph_handle_s* h, int nrhs, const T* v, T* out, double coef,
                    hipStream_t s) {
  const int Q = h->g.Q;
  if (Q <= 64) return launch_M_cfg<T, 64, 1, MODE>(h, nrhs, v, out, coef, s);
  if (Q <= 256) return launch_M_cfg<T, 256, 1, MODE>(h, nrhs, v, out, coef, s);
  if (Q <= 512) return launch_M_cfg<T, 256, 2, MODE>(h, nrhs, v, out, coef, s);
  return launch_M_cfg<T, 256, 4, MODE>(h, nrhs, v, out, coef, s);
}

template <typename T, int NT, int MS>
hipError_t launch_MT_cfg(const fph_handle_s* h, int nrhs, const T* w, T* out, hipStream_t s) {
  const Geom& g = h->g;
  const int S = (g.Q <= NT) ? NT / g.Q : 1;
  const int nblk = (g.Ltau + S - 1) / S;
  const size_t lds = (size_t)S * g.N * sizeof(T);
  auto kern = k_apply_MT<T, NT, MS>;
  if (lds > 48 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  const T* E = (const T*)(sizeof(T) == 8 ? (const void*)h->E64 : (const void*)h->E32);
  hipLaunchKernelGGL(kern, dim3(nblk, nrhs), dim3(NT), lds, s, g, E, (T)h->ch, (T)h->sh, 1,
                     w, out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_MT(const fph_handle_s* h, int nrhs, const T* w, T* out, hipStream_t s) {
  const int Q = h->g.Q;
  if (Q <= 64) return launch_MT_cfg<T, 64, 1>(h, nrhs, w, out, s);
  if (Q <= 256) return launch_MT_cfg<T, 256, 1>(h, nrhs, w, out, s);
  if (Q <= 512) return launch_MT_cfg<T, 256, 2>(h, nrhs, w, out, s);
  return launch_MT_cfg<T, 256, 4>(h, nrhs, w, out, s);
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

}  // namespace

// =================================================================== ABI

extern "C" {

const char* fph_version(void) { return "holstein-hmc-gfx950 0.1"; }

const char* fph_strerror(int code) {
  switch (code) {
    case FPH_OK: return "ok";
    case FPH_E_NULL: return "required pointer is NULL";
    case FPH_E_LATTICE: return "unsupported lattice (need even L in [4, 64], even Ltau >= 2, finite parameters)";
    case FPH_E_NRHS: return "nrhs out of range for this handle";
    case FPH_E_PREC: return "unsupported precision or operator code";
    case FPH_E_NOFIELD: return "fph_set_field has not been called";
    case FPH_E_ALIGN: return "device pointer not 16-byte aligned";
    case FPH_E_ARG: return "invalid argument";
    case FPH_E_HIP: return g_last_hip_error[0] ? g_last_hip_error : "HIP runtime error";
    default: return "unknown error";
  }
}

int fph_create(fph_handle_t* out, const fph_lattice_t* lat, int32_t max_rhs) {
  if (out == nullptr || lat == nullptr) return FPH_E_NULL;
  *out = nullptr;
  if (lat->L < 4 || lat->L % 2 || lat->L > 64 || lat->Ltau < 2 || lat->Ltau % 2 ||
      !std::isfinite(lat->dtau) || !std::isfinite(lat->t) || !std::isfinite(lat->mu) ||
      !std::isfinite(lat->alpha) || lat->dtau <= 0.0)
    return FPH_E_LATTICE;
  if (!pc_supported(lat->Ltau)) return FPH_E_LATTICE;
  if (max_rhs < 1) return FPH_E_NRHS;
  fph_handle_s* h = new fph_handle_s();
  std::memset(h, 0, sizeof(*h));
  h->lat = *lat;
  h->g.L = lat->L;
  h->g.hL = lat->L / 2;
  h->g.N = lat->L * lat->L;
  h->g.Q = h->g.N / 4;
  h->g.Ltau = lat->Ltau;
  h->g.d = (long)h->g.N * lat->Ltau;
  h->max_rhs = max_rhs;
  h->ch = std::cosh(lat->dtau * lat->t);
  h->sh = std::sinh(lat->dtau * lat->t);
  h->a1 = h->a2 = 1.0;
  hipError_t e = hipGetDevice(&h->device);
  const long d = h->g.d;
  h->partial_len = (long)max_rhs * std::max<long>(4096, d / 16 + 1);
#define ALLOC(ptr, bytes)                                   \
  if (e == hipSuccess) e = hipMalloc((void**)&(ptr), (bytes));
  ALLOC(h->E64, d * sizeof(double));
  ALLOC(h->E32, d * sizeof(float));
  ALLOC(h->dbar64, h->g.N * sizeof(double));
  ALLOC(h->dbar32, h->g.N * sizeof(float));
  ALLOC(h->r64, vbytes(h, 8));
  ALLOC(h->pa64, vbytes(h, 8));
  ALLOC(h->pb64, vbytes(h, 8));
  ALLOC(h->Ap64, vbytes(h, 8));
  ALLOC(h->z64, vbytes(h, 8));
  ALLOC(h->u32, vbytes(h, 4));
  ALLOC(h->r32, vbytes(h, 4));
  ALLOC(h->pa32, vbytes(h, 4));
  ALLOC(h->pb32, vbytes(h, 4));
  ALLOC(h->Ap32, vbytes(h, 4));
  ALLOC(h->z32, vbytes(h, 4));
  ALLOC(h->st, max_rhs * sizeof(RhsState));
  ALLOC(h->partial, h->partial_len * sizeof(double));
  ALLOC(h->counter, max_rhs * sizeof(unsigned));
  ALLOC(h->tmp64, max_rhs * sizeof(double));
#undef ALLOC
  if (e == hipSuccess) e = hipHostMalloc((void**)&h->st_host, max_rhs * sizeof(RhsState), hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostMalloc((void**)&h->tmp_host, max_rhs * sizeof(double), hipHostMallocDefault);
  if (e == hipSuccess) e = hipMemset(h->counter, 0, max_rhs * sizeof(unsigned));
  if (e == hipSuccess) e = hipMemset(h->st, 0, max_rhs * sizeof(RhsState));
  if (e == hipSuccess) e = pc_create(&h->pc, h->g, max_rhs);
  h->pc.ch = h->ch;
  h->pc.sh = h->sh;
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    fph_destroy(h);
    return fail_hip(e);
  }
  *out = h;
  return FPH_OK;
}

int fph_destroy(fph_handle_t h) {
  if (h == nullptr) return FPH_E_NULL;
  (void)hipDeviceSynchronize();
  void* devptrs[] = {h->E64, h->E32, h->dbar64, h->dbar32, h->r64, h->pa64, h->pb64,
                     h->Ap64, h->z64, h->u32, h->r32, h->pa32, h->pb32, h->Ap32, h->z32,
                     h->st, h->partial, h->counter, h->tmp64};
  for (void* p : devptrs)
    if (p) (void)hipFree(p);
  if (h->st_host) (void)hipHostFree(h->st_host);
  if (h->tmp_host) (void)hipHostFree(h->tmp_host);
  pc_destroy(&h->pc);
  delete h;
  return FPH_OK;
}

int fph_set_field(fph_handle_t h, const double* x_dev, double a1, double a2, void* stream) {
  if (h == nullptr || x_dev == nullptr) return FPH_E_NULL;
  if (!std::isfinite(a1) || !std::isfinite(a2)) return FPH_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  const long d = h->g.d;
  h->a1 = a1 > 0.0 ? a1 : 1.0;
  h->a2 = a2 > 0.0 ? a2 : 1.0;
  hipLaunchKernelGGL(k_set_field, dim3(elem_blocks(d)), dim3(256), 0, s, d, x_dev,
                     h->lat.dtau, h->lat.alpha, h->lat.mu, h->E64, h->E32);
  FPH_CHECK(hipGetLastError());
  hipLaunchKernelGGL(k_dbar, dim3((h->g.N + 255) / 256), dim3(256), 0, s, h->g.N, h->g.Ltau,
                     h->E64, h->dbar64, h->dbar32);
  FPH_CHECK(hipGetLastError());
  FPH_CHECK(pc_set_field(&h->pc, h->g, h->dbar64, h->lat.dtau, h->lat.t, h->a1, h->a2, s));
  h->have_field = true;
  return FPH_OK;
}

int fermion_matvec(fph_handle_t h, int32_t op, int32_t prec, int32_t nrhs, const void* in_dev,
                   void* out_dev, void* stream) {
  if (h == nullptr || in_dev == nullptr || out_dev == nullptr) return FPH_E_NULL;
  if (!h->have_field) return FPH_E_NOFIELD;
  if (nrhs < 1 || nrhs > 65535) return FPH_E_NRHS;
  if (op < 0 || op > 2 || (prec != FPH_F64 && prec != FPH_F32)) return FPH_E_PREC;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  if (prec == FPH_F64) {
    const double* in = (const double*)in_dev;
    double* out = (double*)out_dev;
    if (op == FPH_OP_M) e = launch_M<double, 0>(h, nrhs, in, out, 0.0, s);
    else if (op == FPH_OP_MT) e = launch_MT<double>(h, nrhs, in, out, s);
    else e = launch_mtm<double>(h, nrhs, InPlain<double>{in}, EpiStore<double>{out}, nullptr, s);
  } else {
    const float* in = (const float*)in_dev;
    float* out = (float*)out_dev;
    if (op == FPH_OP_M) e = launch_M<float, 0>(h, nrhs, in, out, 0.0, s);
    else if (op == FPH_OP_MT) e = launch_MT<float>(h, nrhs, in, out, s);
    else e = launch_mtm<float>(h, nrhs, InPlain<float>{in}, EpiStore<float>{out}, nullptr, s);
  }
  if (e != hipSuccess) return fail_hip(e);
  return FPH_OK;
}

int fermion_force(fph_handle_t h, int32_t nrhs, const double* u_dev, double* grad_dev,
                  double scale, void* stream) {
  if (h == nullptr || u_dev == nullptr || grad_dev == nullptr) return FPH_E_NULL;
  if (!h->have_field) return FPH_E_NOFIELD;
  if (nrhs < 1) return FPH_E_NRHS;
  if (!std::isfinite(scale)) return FPH_E_ARG;
  const double coef = -2.0 * h->lat.dtau * h->lat.alpha * scale;
  hipError_t e = launch_M<double, 1>(h, nrhs, u_dev, grad_dev, coef, (hipStream_t)stream);
  if (e != hipSuccess) return fail_hip(e);
  return FPH_OK;
}

int fermion_action(fph_handle_t h, int32_t nrhs, const double* b_dev, const double* u_dev,
                   double* out_dev, void* stream) {
  if (h == nullptr || b_dev == nullptr || u_dev == nullptr || out_dev == nullptr) return FPH_E_NULL;
  if (nrhs < 1 || nrhs > h->max_rhs) return FPH_E_NRHS;
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_dot_out, dim3(elem_blocks(h->g.d), nrhs), dim3(256), 0, s, h->g.d, b_dev,
                     u_dev, h->partial, h->counter, out_dev);
  FPH_CHECK(hipGetLastError());
  return FPH_OK;
}

int fph_precond_apply(fph_handle_t h, int32_t op, int32_t prec, int32_t nrhs, const void* in_dev,
                      void* out_dev, void* stream) {
  if (h == nullptr || in_dev == nullptr || out_dev == nullptr) return FPH_E_NULL;
  if (!h->have_field) return FPH_E_NOFIELD;
  if (nrhs < 1 || nrhs > h->max_rhs) return FPH_E_NRHS;
  if (op < 0 || op > 2 || (prec != FPH_F64 && prec != FPH_F32)) return FPH_E_PREC;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  if (prec == FPH_F64)
    e = pc_apply<double>(&h->pc, h->g, h->dbar64, op, nrhs, (const double*)in_dev,
                         (double*)out_dev, nullptr, nullptr, nullptr, h->partial, h->counter, s);
  else
    e = pc_apply<float>(&h->pc, h->g, h->dbar32, op, nrhs, (const float*)in_dev,
                        (float*)out_dev, nullptr, nullptr, nullptr, h->partial, h->counter, s);
  if (e != hipSuccess) return fail_hip(e);
  return FPH_OK;
}

int fph_precond_info(fph_handle_t h, double* bounds_host, int32_t* np_host, void* stream) {
  if (h == nullptr || bounds_host == nullptr) return FPH_E_NULL;
  if (!h->have_field) return FPH_E_NOFIELD;
  hipStream_t s = (hipStream_t)stream;
  PcInfo info;
  FPH_CHECK(hipMemcpyAsync(&info, h->pc.info, sizeof(PcInfo), hipMemcpyDeviceToHost, s));
  if (np_host)
    FPH_CHECK(hipMemcpyAsync(np_host, h->pc.np, h->g.Ltau * sizeof(int), hipMemcpyDeviceToHost, s));
  FPH_CHECK(hipStreamSynchronize(s));
  bounds_host[0] = info.bmin;
  bounds_host[1] = info.bmax;
  return FPH_OK;
}

}  // extern "C"

// ============================================================ CG driver

namespace {

// One CG iteration for right-hand sides 0..nrhs-1 in precision T.  The
// direction buffers pa/pb alternate on the device with each right-hand
// side's own iteration parity (right-hand sides that are paused or done
// skip the iteration without flipping it).
template <typename T>
hipError_t cg_iteration(fph_handle_s* h, int nrhs, bool precond, T* u, T* r, T* z, T* pa,
                        T* pb, T* Ap, const T* dbar, hipStream_t s) {
  const long d = h->g.d;
  const T* zz = precond ? z : r;
  InPUpdate<T> in{zz, pa, pb, nullptr, nullptr, (T)0, 0};
  hipError_t e = launch_mtm<T>(h, nrhs, in, EpiDotAlpha<T>{Ap}, h->st, s);
  if (e != hipSuccess) return e;
  if (!precond) {
    hipLaunchKernelGGL(k_cg_update<T>, dim3(elem_blocks(d), nrhs), dim3(256), 0, s, d, u,
                       (const T*)pa, (const T*)pb, r, (const T*)Ap, h->st, h->partial,
                       h->counter);
    e = hipGetLastError();
  } else {
    e = pc_cg_update<T>(&h->pc, h->g, dbar, nrhs, u, pa, pb, r, Ap, z, h->st, h->partial,
                        h->counter, s);
  }
  return e;
}

// z = F F^T r and r.z for the current residual, updating rz/beta (after a
// residual replacement).
template <typename T>
hipError_t precondition_residual(fph_handle_s* h, int nrhs, T* r, T* z, const T* dbar,
                                 hipStream_t s) {
  return pc_apply<T>(&h->pc, h->g, dbar, FPH_PC_FFT, nrhs, r, z, h->st, r, nullptr, h->partial,
                     h->counter, s);
}

hipError_t sync_state(fph_handle_s* h, int nrhs, hipStream_t s) {
  hipError_t e = hipMemcpyAsync(h->st_host, h->st, nrhs * sizeof(RhsState),
                                hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(s);
}

hipError_t push_state(fph_handle_s* h, int nrhs, hipStream_t s) {
  return hipMemcpyAsync(h->st, h->st_host, nrhs * sizeof(RhsState), hipMemcpyHostToDevice, s);
}

}  // namespace

extern "C" int pcg_solve(fph_handle_t h, int32_t nrhs, const double* b_dev, double* u_dev,
                         const fph_pcg_opts_t* opts, fph_pcg_stats_t* stats, void* stream) {
  if (h == nullptr || b_dev == nullptr || u_dev == nullptr || opts == nullptr) return FPH_E_NULL;
  if (!h->have_field) return FPH_E_NOFIELD;
  if (nrhs < 1 || nrhs > h->max_rhs) return FPH_E_NRHS;
  if (opts->prec != FPH_F64 && opts->prec != FPH_F32_REFINED) return FPH_E_PREC;
  if (!(opts->tol >= 0.0) || opts->maxiter < 1) return FPH_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  const long d = h->g.d;
  const int nb = elem_blocks(d);
  const bool pre = opts->use_precond != 0;
  const bool mixed = opts->prec == FPH_F32_REFINED;
  const double delta = opts->ru_delta > 0.0 ? opts->ru_delta : 0.1;

  // State: bb = |b|^2, tol2, counters.
  hipLaunchKernelGGL(k_norm2<double>, dim3(nb, nrhs), dim3(256), 0, s, d, b_dev, h->partial,
                     h->counter, h->st, opts->tol, opts->maxiter, 0);
  FPH_CHECK(hipGetLastError());
  if (opts->zero_guess) FPH_CHECK(hipMemsetAsync(u_dev, 0, nrhs * d * sizeof(double), s));

  // Initial residual.
  if (!mixed) {
    if (opts->zero_guess) {
      FPH_CHECK(hipMemcpyAsync(h->r64, b_dev, nrhs * d * sizeof(double), hipMemcpyDeviceToDevice, s));
    } else {
      FPH_CHECK(launch_mtm<double>(h, nrhs, InPlain<double>{u_dev},
                                   EpiResidual<double>{b_dev, h->r64}, h->st, s));
      hipLaunchKernelGGL(k_norm2<double>, dim3(nb, nrhs), dim3(256), 0, s, d, h->r64,
                         h->partial, h->counter, h->st, opts->tol, opts->maxiter, 1);
      FPH_CHECK(hipGetLastError());
    }
    if (pre) FPH_CHECK(precondition_residual<double>(h, nrhs, h->r64, h->z64, h->dbar64, s));
  } else {
    FPH_CHECK(hipMemsetAsync(h->u32, 0, nrhs * d * sizeof(float), s));
    if (opts->zero_guess) {
      hipLaunchKernelGGL((k_cast<double, float>), dim3(nb), dim3(256), 0, s, nrhs * d, b_dev, h->r32);
      FPH_CHECK(hipGetLastError());
    } else {
      FPH_CHECK(launch_mtm<double>(h, nrhs, InPlain<double>{u_dev},
                                   EpiResidual<float>{b_dev, h->r32}, h->st, s));
    }
    hipLaunchKernelGGL(k_norm2<float>, dim3(nb, nrhs), dim3(256), 0, s, d, h->r32, h->partial,
                       h->counter, h->st, opts->tol, opts->maxiter, 1);
    FPH_CHECK(hipGetLastError());
    if (pre) FPH_CHECK(precondition_residual<float>(h, nrhs, h->r32, h->z32, h->dbar32, s));
  }

  std::vector<int> final_(nrhs, 0);
  std::vector<int> outer(nrhs, 0);
  std::vector<int> iter_at_ru(nrhs, 0);
  std::vector<double> rr_iter(nrhs, 0.0);
  FPH_CHECK(sync_state(h, nrhs, s));
  for (int r = 0; r < nrhs; ++r) {
    RhsState& st = h->st_host[r];
    if (st.bb == 0.0) {  // b = 0: u = 0 exactly
      final_[r] = 1;
      FPH_CHECK(hipMemsetAsync(u_dev + (long)r * d, 0, d * sizeof(double), s));
    } else if (st.status & 8) {  // non-finite b
      final_[r] = 1;
    }
    if (mixed) st.ru_thresh = delta * delta * st.rr;
  }
  FPH_CHECK(push_state(h, nrhs, s));

  // Iterations enqueued between host checks.  FP32 with residual
  // replacement: about 1.5 times the length of the last replacement cycle,
  // so that few launches are wasted on paused right-hand sides.
  int chunk = opts->chunk > 0 ? opts->chunk : (mixed ? 8 : 32);
  int guard = 0;
  while (true) {
    bool all_final = true;
    for (int r = 0; r < nrhs; ++r) all_final = all_final && final_[r];
    if (all_final) break;
    if (++guard > 10000000) break;

    for (int it = 0; it < chunk; ++it) {
      hipError_t e;
      if (!mixed)
        e = cg_iteration<double>(h, nrhs, pre, u_dev, h->r64, h->z64, h->pa64, h->pb64, h->Ap64,
                                 h->dbar64, s);
      else
        e = cg_iteration<float>(h, nrhs, pre, h->u32, h->r32, h->z32, h->pa32, h->pb32, h->Ap32,
                                h->dbar32, s);
      if (e != hipSuccess) return fail_hip(e);
    }
    FPH_CHECK(sync_state(h, nrhs, s));

    // Right-hand sides that stopped (converged iterate, pause, cap) get an
    // FP64 residual evaluation.
    bool need = false;
    for (int r = 0; r < nrhs; ++r) {
      if (final_[r]) continue;
      const RhsState& st = h->st_host[r];
      if (st.status & (4 | 8)) {  // breakdown / non-finite: stop
        final_[r] = 1;
        continue;
      }
      if (st.done) need = true;
    }
    if (!need) continue;

    // FP64 residual of the current iterate for every non-final rhs (the
    // others are cheap to include and keep their direction).
    for (int r = 0; r < nrhs; ++r) {
      rr_iter[r] = h->st_host[r].rr;
      h->st_host[r].done = final_[r];
    }
    FPH_CHECK(push_state(h, nrhs, s));
    if (mixed) {
      hipLaunchKernelGGL(k_flush, dim3(nb, nrhs), dim3(256), 0, s, d, h->u32, u_dev, h->st);
      FPH_CHECK(hipGetLastError());
      FPH_CHECK(launch_mtm<double>(h, nrhs, InPlain<double>{u_dev},
                                   EpiResidual<float>{b_dev, h->r32}, h->st, s));
      hipLaunchKernelGGL(k_norm2<float>, dim3(nb, nrhs), dim3(256), 0, s, d, h->r32,
                         h->partial, h->counter, h->st, opts->tol, opts->maxiter, 1);
      FPH_CHECK(hipGetLastError());
      if (pre) FPH_CHECK(precondition_residual<float>(h, nrhs, h->r32, h->z32, h->dbar32, s));
    } else {
      FPH_CHECK(launch_mtm<double>(h, nrhs, InPlain<double>{u_dev},
                                   EpiResidual<double>{b_dev, h->r64}, h->st, s));
      hipLaunchKernelGGL(k_norm2<double>, dim3(nb, nrhs), dim3(256), 0, s, d, h->r64,
                         h->partial, h->counter, h->st, opts->tol, opts->maxiter, 1);
      FPH_CHECK(hipGetLastError());
      if (pre) FPH_CHECK(precondition_residual<double>(h, nrhs, h->r64, h->z64, h->dbar64, s));
    }
    FPH_CHECK(sync_state(h, nrhs, s));
    int cycle = 0;
    for (int r = 0; r < nrhs; ++r) {
      if (final_[r]) continue;
      RhsState& st = h->st_host[r];
      outer[r] += 1;
      cycle = std::max(cycle, st.iter - iter_at_ru[r]);
      iter_at_ru[r] = st.iter;
      if (st.rr_true <= st.tol2) {
        st.status |= 1;
        final_[r] = 1;
        st.done = 1;
      } else if (st.status & (4 | 8)) {
        final_[r] = 1;
        st.done = 1;
      } else if (st.iter >= st.maxiter) {
        st.status |= 2;
        final_[r] = 1;
        st.done = 1;
      } else {
        st.done = 0;
        // FP64: restart the directions from the true residual.  FP32: keep
        // them (reliable update) unless the replaced residual is far from
        // the iterated one.
        if (!mixed || st.rr > 100.0 * rr_iter[r]) st.fresh = 1;
        if (mixed) st.ru_thresh = delta * delta * st.rr;
      }
    }
    FPH_CHECK(push_state(h, nrhs, s));
    if (mixed && opts->chunk <= 0) chunk = std::max(2, std::min(64, cycle + cycle / 2 + 1));
  }

  // Final statistics: relative residual and action b.u in FP64.
  FPH_CHECK(fermion_action(h, nrhs, b_dev, u_dev, h->tmp64, stream) == FPH_OK ? hipSuccess
                                                                                : hipErrorUnknown);
  FPH_CHECK(hipMemcpyAsync(h->tmp_host, h->tmp64, nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
  FPH_CHECK(sync_state(h, nrhs, s));
  if (stats) {
    for (int r = 0; r < nrhs; ++r) {
      const RhsState& st = h->st_host[r];
      stats[r].status = st.status;
      stats[r].iters = st.iter;
      stats[r].outer_iters = outer[r];
      stats[r].matvecs = st.matvecs;
      stats[r].rel_resid = st.bb > 0.0 ? std::sqrt(st.rr_true / st.bb) : 0.0;
      stats[r].action = h->tmp_host[r];
    }
  }
  return FPH_OK;
}
