// C ABI of the gfx950 fermion solver (declared in include/holstein_hmc.h).
//
// One translation unit: kernels come from the fph_*.h headers; this file
// owns the handle, workspace, launch configuration and the enqueueing of
// the conjugate-gradient solve (whose control runs on the device).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "../../include/holstein_hmc.h"
#include "fph_batch.h"
#include "fph_blas.h"
#include "fph_common.h"
#include "fph_coop.h"
#include "fph_internal.h"
#include "fph_matvec.h"
#include "fph_precond.h"
#include "fph_solve.h"

using namespace fph;

static_assert(sizeof(PcgStatsDev) == sizeof(fph_pcg_stats_t), "stats layout");

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

int fph::record_hip_error(hipError_t e) { return fail_hip(e); }

// ------------------------------------------- no-allocation scratch array --
//
// fermion_action_noalloc takes the partial sums of its dot products from
// this file-scope device array instead of the handle's workspace: 64
// right-hand sides x 1024 partials (512 KiB), held by every GPU the library
// runs on until the process ends.  In host code `scratch` only names the
// symbol; its device address comes from hipGetSymbolAddress, taken once per
// device with that device current (fph_create does it for the handle's
// device) and kept in kScratchPtr[device].
constexpr int kNoAllocMaxRhs = 64;
constexpr int kNoAllocMaxBlocks = 1024;  // elem_blocks() never exceeds this
static __device__ __align__(256) double scratch[kNoAllocMaxRhs * kNoAllocMaxBlocks];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device dev (current), looked up once.
hipError_t scratch_address(int dev, double** out) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace

struct fph_handle_s {
  fph_lattice_t lat;
  Geom g;
  int max_rhs;
  int device;
  double th, c4;  // tanh(dtau t), cosh(dtau t)^4 (operator kernels: C = c4 C', E stored as c4 E)
  bool have_field;
  int nfields;  // 0: one field shared by every right-hand side; else fields set by fph_set_fields
  double a1, a2;
  // field
  double* E64;
  float* E32;
  double* dbar64;
  float* dbar32;
  // CG workspace, max_rhs right-hand sides each: r, z, the two direction
  // buffers pa/pb, Ap in the iteration precision; FP32-refined also uses the
  // FP32 correction u32 and the second FP64 iterate buffer u64b.
  double *r64, *pa64, *pb64, *Ap64, *z64, *u64b;
  float *u32, *r32, *pa32, *pb32, *Ap32, *z32;
  // CG state (two alternating copies) and partial sums (two buffers)
  RhsState* st[2];
  double* part[2];    // max_rhs * kPStride each
  double* fin_part;   // partials of the final S_F, max_rhs * kPStride
  PcgStatsDev* stats_dev;   // statistics of the last blocking solve
  PcgStatsDev* stats_pin;   // pinned mirror
  int* open_pin;            // pinned: right-hand sides not finished (two probes)
  hipEvent_t probe_ev[2];
  double* tmp64;      // max_rhs doubles
  double* tmp_host;   // pinned, max_rhs doubles
  // preconditioner
  PcTables pc;
  // scratch partials for plain reductions outside a solve
  double* tmp_part() const { return part[1]; }
  // device address of the library's static scratch array on this device
  double* noalloc_part;
};

namespace {

// Residual evaluations after the first that a solve may use (opts.max_outer
// = 0), and slots between the probes of the blocking driver (opts.chunk = 0):
// 16, or 8 above 2^20 unknowns per right-hand side.  Once a solve has
// finished, the rest of its chunk and the chunk queued behind it still run
// (as idle slots); a probe costs a few microseconds.  At 409 600 unknowns
// (one or ten right-hand sides) 16 wins; at 1 638 400 the idle slots cost
// more than the extra probes, and 8 wins.
constexpr int kDefaultMaxOuter = 32;
constexpr long kDefaultSlotChunk = 16;
constexpr long kDefaultSlotChunkLarge = 8;
constexpr long kSlotChunkLargeAbove = 1L << 20;

size_t vbytes(const fph_handle_s* h, size_t elem) { return (size_t)h->g.d * h->max_rhs * elem; }

// Blocks of 256 threads for an elementwise pass over d values with 4 values
// per thread per step; at most 1024 blocks (partials fit kPStride).
int elem_blocks(long d) {
  long nb = (d + 1023) / 1024;
  return (int)std::max(1L, std::min(nb, 1024L));
}

// ------------------------------------------------ operator launch helpers

// Workgroups of `kern` resident per CU with `lds` bytes of dynamic LDS,
// times the CU count (cached per device, kernel and LDS size).
inline int resident_slots(const void* kern, int nt, size_t lds) {
  static std::mutex mu;
  static std::map<std::tuple<int, const void*, size_t>, int> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  std::lock_guard<std::mutex> lk(mu);
  auto key = std::make_tuple(dev, kern, lds);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  int per_cu = 0, ncu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, nt, lds) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 256;
  const int slots = std::max(1, per_cu) * std::max(1, ncu);
  cache[key] = slots;
  return slots;
}

// Slices per chunk of the fused operator.  A chunk costs about Tch + 1
// slice steps plus a start-up of ~2; the launch runs in ceil(blocks /
// slots) rounds of resident workgroups.  Pick the chunk length with the
// least rounds x steps (short chunks for small problems: one round of
// one-slice chunks; for large ones exactly enough chunks to fill the
// resident slots, which also keeps halo re-reads low).  Chunks may span
// the whole time axis.  Memoised: the solver asks once per launch.
int pick_chunk(const Geom& g, int nrhs, int S, int slots) {
  static std::mutex mu;
  static std::map<std::tuple<int, int, int, int>, int> cache;
  const auto key = std::make_tuple(g.Ltau, nrhs, S, slots);
  std::lock_guard<std::mutex> lk(mu);
  const auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  int best = 1;
  long best_cost = -1;
  for (int T = 1; T <= g.Ltau; ++T) {
    const long nblk = (long)(((g.Ltau + T - 1) / T + S - 1) / S) * nrhs;
    const long rounds = (nblk + slots - 1) / slots;
    const long cost = rounds * (T + 3);
    if (best_cost < 0 || cost < best_cost) {
      best_cost = cost;
      best = T;
    }
  }
  cache[key] = best;
  return best;
}

template <typename T, int NT, int MS, class In, class Epi>
hipError_t launch_mtm_cfg(const fph_handle_s* h, int nrhs, In in, Epi epi, hipStream_t s) {
  const Geom& g = h->g;
  const int S = (g.Q <= NT) ? NT / g.Q : 1;
  const size_t lds = 4 * (size_t)S * g.N * sizeof(T);
  auto kern = k_mtm<T, NT, MS, In, Epi>;
  {
    hipError_t e = allow_lds((const void*)kern, lds);
    if (e != hipSuccess) return e;
  }
  const int Tch = pick_chunk(g, nrhs, S, resident_slots((const void*)kern, NT, lds));
  const int nchunks = (g.Ltau + Tch - 1) / Tch;
  const int nblk = (nchunks + S - 1) / S;
  hipLaunchKernelGGL(kern, dim3(nblk * nrhs), dim3(NT), lds, s, g,
                     (const T*)(sizeof(T) == 8 ? (const void*)h->E64 : (const void*)h->E32),
                     (T)h->th, Tch, nblk, in, epi);
  return hipGetLastError();
}

// Fused operator launch (plain apply).
template <typename T, class In, class Epi>
hipError_t launch_mtm(const fph_handle_s* h, int nrhs, In in, Epi epi, hipStream_t s) {
  // One plaquette per thread; up to 1024 plaquettes (L <= 64) per slice.
  const int Q = h->g.Q;
  if (Q <= 64) return launch_mtm_cfg<T, 64, 1>(h, nrhs, in, epi, s);
  if (Q <= 256) return launch_mtm_cfg<T, 256, 1>(h, nrhs, in, epi, s);
  if (Q <= 512) return launch_mtm_cfg<T, 512, 1>(h, nrhs, in, epi, s);
  return launch_mtm_cfg<T, 1024, 1>(h, nrhs, in, epi, s);
}

// The operator kernel of a solver slot (k_slot_mtm), TI the iteration
// precision; LDS sized for the FP64 residual path.
template <typename TI, int NT>
hipError_t launch_slot_mtm_cfg(const fph_handle_s* h, int nrhs, const SlotArgs<TI>& a,
                               StateSeq& sq, hipStream_t s) {
  const Geom& g = h->g;
  const int S = (g.Q <= NT) ? NT / g.Q : 1;
  const size_t lds = 4 * (size_t)S * g.N * sizeof(double);
  // Small systems are latency bound: there the first slices are loaded
  // ahead of the solver state, both direction buffers included.
  const bool pf = (long)g.d * nrhs <= (1L << 20);
  auto kern = pf ? k_slot_mtm<TI, NT, 1, true> : k_slot_mtm<TI, NT, 1, false>;
  {
    hipError_t e = allow_lds((const void*)kern, lds);
    if (e != hipSuccess) return e;
  }
  const int Tch = pick_chunk(g, nrhs, S, resident_slots((const void*)kern, NT, lds));
  const int nchunks = (g.Ltau + Tch - 1) / Tch;
  const int nblk = (nchunks + S - 1) / S;
  if (nblk > kPHalf) return hipErrorInvalidConfiguration;  // two-value partials
  const StIO io = sq.next();
  hipLaunchKernelGGL(kern, dim3(nblk * nrhs), dim3(NT), lds, s, g, Tch, nblk, a, io);
  return hipGetLastError();
}

template <typename TI>
hipError_t launch_slot_mtm(const fph_handle_s* h, int nrhs, const SlotArgs<TI>& a, StateSeq& sq,
                           hipStream_t s) {
  const int Q = h->g.Q;
  if (Q <= 64) return launch_slot_mtm_cfg<TI, 64>(h, nrhs, a, sq, s);
  if (Q <= 256) return launch_slot_mtm_cfg<TI, 256>(h, nrhs, a, sq, s);
  if (Q <= 512) return launch_slot_mtm_cfg<TI, 512>(h, nrhs, a, sq, s);
  return launch_slot_mtm_cfg<TI, 1024>(h, nrhs, a, sq, s);
}

template <typename T, int NT, int MS, int MODE>
hipError_t launch_M_cfg(const fph_handle_s* h, int nrhs, const T* v, T* out, double coef,
                        const double* scale_dev, hipStream_t s) {
  const Geom& g = h->g;
  const int S = (g.Q <= NT) ? NT / g.Q : 1;
  const int nblk = (g.Ltau + S - 1) / S;
  const size_t lds = (size_t)S * g.N * sizeof(T);
  auto kern = k_apply_M<T, NT, MS, MODE>;
  {
    hipError_t e = allow_lds((const void*)kern, lds);
    if (e != hipSuccess) return e;
  }
  const T* E = (const T*)(sizeof(T) == 8 ? (const void*)h->E64 : (const void*)h->E32);
  const int ny = (MODE == 0) ? nrhs : (g.fs ? (nrhs + g.rpf - 1) / g.rpf : 1);
  hipLaunchKernelGGL(kern, dim3(nblk, ny), dim3(NT), lds, s, g, E, (T)h->th, 1, nrhs, v, out,
                     coef, scale_dev);
  return hipGetLastError();
}

template <typename T, int MODE>
hipError_t launch_M(const fph_handle_s* h, int nrhs, const T* v, T* out, double coef,
                    hipStream_t s, const double* scale_dev = nullptr) {
  const int Q = h->g.Q;
  if (Q <= 64) return launch_M_cfg<T, 64, 1, MODE>(h, nrhs, v, out, coef, scale_dev, s);
  if (Q <= 256) return launch_M_cfg<T, 256, 1, MODE>(h, nrhs, v, out, coef, scale_dev, s);
  if (Q <= 512) return launch_M_cfg<T, 512, 1, MODE>(h, nrhs, v, out, coef, scale_dev, s);
  return launch_M_cfg<T, 1024, 1, MODE>(h, nrhs, v, out, coef, scale_dev, s);
}

template <typename T, int NT, int MS>
hipError_t launch_MT_cfg(const fph_handle_s* h, int nrhs, const T* w, T* out, hipStream_t s) {
  const Geom& g = h->g;
  const int S = (g.Q <= NT) ? NT / g.Q : 1;
  const int nblk = (g.Ltau + S - 1) / S;
  const size_t lds = (size_t)S * g.N * sizeof(T);
  auto kern = k_apply_MT<T, NT, MS>;
  {
    hipError_t e = allow_lds((const void*)kern, lds);
    if (e != hipSuccess) return e;
  }
  const T* E = (const T*)(sizeof(T) == 8 ? (const void*)h->E64 : (const void*)h->E32);
  hipLaunchKernelGGL(kern, dim3(nblk, nrhs), dim3(NT), lds, s, g, E, (T)h->th, 1,
                     w, out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_MT(const fph_handle_s* h, int nrhs, const T* w, T* out, hipStream_t s) {
  const int Q = h->g.Q;
  if (Q <= 64) return launch_MT_cfg<T, 64, 1>(h, nrhs, w, out, s);
  if (Q <= 256) return launch_MT_cfg<T, 256, 1>(h, nrhs, w, out, s);
  if (Q <= 512) return launch_MT_cfg<T, 512, 1>(h, nrhs, w, out, s);
  return launch_MT_cfg<T, 1024, 1>(h, nrhs, w, out, s);
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
    case FPH_E_LATTICE: return "unsupported lattice (need even L in [4, 64], even Ltau in [2, 2048] with Ltau/2 = H1*H2, finite parameters)";
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
      lat->Ltau > kPHalf ||
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
  const double ch = std::cosh(lat->dtau * lat->t);
  h->th = std::tanh(lat->dtau * lat->t);
  h->c4 = ch * ch * ch * ch;
  h->a1 = h->a2 = 1.0;
  hipError_t e = hipGetDevice(&h->device);
  const long d = h->g.d;

#define ALLOC(ptr, bytes)                                   \
  if (e == hipSuccess) e = hipMalloc((void**)&(ptr), (bytes));
  // field tables for up to max_rhs fields (fph_set_fields)
  ALLOC(h->E64, (size_t)max_rhs * d * sizeof(double));
  ALLOC(h->E32, (size_t)max_rhs * d * sizeof(float));
  ALLOC(h->dbar64, (size_t)max_rhs * h->g.N * sizeof(double));
  ALLOC(h->dbar32, (size_t)max_rhs * h->g.N * sizeof(float));
  ALLOC(h->r64, vbytes(h, 8));
  ALLOC(h->pa64, vbytes(h, 8));
  ALLOC(h->pb64, vbytes(h, 8));
  ALLOC(h->Ap64, vbytes(h, 8));
  ALLOC(h->z64, vbytes(h, 8));
  ALLOC(h->u64b, vbytes(h, 8));
  ALLOC(h->u32, vbytes(h, 4));
  ALLOC(h->r32, vbytes(h, 4));
  ALLOC(h->pa32, vbytes(h, 4));
  ALLOC(h->pb32, vbytes(h, 4));
  ALLOC(h->Ap32, vbytes(h, 4));
  ALLOC(h->z32, vbytes(h, 4));
  ALLOC(h->st[0], max_rhs * sizeof(RhsState));
  ALLOC(h->st[1], max_rhs * sizeof(RhsState));
  ALLOC(h->part[0], (size_t)max_rhs * kPStride * sizeof(double));
  ALLOC(h->part[1], (size_t)max_rhs * kPStride * sizeof(double));
  ALLOC(h->fin_part, (size_t)max_rhs * kPStride * sizeof(double));
  ALLOC(h->stats_dev, max_rhs * sizeof(PcgStatsDev));
  ALLOC(h->tmp64, max_rhs * sizeof(double));
#undef ALLOC
  if (e == hipSuccess) e = hipHostMalloc((void**)&h->stats_pin, max_rhs * sizeof(PcgStatsDev), hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostMalloc((void**)&h->open_pin, 2 * sizeof(int), hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostMalloc((void**)&h->tmp_host, max_rhs * sizeof(double), hipHostMallocDefault);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&h->probe_ev[0], hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&h->probe_ev[1], hipEventDisableTiming);
  if (e == hipSuccess) e = hipMemset(h->st[0], 0, max_rhs * sizeof(RhsState));
  if (e == hipSuccess) e = hipMemset(h->st[1], 0, max_rhs * sizeof(RhsState));
  if (e == hipSuccess) e = pc_create(&h->pc, h->g, max_rhs);
  if (e == hipSuccess) e = scratch_address(h->device, &h->noalloc_part);
  h->pc.th = h->th;
  h->pc.c4 = h->c4;
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    fph_destroy(h);
    return fail_hip(e);
  }
  *out = h;
  return FPH_OK;
}

int fph_get_lattice(fph_handle_t h, fph_lattice_t* lat, int32_t* max_rhs) {
  if (h == nullptr) return FPH_E_NULL;
  if (lat) *lat = h->lat;
  if (max_rhs) *max_rhs = h->max_rhs;
  return FPH_OK;
}

int fph_destroy(fph_handle_t h) {
  if (h == nullptr) return FPH_E_NULL;
  (void)hipDeviceSynchronize();
  void* devptrs[] = {h->E64, h->E32, h->dbar64, h->dbar32, h->r64, h->pa64, h->pb64,
                     h->Ap64, h->z64, h->u64b, h->u32, h->r32, h->pa32, h->pb32, h->Ap32,
                     h->z32, h->st[0], h->st[1], h->part[0], h->part[1], h->fin_part,
                     h->stats_dev, h->tmp64};
  for (void* p : devptrs)
    if (p) (void)hipFree(p);
  if (h->stats_pin) (void)hipHostFree(h->stats_pin);
  if (h->open_pin) (void)hipHostFree(h->open_pin);
  if (h->tmp_host) (void)hipHostFree(h->tmp_host);
  for (hipEvent_t ev : h->probe_ev)
    if (ev) (void)hipEventDestroy(ev);
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
  h->g.fs = 0;
  h->g.rpf = 1;
  h->nfields = 0;
  hipLaunchKernelGGL(k_set_field, dim3(elem_blocks(d)), dim3(256), 0, s, d, x_dev,
                     h->lat.dtau, h->lat.alpha, h->lat.mu, h->c4, h->E64, h->E32);
  FPH_CHECK(hipGetLastError());
  hipLaunchKernelGGL(k_dbar, dim3((h->g.N + 63) / 64), dim3(64, 16), 0, s, h->g.N, h->g.Ltau,
                     h->E64, h->c4, h->dbar64, h->dbar32);
  FPH_CHECK(hipGetLastError());
  FPH_CHECK(pc_set_field(&h->pc, h->g, h->dbar64, h->lat.dtau, h->lat.t, h->a1, h->a2, s));
  h->have_field = true;
  return FPH_OK;
}

int fph_set_fields(fph_handle_t h, int32_t nfields, int32_t rhs_per_field, const double* x_dev,
                   double a1, double a2, void* stream) {
  if (h == nullptr || x_dev == nullptr) return FPH_E_NULL;
  if (!std::isfinite(a1) || !std::isfinite(a2) || rhs_per_field < 1) return FPH_E_ARG;
  if (nfields < 1 || nfields > h->max_rhs) return FPH_E_NRHS;
  hipStream_t s = (hipStream_t)stream;
  const long d = h->g.d;
  h->a1 = a1 > 0.0 ? a1 : 1.0;
  h->a2 = a2 > 0.0 ? a2 : 1.0;
  hipLaunchKernelGGL(k_set_field, dim3(elem_blocks((long)nfields * d)), dim3(256), 0, s,
                     (long)nfields * d, x_dev, h->lat.dtau, h->lat.alpha, h->lat.mu, h->c4, h->E64,
                     h->E32);
  FPH_CHECK(hipGetLastError());
  hipLaunchKernelGGL(k_dbar, dim3((h->g.N + 63) / 64, nfields), dim3(64, 16), 0, s, h->g.N,
                     h->g.Ltau, h->E64, h->c4, h->dbar64, h->dbar32);
  FPH_CHECK(hipGetLastError());
  for (int f = 0; f < nfields; ++f)
    FPH_CHECK(pc_set_field(&h->pc, h->g, h->dbar64 + (long)f * h->g.N, h->lat.dtau, h->lat.t,
                           h->a1, h->a2, s, f));
  h->g.fs = d;
  h->g.rpf = rhs_per_field;
  h->nfields = nfields;
  h->have_field = true;
  return FPH_OK;
}

int fermion_matvec(fph_handle_t h, int32_t op, int32_t prec, int32_t nrhs, const void* in_dev,
                   void* out_dev, void* stream) {
  if (h == nullptr || in_dev == nullptr || out_dev == nullptr) return FPH_E_NULL;
  if (!h->have_field) return FPH_E_NOFIELD;
  if (nrhs < 1 || nrhs > 65535 || (h->nfields && nrhs > h->nfields * h->g.rpf)) return FPH_E_NRHS;
  if (op < 0 || op > 2 || (prec != FPH_F64 && prec != FPH_F32)) return FPH_E_PREC;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  // Fused applies that move more than the 256 MB Infinity Cache write their
  // output with nontemporal stores.
  const size_t wbytes = prec == FPH_F64 ? 8 : 4;
  const bool stream_out = (size_t)(2 * nrhs + 1) * h->g.d * wbytes > ((size_t)256 << 20);
  if (prec == FPH_F64) {
    const double* in = (const double*)in_dev;
    double* out = (double*)out_dev;
    if (op == FPH_OP_M) e = launch_M<double, 0>(h, nrhs, in, out, 0.0, s);
    else if (op == FPH_OP_MT) e = launch_MT<double>(h, nrhs, in, out, s);
    else if (stream_out) e = launch_mtm<double>(h, nrhs, InPlain<double>{in}, EpiStream<double>{out}, s);
    else e = launch_mtm<double>(h, nrhs, InPlain<double>{in}, EpiStore<double>{out}, s);
  } else {
    const float* in = (const float*)in_dev;
    float* out = (float*)out_dev;
    if (op == FPH_OP_M) e = launch_M<float, 0>(h, nrhs, in, out, 0.0, s);
    else if (op == FPH_OP_MT) e = launch_MT<float>(h, nrhs, in, out, s);
    else if (stream_out) e = launch_mtm<float>(h, nrhs, InPlain<float>{in}, EpiStream<float>{out}, s);
    else e = launch_mtm<float>(h, nrhs, InPlain<float>{in}, EpiStore<float>{out}, s);
  }
  if (e != hipSuccess) return fail_hip(e);
  return FPH_OK;
}

int fermion_force(fph_handle_t h, int32_t nrhs, const double* u_dev, double* grad_dev,
                  double scale, const double* scale_dev, void* stream) {
  if (h == nullptr || u_dev == nullptr || grad_dev == nullptr) return FPH_E_NULL;
  if (!h->have_field) return FPH_E_NOFIELD;
  if (nrhs < 1 || (h->nfields && nrhs > h->nfields * h->g.rpf)) return FPH_E_NRHS;
  if (!std::isfinite(scale)) return FPH_E_ARG;
  const double coef = -2.0 * h->lat.dtau * h->lat.alpha * scale;
  hipError_t e = launch_M<double, 1>(h, nrhs, u_dev, grad_dev, coef, (hipStream_t)stream, scale_dev);
  if (e != hipSuccess) return fail_hip(e);
  return FPH_OK;
}

int fermion_action(fph_handle_t h, int32_t nrhs, const double* b_dev, const double* u_dev,
                   double* out_dev, void* stream) {
  if (h == nullptr || b_dev == nullptr || u_dev == nullptr || out_dev == nullptr) return FPH_E_NULL;
  if (nrhs < 1 || nrhs > h->max_rhs) return FPH_E_NRHS;
  hipStream_t s = (hipStream_t)stream;
  const int nb = elem_blocks(h->g.d);
  hipLaunchKernelGGL(k_dot_partials, dim3(nb, nrhs), dim3(256), 0, s, h->g.d, b_dev, u_dev,
                     h->tmp_part(), (long)kPStride);
  FPH_CHECK(hipGetLastError());
  hipLaunchKernelGGL(k_sum_partials, dim3(nrhs), dim3(256), 0, s, nb, (const double*)h->tmp_part(),
                     (long)kPStride, out_dev);
  FPH_CHECK(hipGetLastError());
  return FPH_OK;
}

int fermion_action_noalloc(fph_handle_t h, int32_t nrhs, const double* b_dev,
                           const double* u_dev, double* out_dev, void* stream) {
  if (h == nullptr || b_dev == nullptr || u_dev == nullptr || out_dev == nullptr) return FPH_E_NULL;
  if (nrhs < 1 || nrhs > h->max_rhs || nrhs > kNoAllocMaxRhs) return FPH_E_NRHS;
  int dev = -1;
  FPH_CHECK(hipGetDevice(&dev));
  if (dev != h->device || h->noalloc_part == nullptr) return FPH_E_ARG;
  const int nb = elem_blocks(h->g.d);
  if (nb > kNoAllocMaxBlocks) return FPH_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_dot_partials, dim3(nb, nrhs), dim3(256), 0, s, h->g.d, b_dev, u_dev,
                     h->noalloc_part, (long)kNoAllocMaxBlocks);
  FPH_CHECK(hipGetLastError());
  hipLaunchKernelGGL(k_sum_partials, dim3(nrhs), dim3(256), 0, s, nb,
                     (const double*)h->noalloc_part, (long)kNoAllocMaxBlocks, out_dev);
  FPH_CHECK(hipGetLastError());
  return FPH_OK;
}

int fph_precond_apply(fph_handle_t h, int32_t op, int32_t prec, int32_t nrhs, const void* in_dev,
                      void* out_dev, void* stream) {
  if (h == nullptr || in_dev == nullptr || out_dev == nullptr) return FPH_E_NULL;
  if (!h->have_field) return FPH_E_NOFIELD;
  if (nrhs < 1 || nrhs > h->max_rhs || (h->nfields && nrhs > h->nfields * h->g.rpf)) return FPH_E_NRHS;
  if (op < 0 || op > 2 || (prec != FPH_F64 && prec != FPH_F32)) return FPH_E_PREC;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  StateSeq sq{{nullptr, nullptr}, {nullptr, nullptr}, 0, 0, false};
  if (prec == FPH_F64)
    e = pc_apply<double>(&h->pc, h->g, h->dbar64, op, nrhs, (const double*)in_dev,
                         (double*)out_dev, nullptr, sq, s);
  else
    e = pc_apply<float>(&h->pc, h->g, h->dbar32, op, nrhs, (const float*)in_dev,
                        (float*)out_dev, nullptr, sq, s);
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

// Buffers of one precision for a solve.
template <typename T>
struct Work {
  T *r, *z, *pa, *pb, *Ap;
  const T* dbar;
};

// One slot (fph_solve.h): the operator kernel, then the CG update (without
// preconditioner) or the forward transform with the update, the series
// F F^T and the inverse transform with r.z.  `uit` is the vector the update
// advances: u_dev in FP64, the FP32 correction in FP32-refined solves.
template <typename TI>
hipError_t enqueue_slot(fph_handle_s* h, int nrhs, bool pre, const SlotArgs<TI>& a, TI* uit,
                        const Work<TI>& w, StateSeq& sq, hipStream_t s) {
  hipError_t e = launch_slot_mtm<TI>(h, nrhs, a, sq, s);
  if (e != hipSuccess) return e;
  if (!pre) {
    const int nb = elem_blocks(h->g.d);
    hipLaunchKernelGGL(k_cg_update<TI>, dim3(nb, nrhs), dim3(256), 0, s, h->g.d, uit,
                       (const TI*)w.pa, (const TI*)w.pb, w.r, (const TI*)w.Ap, sq.next());
    return hipGetLastError();
  }
  return pc_cg_update<TI>(&h->pc, h->g, w.dbar, nrhs, uit, w.pa, w.pb, w.r, w.Ap, w.z, sq, s);
}

// A solve as a fixed sequence of launches: start, `total` slots, finish.
struct SolveRun {
  fph_handle_s* h;
  int nrhs;
  const double* b;
  double* u;
  bool pre, mixed, zero;
  long total;  // 1 + maxiter + max_outer
  SolveInit init;
  StateSeq sq;
  SlotArgs<double> a64;
  SlotArgs<float> a32;
  Work<double> w64;
  Work<float> w32;

  SolveRun(fph_handle_s* hh, int nr, const double* bb, double* uu, const fph_pcg_opts_t* o)
      : h(hh), nrhs(nr), b(bb), u(uu) {
    pre = o->use_precond != 0;
    mixed = o->prec == FPH_F32_REFINED;
    zero = o->zero_guess != 0;
    const int max_outer = o->max_outer > 0 ? o->max_outer : kDefaultMaxOuter;
    total = 1L + o->maxiter + max_outer;
    init.tol = o->tol;
    // Replacement factor: FP32 CG drifts from the true residual at a rate
    // set by the condition number, which the preconditioner lowers.
    init.rdelta = o->ru_delta > 0.0 ? std::min(o->ru_delta, 0.5) : (pre ? 0.1 : 0.3);
    init.maxiter = o->maxiter;
    init.max_outer = max_outer;
    init.refined = mixed ? 1 : 0;
    init.pad = 0;
    sq = StateSeq{{h->st[0], h->st[1]}, {h->part[0], h->part[1]}, 0, pre ? 1 : 0, true};
    w64 = Work<double>{h->r64, h->z64, h->pa64, h->pb64, h->Ap64, h->dbar64};
    w32 = Work<float>{h->r32, h->z32, h->pa32, h->pb32, h->Ap32, h->dbar32};
    a64 = SlotArgs<double>{h->E64, h->E64, h->th, h->th, pre ? w64.z : w64.r, w64.pa, w64.pb,
                           w64.Ap, b, w64.r, u, h->u64b, h->u32};
    a32 = SlotArgs<float>{h->E32, h->E64, (float)h->th, h->th, pre ? w32.z : w32.r, w32.pa,
                          w32.pb, w32.Ap, b, w32.r, u, h->u64b, h->u32};
  }

  hipError_t start(hipStream_t s) {
    hipLaunchKernelGGL(k_solve_init, dim3(1), dim3(64), 0, s, nrhs, init, sq.latest());
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !zero) return e;
    const long n = (long)nrhs * h->g.d;
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)std::min<long>((n + 1023) / 1024, 2048)),
                       dim3(256), 0, s, n, u);
    return hipGetLastError();
  }

  hipError_t slots(long n, hipStream_t s) {
    for (long k = 0; k < n; ++k) {
      const hipError_t e = mixed ? enqueue_slot<float>(h, nrhs, pre, a32, h->u32, w32, sq, s)
                                 : enqueue_slot<double>(h, nrhs, pre, a64, u, w64, sq, s);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }

  hipError_t finish(PcgStatsDev* stats, hipStream_t s) {
    const int nb = elem_blocks(h->g.d);
    hipLaunchKernelGGL(k_solve_final, dim3(nb, nrhs), dim3(256), 0, s, h->g.d,
                       (const RhsState*)sq.latest(), b, u, (const double*)h->u64b,
                       (const float*)h->u32, h->fin_part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_solve_stats, dim3(nrhs), dim3(256), 0, s, nb,
                       (const RhsState*)sq.latest(), (const double*)h->fin_part, stats);
    return hipGetLastError();
  }
};

// The one-launch cooperative FP32-refined solve (fph_coop.h) for one
// right-hand side.  Workgroups own chunks of slices; the chunk length is
// the shortest that keeps the workgroup count within the exchange's limit
// (kCoopMaxBlocks), co-residency, and `target` workgroups.
template <int NT>
hipError_t coop_launch(fph_handle_s* h, const double* b, double* u, const fph_pcg_opts_t* opts,
                       double delta, int target, CoopStats* out, hipStream_t s) {
  const Geom& g = h->g;
  const int S = (g.Q <= NT) ? NT / g.Q : 1;
  const size_t lds = 4 * (size_t)S * g.N * sizeof(double);
  const void* kern = (const void*)k_cg_coop<NT>;
  hipError_t e = allow_lds(kern, lds);
  if (e != hipSuccess) return e;
  int per_cu = 0, ncu = 0, dev = 0;
  if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
  if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, NT, lds)) != hipSuccess)
    return e;
  if ((e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
    return e;
  const int cap = std::min(kCoopMaxBlocks, std::max(1, per_cu) * ncu);
  int Tch = 1, nblk = 0;
  for (Tch = 1; Tch <= g.Ltau; ++Tch) {
    nblk = ((g.Ltau + Tch - 1) / Tch + S - 1) / S;
    if (nblk <= std::min(cap, target)) break;
  }
  if (nblk > cap) return hipErrorInvalidConfiguration;
  // exchange regions (empty; kRegions * kCoopMaxBlocks * 2 words = the
  // first kPStride partials of part[0]) and the abort flag (in part[1],
  // after the statistics)
  static_assert((long)kRegions * kCoopMaxBlocks * 2 <= kPStride, "exchange regions");
  uint64_t* slots = reinterpret_cast<uint64_t*>(h->part[0]);
  uint64_t* abort_flag = reinterpret_cast<uint64_t*>(h->part[1]) + 64;
  const long nslots = (long)kRegions * kCoopMaxBlocks * 2;
  hipLaunchKernelGGL(k_fill_u64, dim3(64), dim3(256), 0, s, slots, nslots, kEmptySlot);
  hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, s, abort_flag, 1L, (uint64_t)0);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  CoopArgs a;
  a.g = g;
  a.th32 = (float)h->th;
  a.th = h->th;
  a.E32 = h->E32;
  a.E64 = h->E64;
  a.b = b;
  a.u = u;
  a.r = h->r32;
  a.pa = h->pa32;
  a.pb = h->pb32;
  a.Ap = h->Ap32;
  a.u32 = h->u32;
  a.x = CoopExchange{slots, abort_flag, nblk};
  a.out = out;
  a.Tch = Tch;
  a.tol = opts->tol;
  a.maxiter = opts->maxiter;
  a.delta = delta;
  a.zero_guess = opts->zero_guess;
  void* args[] = {&a};
  return hipLaunchCooperativeKernel(kern, dim3(nblk), dim3(NT), args, (unsigned)lds, s);
}

// Statistics of a cooperative solve in the layout of fph_pcg_stats_t, with
// S_F from the partials of b . u.
__global__ void __launch_bounds__(256)
k_coop_stats(int nb, const CoopStats* __restrict__ in, const double* __restrict__ part,
             PcgStatsDev* __restrict__ out) {
  __shared__ double red_sh[4];
  const double act = reduce_partials<256>(part, nb, red_sh);
  if (threadIdx.x == 0) {
    const CoopStats c = *in;
    PcgStatsDev o;
    o.status = c.status;
    o.iters = c.iters;
    o.outer_iters = c.outer;
    o.matvecs = c.matvecs;
    o.rel_resid = c.bb > 0.0 ? sqrt(c.rr_true / c.bb) : 0.0;
    o.action = act;
    *out = o;
  }
}

hipError_t coop_enqueue(fph_handle_s* h, const double* b_dev, double* u_dev,
                        const fph_pcg_opts_t* opts, PcgStatsDev* stats, hipStream_t s) {
  CoopStats* out = reinterpret_cast<CoopStats*>(h->part[1]);
  const int Q = h->g.Q;
  const int target = opts->chunk > 0 ? opts->chunk : 128;
  const double delta = opts->ru_delta > 0.0 ? std::min(opts->ru_delta, 0.5) : 0.3;
  hipError_t e;
  if (Q <= 64) e = coop_launch<64>(h, b_dev, u_dev, opts, delta, target, out, s);
  else if (Q <= 256) e = coop_launch<256>(h, b_dev, u_dev, opts, delta, target, out, s);
  else if (Q <= 512) e = coop_launch<512>(h, b_dev, u_dev, opts, delta, target, out, s);
  else e = coop_launch<1024>(h, b_dev, u_dev, opts, delta, target, out, s);
  if (e != hipSuccess) return e;
  const int nb = elem_blocks(h->g.d);
  hipLaunchKernelGGL(k_dot_partials, dim3(nb, 1), dim3(256), 0, s, h->g.d, b_dev,
                     (const double*)u_dev, h->fin_part, (long)kPStride);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_coop_stats, dim3(1), dim3(256), 0, s, nb, (const CoopStats*)out,
                     (const double*)h->fin_part, stats);
  return hipGetLastError();
}

int check_solve(const fph_handle_s* h, int nrhs, const double* b_dev, const double* u_dev,
                const fph_pcg_opts_t* opts) {
  if (h == nullptr || b_dev == nullptr || u_dev == nullptr || opts == nullptr) return FPH_E_NULL;
  if (!h->have_field) return FPH_E_NOFIELD;
  if (nrhs < 1 || nrhs > h->max_rhs || (h->nfields && nrhs > h->nfields * h->g.rpf))
    return FPH_E_NRHS;
  if (opts->prec != FPH_F64 && opts->prec != FPH_F32_REFINED) return FPH_E_PREC;
  if (!(opts->tol >= 0.0) || opts->maxiter < 1 || opts->max_outer < 0 ||
      (opts->variant != 0 && opts->variant != 2))
    return FPH_E_ARG;
  if (opts->variant == 2 &&
      (opts->prec != FPH_F32_REFINED || opts->use_precond != 0 || nrhs != 1 || h->nfields))
    return FPH_E_ARG;
  return FPH_OK;
}

}  // namespace

extern "C" int pcg_solve(fph_handle_t h, int32_t nrhs, const double* b_dev, double* u_dev,
                         const fph_pcg_opts_t* opts, fph_pcg_stats_t* stats_dev, void* stream) {
  const int rc = check_solve(h, nrhs, b_dev, u_dev, opts);
  if (rc != FPH_OK) return rc;
  if (stats_dev == nullptr) return FPH_E_NULL;
  hipStream_t s = (hipStream_t)stream;
  PcgStatsDev* st = reinterpret_cast<PcgStatsDev*>(stats_dev);
  if (opts->variant == 2) {
    FPH_CHECK(coop_enqueue(h, b_dev, u_dev, opts, st, s));
    return FPH_OK;
  }
  SolveRun run(h, nrhs, b_dev, u_dev, opts);
  FPH_CHECK(run.start(s));
  FPH_CHECK(run.slots(run.total, s));
  FPH_CHECK(run.finish(st, s));
  return FPH_OK;
}

extern "C" int pcg_solve_sync(fph_handle_t h, int32_t nrhs, const double* b_dev, double* u_dev,
                              const fph_pcg_opts_t* opts, fph_pcg_stats_t* stats_host,
                              void* stream) {
  const int rc = check_solve(h, nrhs, b_dev, u_dev, opts);
  if (rc != FPH_OK) return rc;
  hipStream_t s = (hipStream_t)stream;
  if (opts->variant == 2) {
    FPH_CHECK(coop_enqueue(h, b_dev, u_dev, opts, h->stats_dev, s));
  } else {
    // The same launches as pcg_solve, in chunks of slots; after each chunk
    // a probe kernel writes how many right-hand sides are still open to
    // pinned host memory.  The host waits for the probe of the previous
    // chunk only (so the GPU always has a chunk queued) and stops
    // enqueueing once it reads zero; slots already queued return at once.
    SolveRun run(h, nrhs, b_dev, u_dev, opts);
    FPH_CHECK(run.start(s));
    int* open_dev = nullptr;
    FPH_CHECK(hipHostGetDevicePointer((void**)&open_dev, h->open_pin, 0));
    const long chunk = opts->chunk > 0 ? opts->chunk
                       : (h->g.d > kSlotChunkLargeAbove ? kDefaultSlotChunkLarge
                                                         : kDefaultSlotChunk);
    long enq = 0;
    for (int k = 0; enq < run.total; ++k) {
      const long n = std::min(chunk, run.total - enq);
      FPH_CHECK(run.slots(n, s));
      enq += n;
      hipLaunchKernelGGL(k_solve_open, dim3(1), dim3(64), 0, s, nrhs,
                         (const RhsState*)run.sq.latest(), open_dev + (k & 1));
      FPH_CHECK(hipGetLastError());
      FPH_CHECK(hipEventRecord(h->probe_ev[k & 1], s));
      if (k >= 1) {
        FPH_CHECK(hipEventSynchronize(h->probe_ev[(k - 1) & 1]));
        if (reinterpret_cast<volatile int*>(h->open_pin)[(k - 1) & 1] == 0) break;
      }
    }
    FPH_CHECK(run.finish(h->stats_dev, s));
  }
  FPH_CHECK(hipMemcpyAsync(h->stats_pin, h->stats_dev, nrhs * sizeof(PcgStatsDev),
                           hipMemcpyDeviceToHost, s));
  FPH_CHECK(hipStreamSynchronize(s));
  if (stats_host) std::memcpy(stats_host, h->stats_pin, nrhs * sizeof(PcgStatsDev));
  return FPH_OK;
}

// ============================================================ batches

// What a captured batch graph was made for.
struct BatchRunCfg {
  double tol, delta, a1, a2;
  int maxiter;
  bool pre;
};

struct fph_batch_s {
  int nsys;
  int nitems;
  std::vector<fph_system_t> sys;
  std::vector<long> eoff;     // offset of each system's field in E64/E32
  std::vector<long> noff;     // offset of each system's sites in the dbar arrays
  double* E64;
  float* E32;
  float* work;
  BatchItem* items;
  BatchStat* stats;
  unsigned* queue;
  // preconditioner tables, per system
  double* dbar64;
  float* dbar32;
  PcInfo* info;
  int* np;                    // [Ltau] per system (offset eoff / N = tau offsets)
  std::vector<long> npoff, coff, twoff, foff;
  double2* coef64;
  float2* coef32;
  double2 *tw64, *W64, *F64;
  float2 *tw32, *W32, *F32;
  int nt, ms, per_cu;         // launch shape
  int num_cu;
  int qmax;
  size_t lds_pc;              // LDS of the transforms and the series (bytes, largest system)
  hipStream_t cap;            // capture stream
  hipGraphExec_t exec;
  bool have_graph;
  BatchRunCfg gcfg;           // configuration the graph was captured with
};

namespace {

bool same_cfg(const BatchRunCfg& a, const BatchRunCfg& c) {
  return a.tol == c.tol && a.maxiter == c.maxiter && a.delta == c.delta && a.pre == c.pre &&
         a.a1 == c.a1 && a.a2 == c.a2;
}

BatchRunCfg batch_cfg(const fph_pcg_opts_t* o) {
  BatchRunCfg c;
  c.tol = o->tol;
  c.maxiter = o->maxiter;
  c.pre = o->use_precond != 0;
  // FP32 residual-replacement factor (as pcg_solve): shorter with the preconditioner.
  c.delta = o->ru_delta > 0.0 ? std::min(o->ru_delta, 0.5) : (c.pre ? 0.1 : 0.3);
  c.a1 = o->cheb_a1 > 0.0 ? o->cheb_a1 : 1.0;
  c.a2 = o->cheb_a2 > 0.0 ? o->cheb_a2 : 1.0;
  return c;
}

template <int NT, int MS>
hipError_t batch_launch(fph_batch_s* b, const BatchRunCfg& c, hipStream_t s) {
  // LDS: four FP64 slices per chunk, chunks side by side (largest over
  // systems); with the preconditioner also the transforms and the series.
  long sn = 0;
  for (const auto& sy : b->sys) {
    const int N = sy.lat.L * sy.lat.L, Q = N / 4;
    const int S = (Q <= NT) ? NT / Q : 1;
    sn = std::max<long>(sn, (long)S * N);
  }
  size_t lds = 4 * (size_t)sn * sizeof(double);
  if (c.pre) lds = std::max(lds, b->lds_pc);
  auto kern = k_batch_solve<NT, MS>;
  {
    hipError_t e = allow_lds((const void*)kern, lds);
    if (e != hipSuccess) return e;
  }
  const int grid = std::max(1, std::min(b->nitems, b->num_cu * b->per_cu));
  hipLaunchKernelGGL(kern, dim3(grid), dim3(NT), lds, s, b->items, b->nitems, b->queue, c.tol,
                     c.maxiter, c.delta, c.pre ? 1 : 0, b->stats);
  return hipGetLastError();
}

// Field setup of every system (with the preconditioner: dbar, bounds,
// N_P and the Chebyshev coefficients of App. C as in fph_set_field), queue
// reset and the persistent solve.
hipError_t batch_enqueue(fph_batch_s* b, const BatchRunCfg& c, hipStream_t s) {
  for (int k = 0; k < b->nsys; ++k) {
    const fph_lattice_t& L = b->sys[k].lat;
    const int N = L.L * L.L;
    const long d = (long)N * L.Ltau;
    const double ch = std::cosh(L.dtau * L.t);
    const double c4 = ch * ch * ch * ch;
    hipLaunchKernelGGL(k_set_field, dim3(elem_blocks(d)), dim3(256), 0, s, d, b->sys[k].x_dev,
                       L.dtau, L.alpha, L.mu, c4, b->E64 + b->eoff[k], b->E32 + b->eoff[k]);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (!c.pre) continue;
    hipLaunchKernelGGL(k_dbar, dim3((N + 63) / 64), dim3(64, 16), 0, s, N, L.Ltau,
                       (const double*)(b->E64 + b->eoff[k]), c4, b->dbar64 + b->noff[k],
                       b->dbar32 + b->noff[k]);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_pc_bounds, dim3(1), dim3(256), 0, s, N, L.Ltau,
                       (const double*)(b->dbar64 + b->noff[k]), L.dtau, L.t, c.a1, c.a2,
                       b->info + k, b->np + b->npoff[k]);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_pc_coef, dim3(L.Ltau / 2), dim3(256), 0, s, L.Ltau,
                       (const PcInfo*)(b->info + k), (const int*)(b->np + b->npoff[k]),
                       b->coef64 + b->coff[k], b->coef32 + b->coff[k]);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, s, b->queue);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (b->nt == 256 && b->ms == 1) return batch_launch<256, 1>(b, c, s);
  if (b->nt == 128 && b->ms == 2) return batch_launch<128, 2>(b, c, s);
  if (b->nt == 512 && b->ms == 1) return batch_launch<512, 1>(b, c, s);
  return hipErrorInvalidValue;
}

// Batch statistics in the layout of fph_pcg_stats_t.
__global__ void k_copy_batch_stats(int n, const BatchStat* __restrict__ in,
                                   PcgStatsDev* __restrict__ out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const BatchStat s = in[k];
  out[k] = PcgStatsDev{s.status, s.iters, s.outer, s.matvecs, s.rel_resid, s.action};
}

hipError_t batch_graph(fph_batch_s* b, const BatchRunCfg& c) {
  if (b->have_graph) {
    (void)hipGraphExecDestroy(b->exec);
    b->have_graph = false;
  }
  hipGraph_t graph;
  hipError_t e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return e;
  hipError_t e2 = batch_enqueue(b, c, b->cap);
  e = hipStreamEndCapture(b->cap, &graph);
  if (e2 != hipSuccess) return e2;
  if (e != hipSuccess) return e;
  e = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return e;
  b->have_graph = true;
  b->gcfg = c;
  return hipSuccess;
}

int check_batch_opts(const fph_batch_s* b, const fph_pcg_opts_t* opts) {
  if (opts->prec != FPH_F32_REFINED) return FPH_E_PREC;
  if (!(opts->tol >= 0.0) || opts->maxiter < 1 || !std::isfinite(opts->cheb_a1) ||
      !std::isfinite(opts->cheb_a2))
    return FPH_E_ARG;
  // the in-workgroup series needs one even plaquette per thread
  if (opts->use_precond && b->nt < b->qmax) return FPH_E_ARG;
  return FPH_OK;
}

}  // namespace

extern "C" {

int fph_batch_create(fph_batch_t* out, const fph_system_t* sys, int32_t nsys) {
  if (out == nullptr || sys == nullptr) return FPH_E_NULL;
  *out = nullptr;
  if (nsys < 1) return FPH_E_ARG;
  long etot = 0, wtot = 0, ntot = 0, nptot = 0, ctot = 0, twtot = 0, ftot = 0;
  int nitems = 0, qmax = 1;
  size_t lds_pc = 0;
  for (int k = 0; k < nsys; ++k) {
    const fph_lattice_t& L = sys[k].lat;
    if (sys[k].x_dev == nullptr || sys[k].b_dev == nullptr || sys[k].u_dev == nullptr)
      return FPH_E_NULL;
    if (L.L < 4 || L.L % 2 || L.L > 32 || L.Ltau < 2 || L.Ltau % 2 || L.Ltau > kPHalf ||
        !pc_supported(L.Ltau) || !(L.dtau > 0.0) || !std::isfinite(L.t) ||
        !std::isfinite(L.mu) || !std::isfinite(L.alpha))
      return FPH_E_LATTICE;
    if (sys[k].nrhs < 1) return FPH_E_NRHS;
    const int N = L.L * L.L;
    const long d = (long)N * L.Ltau;
    const int H = L.Ltau / 2, H1 = pick_h1(H), H2 = H / H1;
    etot += d;
    wtot += 7 * d * sys[k].nrhs;
    ntot += N;
    nptot += L.Ltau;
    ctot += (long)H * kNPMax;
    twtot += H;
    ftot += (long)H1 * H1 + (long)H2 * H2;
    nitems += sys[k].nrhs;
    qmax = std::max(qmax, N / 4);
    lds_pc = std::max(lds_pc, (size_t)std::max(bpc_lds_tf(H, H1, H2, bpc_tile_n(N)),
                                               bpc_lds_series(L.L)) * sizeof(float2));
  }
  fph_batch_s* b = new fph_batch_s();
  b->nsys = nsys;
  b->nitems = nitems;
  b->qmax = qmax;
  b->lds_pc = lds_pc;
  b->sys.assign(sys, sys + nsys);
  b->have_graph = false;
  b->nt = qmax <= 256 ? 256 : 512;
  b->ms = 1;
  b->per_cu = 2;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  hipDeviceProp_t prop;
  if (e == hipSuccess) e = hipGetDeviceProperties(&prop, dev);
  b->num_cu = (e == hipSuccess) ? prop.multiProcessorCount : 256;
#define BALLOC(ptr, n) \
  if (e == hipSuccess) e = hipMalloc((void**)&(ptr), (size_t)(n) * sizeof(*(ptr)));
  BALLOC(b->E64, etot);
  BALLOC(b->E32, etot);
  BALLOC(b->work, wtot);
  BALLOC(b->items, nitems);
  BALLOC(b->stats, nitems);
  BALLOC(b->queue, 1);
  BALLOC(b->dbar64, ntot);
  BALLOC(b->dbar32, ntot);
  BALLOC(b->info, nsys);
  BALLOC(b->np, nptot);
  BALLOC(b->coef64, ctot);
  BALLOC(b->coef32, ctot);
  BALLOC(b->tw64, twtot);
  BALLOC(b->W64, twtot);
  BALLOC(b->tw32, twtot);
  BALLOC(b->W32, twtot);
  BALLOC(b->F64, ftot);
  BALLOC(b->F32, ftot);
#undef BALLOC
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
  if (e != hipSuccess) {
    fph_batch_destroy(b);
    return fail_hip(e);
  }
  // Per-system offsets, twiddle tables (they depend on Ltau only), and the
  // preconditioner view of each system.
  std::vector<BatchPc> pcs(nsys);
  {
    long eo = 0, no = 0, npo = 0, co = 0, two = 0, fo = 0;
    for (int k = 0; k < nsys; ++k) {
      const fph_lattice_t& L = sys[k].lat;
      const int N = L.L * L.L;
      const int H = L.Ltau / 2, H1 = pick_h1(H), H2 = H / H1;
      b->eoff.push_back(eo);
      b->noff.push_back(no);
      b->npoff.push_back(npo);
      b->coff.push_back(co);
      b->twoff.push_back(two);
      b->foff.push_back(fo);
      hipLaunchKernelGGL(k_pc_twiddles, dim3((H + H1 * H1 + H2 * H2 + 255) / 256), dim3(256), 0, 0,
                         H, H1, H2, L.Ltau, b->tw64 + two, b->W64 + two, b->F64 + fo,
                         b->tw32 + two, b->W32 + two, b->F32 + fo);
      const double ch = std::cosh(L.dtau * L.t);
      BatchPc& pc = pcs[k];
      pc.info = b->info + k;
      pc.np = b->np + npo;
      pc.coef = b->coef32 + co;
      pc.dbar = b->dbar32 + no;
      pc.tw = b->tw32 + two;
      pc.W = b->W32 + two;
      pc.F = b->F32 + fo;
      pc.c4 = (float)(ch * ch * ch * ch);
      pc.H = H;
      pc.H1 = H1;
      pc.H2 = H2;
      eo += (long)N * L.Ltau;
      no += N;
      npo += L.Ltau;
      co += (long)H * kNPMax;
      two += H;
      fo += (long)H1 * H1 + (long)H2 * H2;
    }
  }
  if ((e = hipGetLastError()) == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    fph_batch_destroy(b);
    return fail_hip(e);
  }
  // Work items, largest first (stable: system order within equal sizes).
  std::vector<BatchItem> items;
  items.reserve(nitems);
  long wo = 0;
  int gidx = 0;
  for (int k = 0; k < nsys; ++k) {
    const fph_lattice_t& L = sys[k].lat;
    Geom g;
    g.L = L.L;
    g.hL = L.L / 2;
    g.N = L.L * L.L;
    g.Q = g.N / 4;
    g.Ltau = L.Ltau;
    g.d = (long)g.N * L.Ltau;
    for (int j = 0; j < sys[k].nrhs; ++j) {
      BatchItem it;
      std::memset(&it, 0, sizeof(it));
      it.g = g;
      it.th = std::tanh(L.dtau * L.t);
      it.E64 = b->E64 + b->eoff[k];
      it.E32 = b->E32 + b->eoff[k];
      it.b = sys[k].b_dev + (long)j * g.d;
      it.u = sys[k].u_dev + (long)j * g.d;
      it.r = b->work + wo;
      it.pa = it.r + g.d;
      it.pb = it.pa + g.d;
      it.Ap = it.pb + g.d;
      it.u32 = it.Ap + g.d;
      it.z = it.u32 + g.d;
      it.Zw = reinterpret_cast<float2*>(it.z + g.d);
      it.pc = pcs[k];
      it.out = gidx++;
      wo += 7 * g.d;
      items.push_back(it);
    }
  }
  std::stable_sort(items.begin(), items.end(),
                   [](const BatchItem& a, const BatchItem& c) { return a.g.d > c.g.d; });
  e = hipMemcpy(b->items, items.data(), nitems * sizeof(BatchItem), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    fph_batch_destroy(b);
    return fail_hip(e);
  }
  *out = b;
  return FPH_OK;
}

int fph_batch_destroy(fph_batch_t b) {
  if (b == nullptr) return FPH_E_NULL;
  (void)hipDeviceSynchronize();
  if (b->have_graph) (void)hipGraphExecDestroy(b->exec);
  void* ptrs[] = {b->E64, b->E32, b->work, b->items, b->stats, b->queue, b->dbar64, b->dbar32,
                  b->info, b->np, b->coef64, b->coef32, b->tw64, b->W64, b->tw32, b->W32,
                  b->F64, b->F32};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  delete b;
  return FPH_OK;
}

int fph_batch_solve(fph_batch_t b, const fph_pcg_opts_t* opts, fph_pcg_stats_t* stats_dev,
                    void* stream) {
  if (b == nullptr || opts == nullptr) return FPH_E_NULL;
  const int rc = check_batch_opts(b, opts);
  if (rc != FPH_OK) return rc;
  hipStream_t s = (hipStream_t)stream;
  const BatchRunCfg c = batch_cfg(opts);
  if (!b->have_graph || !same_cfg(b->gcfg, c)) FPH_CHECK(batch_graph(b, c));
  FPH_CHECK(hipGraphLaunch(b->exec, s));
  if (stats_dev) {
    hipLaunchKernelGGL(k_copy_batch_stats, dim3((b->nitems + 255) / 256), dim3(256), 0, s,
                       b->nitems, (const BatchStat*)b->stats,
                       reinterpret_cast<PcgStatsDev*>(stats_dev));
    FPH_CHECK(hipGetLastError());
  }
  return FPH_OK;
}

int fph_batch_tune(fph_batch_t b, const fph_pcg_opts_t* opts, int32_t* best, void* stream) {
  if (b == nullptr || opts == nullptr) return FPH_E_NULL;
  if (opts->prec != FPH_F32_REFINED) return FPH_E_PREC;
  if (!(opts->tol >= 0.0) || opts->maxiter < 1) return FPH_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  const BatchRunCfg c = batch_cfg(opts);
  struct Cfg { int nt, ms, per_cu; };
  std::vector<Cfg> cands;
  for (int pc : {1, 2, 4}) {
    if (b->qmax <= 256) cands.push_back({256, 1, pc});
    if (!c.pre) cands.push_back({128, 2, pc});
    if (b->qmax <= 512) cands.push_back({512, 1, pc});
  }
  hipEvent_t e0, e1;
  FPH_CHECK(hipEventCreate(&e0));
  FPH_CHECK(hipEventCreate(&e1));
  float best_ms = 1e30f;
  Cfg best_cfg = {b->nt, b->ms, b->per_cu};
  for (const Cfg& cf : cands) {
    if (cf.ms * cf.nt < b->qmax) continue;  // a slice must fit one block
    b->nt = cf.nt;
    b->ms = cf.ms;
    b->per_cu = cf.per_cu;
    FPH_CHECK(batch_graph(b, c));
    FPH_CHECK(hipGraphLaunch(b->exec, s));  // warm-up
    FPH_CHECK(hipEventRecord(e0, s));
    FPH_CHECK(hipGraphLaunch(b->exec, s));
    FPH_CHECK(hipEventRecord(e1, s));
    FPH_CHECK(hipEventSynchronize(e1));
    float ms = 0.0f;
    FPH_CHECK(hipEventElapsedTime(&ms, e0, e1));
    if (ms < best_ms) {
      best_ms = ms;
      best_cfg = cf;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  b->nt = best_cfg.nt;
  b->ms = best_cfg.ms;
  b->per_cu = best_cfg.per_cu;
  FPH_CHECK(batch_graph(b, c));
  if (best) {
    best[0] = b->nt;
    best[1] = b->ms;
    best[2] = b->per_cu;
  }
  return FPH_OK;
}

}  // extern "C"
