// Stochastic Green's-function measurements with FFT acceleration (Sec. VI),
// built on the solver's C ABI (fermion_matvec, pcg_solve) plus the discrete
// Fourier transforms of this file.
//
// Grid: vectors are v[tau][i], i = x + L*y; a 3-D transform acts on
// (tau, y, x) as a spatial 2-D transform per time slice followed by a
// transform along tau per site.
//  * Space (k_fft_xy): one workgroup per time slice holds the L x L slice in
//    LDS and applies direct DFTs of length L along x, then along y.
//  * Time (k_fft_t): a workgroup holds S sites x Ltau slices in LDS and
//    applies the two-stage factorisation Ltau = P*Q (P, Q <= 64):
//      X[k1 + P k2] = sum_q w_Q^{q k2} w_T^{q k1} sum_p x[Q p + q] w_P^{p k1}.
//    The "twisted" variant multiplies the input by exp(-i pi tau/Ltau) first:
//    it is the transform, on the Ltau odd frequencies, of a sequence extended
//    antiperiodically to 2 Ltau slices, which is how the imaginary-time
//    antiperiodicity of G^ext (Eq. G_def-1) enters; its inverse multiplies
//    the output by exp(+i pi tau/Ltau).
// Transforms are unnormalised (forward exp(-2 pi i k n / n_d), inverse
// exp(+...)); the estimators fold every normalisation into one final scale.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "../../include/holstein_hmc.h"
#include "fph_internal.h"

namespace {

constexpr int kLdsMax = 150 * 1024;  // dynamic LDS budget per workgroup

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cfma(double2 a, double2 b, double2 c) {  // c + a b
  return make_double2(fma(a.x, b.x, fma(-a.y, b.y, c.x)), fma(a.x, b.y, fma(a.y, b.x, c.y)));
}
__device__ __forceinline__ double2 conjd(double2 a) { return make_double2(a.x, -a.y); }

// tw[m] = exp(-2 pi i m / n), m < n.
__global__ void __launch_bounds__(256) k_meas_twiddles(int n, double2* __restrict__ tw) {
  for (int m = blockIdx.x * 256 + threadIdx.x; m < n; m += gridDim.x * 256) {
    double s, c;
    sincospi(2.0 * m / n, &s, &c);
    tw[m] = make_double2(c, -s);
  }
}

enum { IN_COMPLEX = 0, IN_REAL = 1, IN_PRODUCT = 2 };
enum { OUT_COMPLEX = 0, OUT_REAL = 1 };

// Spatial DFT of one time slice per workgroup (grid: Ltau).  Input: complex
// in_c, real a, or the product a*b of two real vectors (slice tau of each).
// Output: complex, or the real part times `scale`.  Each thread computes G
// adjacent outputs of a row (or column) at once: one LDS read of an input
// feeds G independent multiply-add chains.
template <bool INV, int G>
__global__ void __launch_bounds__(256)
k_fft_xy(int L, int N, int in_mode, const double2* __restrict__ in_c, const double* __restrict__ a,
         const double* __restrict__ b, int out_mode, double scale, double2* __restrict__ out_c,
         double* __restrict__ out_r, const double2* __restrict__ twL) {
  extern __shared__ double2 sh[];
  double2* A = sh;          // [N]
  double2* B = sh + N;      // [N]
  double2* tw = sh + 2 * N; // [L]
  const long base = (long)blockIdx.x * N;
  for (int e = threadIdx.x; e < L; e += 256) tw[e] = INV ? conjd(twL[e]) : twL[e];
  for (int e = threadIdx.x; e < N; e += 256) {
    double2 v;
    if (in_mode == IN_COMPLEX) v = in_c[base + e];
    else if (in_mode == IN_REAL) v = make_double2(a[base + e], 0.0);
    else v = make_double2(a[base + e] * b[base + e], 0.0);
    A[e] = v;
  }
  __syncthreads();
  const int ng = L / G;  // groups of G outputs per row
  for (int gi = threadIdx.x; gi < ng * L; gi += 256) {  // along x: B[y][kx0 + j]
    const int y = gi / ng, kx0 = (gi - y * ng) * G;
    double2 acc[G];
    int m[G];
#pragma unroll
    for (int j = 0; j < G; ++j) {
      acc[j] = make_double2(0.0, 0.0);
      m[j] = 0;
    }
    for (int xx = 0; xx < L; ++xx) {
      const double2 v = A[y * L + xx];
#pragma unroll
      for (int j = 0; j < G; ++j) {
        acc[j] = cfma(v, tw[m[j]], acc[j]);
        m[j] += kx0 + j;
        if (m[j] >= L) m[j] -= L;
      }
    }
#pragma unroll
    for (int j = 0; j < G; ++j) B[y * L + kx0 + j] = acc[j];
  }
  __syncthreads();
  for (int gi = threadIdx.x; gi < ng * L; gi += 256) {  // along y: out[ky][kx0 + j]
    const int ky = gi / ng, kx0 = (gi - ky * ng) * G;
    double2 acc[G];
#pragma unroll
    for (int j = 0; j < G; ++j) acc[j] = make_double2(0.0, 0.0);
    int m = 0;
    for (int y = 0; y < L; ++y) {
      const double2 w = tw[m];
#pragma unroll
      for (int j = 0; j < G; ++j) acc[j] = cfma(B[y * L + kx0 + j], w, acc[j]);
      m += ky;
      if (m >= L) m -= L;
    }
    const long o = base + (long)ky * L + kx0;
#pragma unroll
    for (int j = 0; j < G; ++j) {
      if (out_mode == OUT_COMPLEX) out_c[o + j] = acc[j];
      else out_r[o + j] = scale * acc[j].x;
    }
  }
}

// Transform along tau of S sites per workgroup (grid: N/S), Ltau = P*Q.
// in/out complex [Ltau][N]; twist as described at the top of the file.  A
// thread computes one output row for all S sites: one twiddle feeds S
// independent multiply-add chains.
template <bool INV, int S>
__global__ void __launch_bounds__(256)
k_fft_t(int N, int T, int P, int Q, int twist, const double2* __restrict__ in,
        double2* __restrict__ out, const double2* __restrict__ twT) {
  extern __shared__ double2 sh[];
  double2* X = sh;              // [T][S]
  double2* Y = sh + T * S;      // [T][S]
  double2* tw = sh + 2 * T * S; // [T]
  const int site0 = blockIdx.x * S;
  for (int e = threadIdx.x; e < T; e += 256) tw[e] = INV ? conjd(twT[e]) : twT[e];
  for (int e = threadIdx.x; e < T * S; e += 256) {
    const int s = e % S, tau = e / S;
    double2 v = in[(long)tau * N + site0 + s];
    if (twist && !INV) {
      double sn, cs;
      sincospi((double)tau / T, &sn, &cs);
      v = cmul(v, make_double2(cs, -sn));
    }
    X[e] = v;
  }
  __syncthreads();
  // stage A: Y[q P + k1] = w_T^{q k1} sum_p X[Q p + q] w_P^{p k1},  w_P^j = tw[Q j]
  for (int r = threadIdx.x; r < T; r += 256) {
    const int k1 = r % P, q = r / P;
    double2 acc[S];
#pragma unroll
    for (int s = 0; s < S; ++s) acc[s] = make_double2(0.0, 0.0);
    int m = 0;
    const int step = (Q * k1) % T;
    for (int p = 0; p < P; ++p) {
      const double2 w = tw[m];
      const double2* xr = X + (Q * p + q) * S;
#pragma unroll
      for (int s = 0; s < S; ++s) acc[s] = cfma(xr[s], w, acc[s]);
      m += step;
      if (m >= T) m -= T;
    }
    const double2 post = tw[(q * k1) % T];
#pragma unroll
    for (int s = 0; s < S; ++s) Y[r * S + s] = cmul(acc[s], post);
  }
  __syncthreads();
  // stage B: out[k1 + P k2] = sum_q Y[q P + k1] w_Q^{q k2},  w_Q^j = tw[P j]
  for (int k = threadIdx.x; k < T; k += 256) {
    const int k1 = k % P, k2 = k / P;
    double2 acc[S];
#pragma unroll
    for (int s = 0; s < S; ++s) acc[s] = make_double2(0.0, 0.0);
    int m = 0;
    const int step = (P * k2) % T;
    for (int q = 0; q < Q; ++q) {
      const double2 w = tw[m];
      const double2* yr = Y + (q * P + k1) * S;
#pragma unroll
      for (int s = 0; s < S; ++s) acc[s] = cfma(yr[s], w, acc[s]);
      m += step;
      if (m >= T) m -= T;
    }
    double2 tk = make_double2(1.0, 0.0);
    if (twist && INV) {
      double sn, cs;
      sincospi((double)k / T, &sn, &cs);
      tk = make_double2(cs, sn);
    }
#pragma unroll
    for (int s = 0; s < S; ++s) out[(long)k * N + site0 + s] = cmul(acc[s], tk);
  }
}

// acc += conj(A) B over n values.
__global__ void __launch_bounds__(256)
k_acc_cross(long n, const double2* __restrict__ A, const double2* __restrict__ B, double2* __restrict__ acc) {
  for (long k = blockIdx.x * 256L + threadIdx.x; k < n; k += (long)gridDim.x * 256)
    acc[k] = cfma(conjd(A[k]), B[k], acc[k]);
}

// acc += conj(S) B; S += B (running sum over earlier vectors).
__global__ void __launch_bounds__(256)
k_acc_prefix(long n, double2* __restrict__ S, const double2* __restrict__ B, double2* __restrict__ acc) {
  for (long k = blockIdx.x * 256L + threadIdx.x; k < n; k += (long)gridDim.x * 256) {
    const double2 b = B[k];
    const double2 s = S[k];
    acc[k] = cfma(conjd(s), b, acc[k]);
    S[k] = make_double2(s.x + b.x, s.y + b.y);
  }
}

__global__ void __launch_bounds__(256) k_zero2(long n, double2* __restrict__ p) {
  for (long k = blockIdx.x * 256L + threadIdx.x; k < n; k += (long)gridDim.x * 256)
    p[k] = make_double2(0.0, 0.0);
}

int grid_for(long n) {
  const long b = (n + 255) / 256;
  return (int)(b < 1 ? 1 : (b > 4096 ? 4096 : b));
}

// Ltau = P*Q with P <= Q <= 64 and P + Q smallest; false if none.
bool factor_T(int T, int* P, int* Q) {
  int best = -1;
  for (int p = 1; p <= 64; ++p) {
    if (T % p) continue;
    const int q = T / p;
    if (q > 64 || p > q) continue;
    if (best < 0 || p + q < *P + *Q) {
      *P = p;
      *Q = q;
      best = p;
    }
  }
  return best > 0;
}

}  // namespace

struct fph_meas_s {
  fph_handle_t h;
  fph_lattice_t lat;
  int max_rhs;
  int L, N, T, P, Q, S;
  long d;
  double2 *twL, *twT;
  double2 *A, *B, *tmp, *acc, *acc2, *run;  // complex grids [Ltau][N]
  double* bvec;                              // max_rhs real vectors
  size_t lds_xy, lds_t;
};

namespace {

hipError_t launch_xy(const fph_meas_s* m, bool inv, int in_mode, const double2* in_c, const double* a,
                     const double* b, int out_mode, double scale, double2* out_c, double* out_r,
                     hipStream_t s) {
  const bool g4 = (m->L % 4) == 0;
  if (!inv && g4)
    hipLaunchKernelGGL((k_fft_xy<false, 4>), dim3(m->T), dim3(256), m->lds_xy, s, m->L, m->N, in_mode, in_c,
                       a, b, out_mode, scale, out_c, out_r, (const double2*)m->twL);
  else if (!inv)
    hipLaunchKernelGGL((k_fft_xy<false, 2>), dim3(m->T), dim3(256), m->lds_xy, s, m->L, m->N, in_mode, in_c,
                       a, b, out_mode, scale, out_c, out_r, (const double2*)m->twL);
  else if (g4)
    hipLaunchKernelGGL((k_fft_xy<true, 4>), dim3(m->T), dim3(256), m->lds_xy, s, m->L, m->N, in_mode, in_c,
                       a, b, out_mode, scale, out_c, out_r, (const double2*)m->twL);
  else
    hipLaunchKernelGGL((k_fft_xy<true, 2>), dim3(m->T), dim3(256), m->lds_xy, s, m->L, m->N, in_mode, in_c,
                       a, b, out_mode, scale, out_c, out_r, (const double2*)m->twL);
  return hipGetLastError();
}

template <bool INV>
hipError_t launch_t_inv(const fph_meas_s* m, int twist, const double2* in, double2* out, hipStream_t s) {
  dim3 g(m->N / m->S);
#define FPH_T_CASE(SS)                                                                              \
  case SS:                                                                                          \
    hipLaunchKernelGGL((k_fft_t<INV, SS>), g, dim3(256), m->lds_t, s, m->N, m->T, m->P, m->Q, twist, \
                       in, out, (const double2*)m->twT);                                          \
    break;
  switch (m->S) {
    FPH_T_CASE(1)
    FPH_T_CASE(2)
    FPH_T_CASE(4)
    FPH_T_CASE(8)
    FPH_T_CASE(16)
    default: return hipErrorInvalidValue;
  }
#undef FPH_T_CASE
  return hipGetLastError();
}

hipError_t launch_t(const fph_meas_s* m, bool inv, int twist, const double2* in, double2* out, hipStream_t s) {
  return inv ? launch_t_inv<true>(m, twist, in, out, s) : launch_t_inv<false>(m, twist, in, out, s);
}

// Forward 3-D transform of a real input (in_mode IN_REAL / IN_PRODUCT) into `out`.
hipError_t fwd3(const fph_meas_s* m, int in_mode, const double* a, const double* b, int twist,
                double2* out, hipStream_t s) {
  hipError_t e = launch_xy(m, false, in_mode, nullptr, a, b, OUT_COMPLEX, 0.0, m->tmp, nullptr, s);
  if (e != hipSuccess) return e;
  return launch_t(m, false, twist, m->tmp, out, s);
}

// Inverse 3-D transform of `in` (complex), real part times `scale` into out_r.
hipError_t inv3(const fph_meas_s* m, const double2* in, int twist, double scale, double* out_r,
                hipStream_t s) {
  hipError_t e = launch_t(m, true, twist, in, m->tmp, s);
  if (e != hipSuccess) return e;
  return launch_xy(m, true, IN_COMPLEX, m->tmp, nullptr, nullptr, OUT_REAL, scale, nullptr, out_r, s);
}

hipError_t zero2(const fph_meas_s* m, double2* p, hipStream_t s) {
  hipLaunchKernelGGL(k_zero2, dim3(grid_for(m->d)), dim3(256), 0, s, m->d, p);
  return hipGetLastError();
}

hipError_t cross(const fph_meas_s* m, double2* acc, hipStream_t s) {
  hipLaunchKernelGGL(k_acc_cross, dim3(grid_for(m->d)), dim3(256), 0, s, m->d, (const double2*)m->A,
                     (const double2*)m->B, acc);
  return hipGetLastError();
}

}  // namespace

#define MEAS_CHECK(call)                                      \
  do {                                                        \
    hipError_t e_ = (call);                                   \
    if (e_ != hipSuccess) return fph::record_hip_error(e_);   \
  } while (0)

#define MEAS_CALL(call)                \
  do {                                 \
    int rc_ = (call);                  \
    if (rc_ != FPH_OK) return rc_;     \
  } while (0)

extern "C" {

int fph_meas_destroy(fph_meas_t m) {
  if (m == nullptr) return FPH_E_NULL;
  (void)hipDeviceSynchronize();
  void* ptrs[] = {m->twL, m->twT, m->A, m->B, m->tmp, m->acc, m->acc2, m->run, m->bvec};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  delete m;
  return FPH_OK;
}

int fph_meas_create(fph_meas_t* out, fph_handle_t h, void* stream) {
  if (out == nullptr || h == nullptr) return FPH_E_NULL;
  *out = nullptr;
  fph_lattice_t lat;
  int32_t max_rhs = 0;
  MEAS_CALL(fph_get_lattice(h, &lat, &max_rhs));
  int P = 0, Q = 0;
  if (!factor_T(lat.Ltau, &P, &Q)) return FPH_E_LATTICE;
  const int N = lat.L * lat.L;
  const size_t lds_xy = (size_t)(2 * N + lat.L) * sizeof(double2);
  if (lds_xy > (size_t)kLdsMax) return FPH_E_LATTICE;
  // sites per workgroup along tau: a power of two dividing N, within the LDS
  // budget, and small enough to give at least 256 workgroups where possible
  int S = 16;
  while (S > 1 && ((size_t)(2 * S + 0) * lat.Ltau * sizeof(double2) + lat.Ltau * sizeof(double2) >
                       (size_t)kLdsMax || N / S < 256 || N % S))
    S /= 2;
  const size_t lds_t = (size_t)(2 * S * lat.Ltau + lat.Ltau) * sizeof(double2);
  if (lds_t > (size_t)kLdsMax) return FPH_E_LATTICE;
  fph_meas_s* m = new fph_meas_s();
  std::memset(m, 0, sizeof(*m));
  m->h = h;
  m->lat = lat;
  m->max_rhs = max_rhs;
  m->L = lat.L;
  m->N = N;
  m->T = lat.Ltau;
  m->P = P;
  m->Q = Q;
  m->S = S;
  m->d = (long)N * lat.Ltau;
  m->lds_xy = lds_xy;
  m->lds_t = lds_t;
  hipError_t e = hipSuccess;
#define ALLOC(ptr, bytes) \
  if (e == hipSuccess) e = hipMalloc((void**)&(ptr), (bytes));
  ALLOC(m->twL, m->L * sizeof(double2));
  ALLOC(m->twT, m->T * sizeof(double2));
  ALLOC(m->A, m->d * sizeof(double2));
  ALLOC(m->B, m->d * sizeof(double2));
  ALLOC(m->tmp, m->d * sizeof(double2));
  ALLOC(m->acc, m->d * sizeof(double2));
  ALLOC(m->acc2, m->d * sizeof(double2));
  ALLOC(m->run, m->d * sizeof(double2));
  ALLOC(m->bvec, (size_t)max_rhs * m->d * sizeof(double));
#undef ALLOC
  {
    const void* fns[] = {(const void*)k_fft_xy<false, 2>, (const void*)k_fft_xy<false, 4>,
                         (const void*)k_fft_xy<true, 2>,  (const void*)k_fft_xy<true, 4>,
                         (const void*)k_fft_t<false, 1>,  (const void*)k_fft_t<false, 2>,
                         (const void*)k_fft_t<false, 4>,  (const void*)k_fft_t<false, 8>,
                         (const void*)k_fft_t<false, 16>, (const void*)k_fft_t<true, 1>,
                         (const void*)k_fft_t<true, 2>,   (const void*)k_fft_t<true, 4>,
                         (const void*)k_fft_t<true, 8>,   (const void*)k_fft_t<true, 16>};
    for (const void* f : fns)
      if (e == hipSuccess) e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, kLdsMax);
  }
  hipStream_t s = (hipStream_t)stream;
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_meas_twiddles, dim3(1), dim3(256), 0, s, m->L, m->twL);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_meas_twiddles, dim3((m->T + 255) / 256), dim3(256), 0, s, m->T, m->twT);
    e = hipGetLastError();
  }
  if (e != hipSuccess) {
    fph_meas_destroy(m);
    return fph::record_hip_error(e);
  }
  *out = m;
  return FPH_OK;
}

int meas_fft(fph_meas_t m, int32_t inverse, int32_t twist, const double* in_dev, double* out_dev,
             void* stream) {
  if (m == nullptr || in_dev == nullptr || out_dev == nullptr) return FPH_E_NULL;
  if (in_dev == out_dev) return FPH_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  const double2* in = (const double2*)in_dev;
  double2* out = (double2*)out_dev;
  const int tw = twist != 0;
  if (!inverse) {
    MEAS_CHECK(launch_xy(m, false, IN_COMPLEX, in, nullptr, nullptr, OUT_COMPLEX, 0.0, m->tmp, nullptr, s));
    MEAS_CHECK(launch_t(m, false, tw, m->tmp, out, s));
  } else {
    MEAS_CHECK(launch_t(m, true, tw, in, m->tmp, s));
    MEAS_CHECK(launch_xy(m, true, IN_COMPLEX, m->tmp, nullptr, nullptr, OUT_COMPLEX, 0.0, out, nullptr, s));
  }
  return FPH_OK;
}

int green_vectors(fph_meas_t m, int32_t nvec, const double* xi_dev, double* gxi_dev,
                  const fph_pcg_opts_t* opts, fph_pcg_stats_t* stats_host, void* stream) {
  if (m == nullptr || xi_dev == nullptr || gxi_dev == nullptr || opts == nullptr) return FPH_E_NULL;
  if (nvec < 1) return FPH_E_NRHS;
  fph_pcg_opts_t oo = *opts;
  oo.zero_guess = 1;
  for (int r0 = 0; r0 < nvec; r0 += m->max_rhs) {
    const int nr = (nvec - r0 < m->max_rhs) ? nvec - r0 : m->max_rhs;
    MEAS_CALL(fermion_matvec(m->h, FPH_OP_MT, FPH_F64, nr, xi_dev + (long)r0 * m->d, m->bvec, stream));
    MEAS_CALL(pcg_solve_sync(m->h, nr, m->bvec, gxi_dev + (long)r0 * m->d, &oo,
                        stats_host ? stats_host + r0 : nullptr, stream));
  }
  return FPH_OK;
}

int green_average(fph_meas_t m, int32_t nvec, const double* xi_dev, const double* gxi_dev,
                  double* out_dev, void* stream) {
  if (m == nullptr || xi_dev == nullptr || gxi_dev == nullptr || out_dev == nullptr) return FPH_E_NULL;
  if (nvec < 1) return FPH_E_NRHS;
  hipStream_t s = (hipStream_t)stream;
  MEAS_CHECK(zero2(m, m->acc, s));
  for (int n = 0; n < nvec; ++n) {
    MEAS_CHECK(fwd3(m, IN_REAL, xi_dev + (long)n * m->d, nullptr, 1, m->A, s));
    MEAS_CHECK(fwd3(m, IN_REAL, gxi_dev + (long)n * m->d, nullptr, 1, m->B, s));
    MEAS_CHECK(cross(m, m->acc, s));
  }
  // GA = e^{i pi dtau/Ltau} IDFT3[sum_n conj(A_n) B_n] / (nvec Ncal^2), Ncal = N Ltau
  const double ncal = (double)m->d;
  MEAS_CHECK(inv3(m, m->acc, 1, 1.0 / ((double)nvec * ncal * ncal), out_dev, s));
  return FPH_OK;
}

int green_pair_products(fph_meas_t m, int32_t nvec, const double* xi_dev, const double* gxi_dev,
                        double* out_dev, void* stream) {
  if (m == nullptr || xi_dev == nullptr || gxi_dev == nullptr || out_dev == nullptr) return FPH_E_NULL;
  if (nvec < 2) return FPH_E_NRHS;
  hipStream_t s = (hipStream_t)stream;
  const long d = m->d;
  auto xi = [&](int n) { return xi_dev + (long)n * d; };
  auto gx = [&](int n) { return gxi_dev + (long)n * d; };
  const double npairs = 0.5 * (double)nvec * (double)(nvec - 1);
  const double scale = 1.0 / (npairs * (double)d * (double)d);
  // T1: (xi_n . xi_m) * (Gxi_n . Gxi_m);  T3: (xi_n . Gxi_m) * (xi_m . Gxi_n)
  MEAS_CHECK(zero2(m, m->acc, s));
  MEAS_CHECK(zero2(m, m->acc2, s));
  for (int a = 0; a < nvec; ++a)
    for (int b = a + 1; b < nvec; ++b) {
      MEAS_CHECK(fwd3(m, IN_PRODUCT, xi(a), xi(b), 0, m->A, s));
      MEAS_CHECK(fwd3(m, IN_PRODUCT, gx(a), gx(b), 0, m->B, s));
      MEAS_CHECK(cross(m, m->acc, s));
      MEAS_CHECK(fwd3(m, IN_PRODUCT, xi(a), gx(b), 0, m->A, s));
      MEAS_CHECK(fwd3(m, IN_PRODUCT, xi(b), gx(a), 0, m->B, s));
      MEAS_CHECK(cross(m, m->acc2, s));
    }
  MEAS_CHECK(inv3(m, m->acc, 0, scale, out_dev, s));
  MEAS_CHECK(inv3(m, m->acc2, 0, scale, out_dev + 2 * d, s));
  // T2: (xi_n . Gxi_n) * (xi_m . Gxi_m), n < m: sum_m conj(sum_{n<m} H_n) H_m
  MEAS_CHECK(zero2(m, m->acc, s));
  MEAS_CHECK(zero2(m, m->run, s));
  for (int n = 0; n < nvec; ++n) {
    MEAS_CHECK(fwd3(m, IN_PRODUCT, xi(n), gx(n), 0, m->B, s));
    hipLaunchKernelGGL(k_acc_prefix, dim3(grid_for(d)), dim3(256), 0, s, d, m->run, (const double2*)m->B,
                       m->acc);
    MEAS_CHECK(hipGetLastError());
  }
  MEAS_CHECK(inv3(m, m->acc, 0, scale, out_dev + d, s));
  return FPH_OK;
}

}  // extern "C"
