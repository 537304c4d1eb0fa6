// Hybrid Monte Carlo update of the phonon field (Sec. III, Algorithm 1),
// built on the solver's C ABI (fph_set_field, fermion_matvec, pcg_solve,
// fermion_force) plus the imaginary-time kernels of this file.
//
// Everything bosonic is diagonal in the Fourier basis over imaginary time:
// the force dS_B/dx = Q x (Eq. bosonic_force), the mass Mass = F^-1 Mtilde F
// (Eq. dynamical_M_def), and the constant force -dtau*alpha of the linear
// term lives in the w = 0 mode only.  Each operator is therefore a real
// symmetric circulant over tau, applied site by site, and the nt bosonic
// sub-steps of one time step compose into one affine map per mode.  The
// circulant kernels are built once per context from per-mode values.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/holstein_hmc.h"
#include "fph_internal.h"

namespace {

constexpr int kRows = 8;         // output time slices per lane (circulant kernel)
constexpr int kRedBlocks = 512;  // partial sums per reduction
constexpr int kNTab = 7;         // circulant tables: 2x2 step map, Mass^-1, sqrt Mass, Mass
constexpr int kEn = 16;          // device energy slots

enum { TAB_XX = 0, TAB_XP = 1, TAB_PX = 2, TAB_PP = 3, TAB_MINV = 4, TAB_MSQRT = 5, TAB_MASS = 6 };
enum { EN_SB_I = 0, EN_LIN_I, EN_R2, EN_K_I, EN_SB_F, EN_LIN_F, EN_K_F };

// ------------------------------------------------------------------ tables

// Per Fourier mode w: the nt-sub-step map of (x, p, 1) under
//   p -= h/2 (q x - f); x += h p / m; p -= h/2 (q x - f),
// with q = Qtilde_w (Eq. Qww_def, sine argument pi w/Ltau), m = Mtilde_w
// and f the constant force per slice (w = 0 only), composed by running the
// sub-steps on the three basis states.  vals[k][w]: the map's 2x2 block,
// 1/m, sqrt m, m.  cst[0..1]: the map's constant column in the w = 0 mode.
__global__ void __launch_bounds__(64)
k_hmc_modes(int Ltau, double dtau, double omega0, double m_reg, double h, int nt, double f_lin,
            double* __restrict__ vals, double* __restrict__ cst) {
  const int w = blockIdx.x * 64 + threadIdx.x;
  if (w >= Ltau) return;
  const double s = sinpi((double)w / Ltau);
  const double lap = 4.0 / (dtau * dtau) * s * s;
  const double q = dtau * (omega0 * omega0 + lap);
  double m = dtau;
  if (m_reg >= 0.0) {
    const double r = m_reg * m_reg + omega0 * omega0;
    m = dtau * (r + lap) / r;
  }
  const double f = (w == 0) ? f_lin : 0.0;
  double T[3][2];  // T[c] = (x, p) image of basis state c
  for (int c = 0; c < 3; ++c) {
    double x = (c == 0) ? 1.0 : 0.0, p = (c == 1) ? 1.0 : 0.0;
    const double one = (c == 2) ? 1.0 : 0.0;
    for (int k = 0; k < nt; ++k) {
      p -= 0.5 * h * (q * x - f * one);
      x += h * p / m;
      p -= 0.5 * h * (q * x - f * one);
    }
    T[c][0] = x;
    T[c][1] = p;
  }
  vals[TAB_XX * Ltau + w] = T[0][0];
  vals[TAB_XP * Ltau + w] = T[1][0];
  vals[TAB_PX * Ltau + w] = T[0][1];
  vals[TAB_PP * Ltau + w] = T[1][1];
  vals[TAB_MINV * Ltau + w] = 1.0 / m;
  vals[TAB_MSQRT * Ltau + w] = sqrt(m);
  vals[TAB_MASS * Ltau + w] = m;
  if (w == 0) {
    cst[0] = T[2][0];
    cst[1] = T[2][1];
  }
}

// tab[k][e] = K_k[(e - off) mod Ltau], K_k[j] = (1/Ltau) sum_w vals[k][w] cos(2 pi w j / Ltau):
// the real circulant of the even mode values, stored over the index range the
// sliding window of k_tau_circ reads (e in [0, ts)).  Launch: grid (ceil(ts/64), kNTab).
__global__ void __launch_bounds__(64)
k_hmc_tables(int Ltau, int ts, int off, const double* __restrict__ vals, double* __restrict__ tab) {
  const int e = blockIdx.x * 64 + threadIdx.x;
  const int k = blockIdx.y;
  if (e >= ts) return;
  const int j = (((e - off) % Ltau) + Ltau) % Ltau;
  const double* v = vals + (long)k * Ltau;
  double acc = 0.0;
  for (int w = 0; w < Ltau; ++w) {
    const int r = (int)(((long)w * j) % Ltau);
    acc += v[w] * cospi(2.0 * r / Ltau);
  }
  tab[(long)k * ts + e] = acc / Ltau;
}

// ------------------------------------------------------- circulant apply

// out_o[tau][i] = sum_n sum_s K_{o,n}[(tau - s) mod Ltau] in_n[s][i] + cst[o]
// for o < NO, n < NI (NI = NO = 1: one circulant; 2: the 2x2 step map).
// Lane = site, kRows output slices per wave.  The kernel values are uniform
// across the wave (scalar loads); a ring of kRows of them per (o, n) slides
// by one entry per input slice s: with t0 and s0 multiples of kRows, slot j
// of the ring holds K[m] for the unique m = j (mod kRows) in the current
// window, and output row j at step u reads slot (j - u) mod kRows.
// tab_{o,n} = tab + (o*NI + n)*ts, indexed by m + off.
// Launch: grid (ceil(N/64), ceil(Ltau/kRows), nvec), block 64.
template <int NI, int NO>
__global__ void __launch_bounds__(64)
k_tau_circ(int N, int Ltau, long d, int ts, int off, const double* __restrict__ tab,
           const double* __restrict__ cst, const double* __restrict__ in0,
           const double* __restrict__ in1, double* __restrict__ out0, double* __restrict__ out1) {
  constexpr int R = kRows;
  const int i = blockIdx.x * 64 + threadIdx.x;
  const bool act = i < N;
  const int ic = act ? i : 0;
  const int t0 = blockIdx.y * R;
  const long voff = (long)blockIdx.z * d;
  const double* in[2] = {in0 + voff, (NI > 1) ? in1 + voff : nullptr};
  double ring[NO][NI][R];
  double acc[NO][R];
#pragma unroll
  for (int o = 0; o < NO; ++o)
#pragma unroll
    for (int n = 0; n < NI; ++n)
#pragma unroll
      for (int j = 0; j < R; ++j) ring[o][n][j] = tab[(o * NI + n) * ts + off + t0 + j];
#pragma unroll
  for (int o = 0; o < NO; ++o)
#pragma unroll
    for (int j = 0; j < R; ++j) acc[o][j] = 0.0;

  for (int s0 = 0; s0 < Ltau; s0 += R) {
    double v[NI][R];
#pragma unroll
    for (int n = 0; n < NI; ++n)
#pragma unroll
      for (int u = 0; u < R; ++u) {
        const int s = s0 + u;
        v[n][u] = (s < Ltau) ? in[n][(long)s * N + ic] : 0.0;
      }
#pragma unroll
    for (int u = 0; u < R; ++u) {
#pragma unroll
      for (int o = 0; o < NO; ++o)
#pragma unroll
        for (int n = 0; n < NI; ++n)
#pragma unroll
          for (int j = 0; j < R; ++j)
            acc[o][j] = fma(ring[o][n][(j - u) & (R - 1)], v[n][u], acc[o][j]);
      const int m = t0 - s0 - u - 1;  // entering the window; leaving: m + R
#pragma unroll
      for (int o = 0; o < NO; ++o)
#pragma unroll
        for (int n = 0; n < NI; ++n) ring[o][n][(R - 1 - u) & (R - 1)] = tab[(o * NI + n) * ts + off + m];
    }
  }
  if (!act) return;
  double* out[2] = {out0 + voff, (NO > 1) ? out1 + voff : nullptr};
#pragma unroll
  for (int o = 0; o < NO; ++o) {
    const double c = cst ? cst[o] : 0.0;
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const int t = t0 + j;
      if (t < Ltau) out[o][(long)t * N + i] = acc[o][j] + c;
    }
  }
}

// ------------------------------------------------------------- reductions

template <int NT>
__device__ double block_sum(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < NT / 64; ++k) t += sh[k];
  __syncthreads();
  return t;
}

// part[0][b], part[1][b]: block partial sums of the S_B summand of Eq. (S_B)
// and of x, over x[Ltau][N] with x_{Ltau} = x_0.  Launch: grid kRedBlocks, block 256.
__global__ void __launch_bounds__(256)
k_sb_partials(int N, int Ltau, const double* __restrict__ x, double omega0, double dtau,
              double* __restrict__ part) {
  __shared__ double sh[4];
  const long d = (long)N * Ltau;
  const double w2 = omega0 * omega0, idt = 1.0 / dtau;
  double a = 0.0, b = 0.0;
  for (long k = blockIdx.x * 256L + threadIdx.x; k < d; k += (long)gridDim.x * 256) {
    const long kn = (k + N < d) ? k + N : k + N - d;
    const double xv = x[k];
    const double g = (x[kn] - xv) * idt;
    a += w2 * xv * xv + g * g;
    b += xv;
  }
  a = block_sum<256>(a, sh);
  b = block_sum<256>(b, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = a;
    part[kRedBlocks + blockIdx.x] = b;
  }
}

// part[b]: block partial sums of a . b over n values.  Launch: grid kRedBlocks, block 256.
__global__ void __launch_bounds__(256)
k_dot_part(long n, const double* __restrict__ a, const double* __restrict__ b, double* __restrict__ part) {
  __shared__ double sh[4];
  double s = 0.0;
  for (long k = blockIdx.x * 256L + threadIdx.x; k < n; k += (long)gridDim.x * 256) s += a[k] * b[k];
  s = block_sum<256>(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// out[c] = scale[c] * sum_b part[c][b] for c < blockIdx count, in block order.
// Launch: grid ncol, block 256.
__global__ void __launch_bounds__(256)
k_sum_cols(const double* __restrict__ part, double s0, double s1, double* __restrict__ out0,
           double* __restrict__ out1) {
  __shared__ double sh[4];
  const int c = blockIdx.x;
  double v = 0.0;
  for (int b = threadIdx.x; b < kRedBlocks; b += 256) v += part[c * kRedBlocks + b];
  v = block_sum<256>(v, sh);
  if (threadIdx.x == 0) {
    if (c == 0) *out0 = s0 * v;
    else *out1 = s1 * v;
  }
}

// grad += scale * (dtau (omega0^2 x - (x_{tau+1} - 2 x_tau + x_{tau-1})/dtau^2) - dtau alpha),
// periodic in tau (Eq. dSB_dx plus the linear term).
__global__ void __launch_bounds__(256)
k_sb_force(int N, int Ltau, const double* __restrict__ x, double omega0, double dtau, double alpha,
           double scale, double* __restrict__ grad) {
  const long d = (long)N * Ltau;
  const double w2 = omega0 * omega0, idt2 = 1.0 / (dtau * dtau);
  for (long k = blockIdx.x * 256L + threadIdx.x; k < d; k += (long)gridDim.x * 256) {
    const long kn = (k + N < d) ? k + N : k + N - d;
    const long kp = (k >= N) ? k - N : k - N + d;
    const double xv = x[k];
    const double f = dtau * (w2 * xv - (x[kn] - 2.0 * xv + x[kp]) * idt2) - dtau * alpha;
    grad[k] += scale * f;
  }
}

// g = 2 u - u_old; u_old = u; u = g  (linear extrapolation of the solution).
__global__ void __launch_bounds__(256)
k_extrapolate(long n, double* __restrict__ u, double* __restrict__ uold) {
  for (long k = blockIdx.x * 256L + threadIdx.x; k < n; k += (long)gridDim.x * 256) {
    const double a = u[k];
    const double g = 2.0 * a - uold[k];
    uold[k] = a;
    u[k] = g;
  }
}

// The Lambda of Eq. (Lambda_def) and its relatives, site by site, one
// time-slice shift each: out[tau] = s(ts) exp(e a x[ts] / 2) in[tau + dsh],
// s(t) = +1 for t = 0 else -1, ts = tau + 1 if dsh = +1 else tau, a = dtau alpha:
//   Lambda:      dsh = +1, e = +1      Lambda^{-1}:  dsh = -1, e = -1
//   Lambda^T:    dsh = -1, e = +1      Lambda^{-T}:  dsh = +1, e = -1
// (slices mod Ltau).  Vector v uses field x + (v / vpx) d (vpx = vectors per
// field; 0: one field for all).  Launch: grid (blocks, nvec), block 256.
__global__ void __launch_bounds__(256)
k_lambda(int N, int Ltau, long d, const double* __restrict__ x, int vpx, double a, int dsh, double e,
         const double* __restrict__ in, double* __restrict__ out) {
  const double* iv = in + (long)blockIdx.y * d;
  double* ov = out + (long)blockIdx.y * d;
  if (vpx > 0) x += (long)(blockIdx.y / vpx) * d;
  for (long k = blockIdx.x * 256L + threadIdx.x; k < d; k += (long)gridDim.x * 256) {
    const int tau = (int)(k / N);
    const int i = (int)(k - (long)tau * N);
    int src = tau + dsh;
    src = src < 0 ? src + Ltau : (src >= Ltau ? src - Ltau : src);
    const int ts = dsh > 0 ? src : tau;
    const double sg = ts == 0 ? 1.0 : -1.0;
    ov[k] = sg * exp(0.5 * e * a * x[(long)ts * N + i]) * iv[(long)src * N + i];
  }
}

// grad[tau][i] += coef * sum_r b_r[tau-1][i] u_r[tau-1][i] (slice tau-1 mod Ltau): the
// Lambda term of the force, coef = -dtau alpha times the caller's scale.
// Block row y sums right-hand sides y*nrhs .. y*nrhs + nrhs - 1 into grad + y d
// (one row per field).  Launch: grid (blocks, fields), block 256.
__global__ void __launch_bounds__(256)
k_lambda_force(int N, int Ltau, long d, int nrhs, const double* __restrict__ b,
               const double* __restrict__ u, double coef, double* __restrict__ grad) {
  b += (long)blockIdx.y * nrhs * d;
  u += (long)blockIdx.y * nrhs * d;
  grad += (long)blockIdx.y * d;
  for (long k = blockIdx.x * 256L + threadIdx.x; k < d; k += (long)gridDim.x * 256) {
    const long km = (k >= N) ? k - N : k - N + d;
    double acc = 0.0;
    for (int r = 0; r < nrhs; ++r) acc += b[(long)r * d + km] * u[(long)r * d + km];
    grad[k] += coef * acc;
  }
}

// Global moves on column i (and j) of x[Ltau][N]: kind 0 reflects x_i, kind 1 swaps x_i, x_j.
__global__ void __launch_bounds__(256)
k_global_move(int N, int Ltau, int kind, int i, int j, double* __restrict__ x) {
  for (int tau = blockIdx.x * 256 + threadIdx.x; tau < Ltau; tau += gridDim.x * 256) {
    double* row = x + (long)tau * N;
    if (kind == 0) {
      row[i] = -row[i];
    } else {
      const double t = row[i];
      row[i] = row[j];
      row[j] = t;
    }
  }
}

int grid_for(long n) {
  const long b = (n + 255) / 256;
  return (int)(b < 1 ? 1 : (b > 4096 ? 4096 : b));
}

bool opts_ok(const fph_pcg_opts_t& o) {
  return std::isfinite(o.tol) && o.tol > 0.0 && o.maxiter >= 1;
}

}  // namespace

struct fph_hmc_s {
  fph_handle_t h;   // the Holstein handle, or NULL with
  fph_ssh_t ssh;    // an SSH context (fph_hmc_create_ssh)
  fph_lattice_t lat;
  int max_rhs;
  int N, Ltau;
  long d;
  int ts, off;  // circulant table stride and index offset
  fph_hmc_opts_t o;
  int K;         // chains (independent systems sharing the launches)
  double* tab;   // [kNTab][ts]
  double* vals;  // [kNTab][Ltau]
  double* cst;   // [2]
  double *xi, *xa, *xb, *pa, *pb, *tmp, *Phi, *u, *uold, *bvec;
  double* part;  // [2][kRedBlocks]
  double* en;    // [K][kEn]
  double* en_host;
};

namespace {

hipError_t circ1(const fph_hmc_s* c, int k, int nvec, const double* in, double* out, hipStream_t s) {
  dim3 grid((c->N + 63) / 64, (c->Ltau + kRows - 1) / kRows, nvec);
  hipLaunchKernelGGL((k_tau_circ<1, 1>), grid, dim3(64), 0, s, c->N, c->Ltau, c->d, c->ts, c->off,
                     (const double*)(c->tab + (long)k * c->ts), (const double*)nullptr, in,
                     (const double*)nullptr, out, (double*)nullptr);
  return hipGetLastError();
}

hipError_t step_map(const fph_hmc_s* c, const double* x, const double* p, double* xo, double* po,
                    hipStream_t s, int nvec = 1) {
  dim3 grid((c->N + 63) / 64, (c->Ltau + kRows - 1) / kRows, nvec);
  hipLaunchKernelGGL((k_tau_circ<2, 2>), grid, dim3(64), 0, s, c->N, c->Ltau, c->d, c->ts, c->off,
                     (const double*)c->tab, (const double*)c->cst, x, p, xo, po);
  return hipGetLastError();
}

// en[i0] = S_B(x), en[i1] = -dtau alpha sum x
hipError_t sb_into(const fph_hmc_s* c, const double* x, double* out0, double* out1, hipStream_t s) {
  hipLaunchKernelGGL(k_sb_partials, dim3(kRedBlocks), dim3(256), 0, s, c->N, c->Ltau, x,
                     c->o.omega0, c->lat.dtau, c->part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sum_cols, dim3(2), dim3(256), 0, s, (const double*)c->part, 0.5 * c->lat.dtau,
                     -c->lat.dtau * c->lat.alpha, out0, out1);
  return hipGetLastError();
}

// *out = scale * a . b over n values
hipError_t dot_into(const fph_hmc_s* c, long n, const double* a, const double* b, double scale,
                    double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_dot_part, dim3(kRedBlocks), dim3(256), 0, s, n, a, b, c->part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sum_cols, dim3(1), dim3(256), 0, s, (const double*)c->part, scale, 0.0, out,
                     (double*)nullptr);
  return hipGetLastError();
}

// *out = p^T Mass^{-1} p / 2 (uses c->tmp)
hipError_t kinetic_into(const fph_hmc_s* c, const double* p, double* out, hipStream_t s) {
  hipError_t e = circ1(c, TAB_MINV, 1, p, c->tmp, s);
  if (e != hipSuccess) return e;
  return dot_into(c, c->d, p, c->tmp, 0.5, out, s);
}

hipError_t lambda_into(const fph_hmc_s* c, int op, int nvec, const double* x, const double* in,
                       double* out, hipStream_t s, int vpx = 0) {
  static const int dsh[4] = {+1, -1, -1, +1};
  static const double ex[4] = {+1.0, -1.0, +1.0, -1.0};
  dim3 grid(grid_for(c->d), nvec);
  hipLaunchKernelGGL(k_lambda, grid, dim3(256), 0, s, c->N, c->Ltau, c->d, x, vpx,
                     c->lat.dtau * c->lat.alpha, dsh[op], ex[op], in, out);
  return hipGetLastError();
}

// nfld fields of nrhs right-hand sides each; grad holds nfld gradients.
hipError_t lambda_force_into(const fph_hmc_s* c, int nrhs, const double* b, const double* u,
                             double* grad, double scale, hipStream_t s, int nfld = 1) {
  hipLaunchKernelGGL(k_lambda_force, dim3(grid_for(c->d), nfld), dim3(256), 0, s, c->N, c->Ltau,
                     c->d, nrhs, b, u, -c->lat.dtau * c->lat.alpha * scale, grad);
  return hipGetLastError();
}

}  // namespace

fph_handle_t fph::hmc_aux(fph_hmc_t c) { return (c && c->ssh) ? fph::ssh_precond(c->ssh) : nullptr; }

const void* fph::hmc_operator(fph_hmc_t c) {
  if (c == nullptr) return nullptr;
  return c->h ? (const void*)c->h : (const void*)c->ssh;
}

namespace {

// The operator calls of the update, on the Holstein handle or the SSH context.
int op_set_fields(const fph_hmc_s* c, int K, const double* x, void* stream) {
  if (c->ssh) return ssh_set_field(c->ssh, x, stream);
  return K == 1 ? fph_set_field(c->h, x, c->o.a1, c->o.a2, stream)
                : fph_set_fields(c->h, K, c->o.nfields, x, c->o.a1, c->o.a2, stream);
}

int op_MT(const fph_hmc_s* c, int nr, const double* in, double* out, void* stream) {
  if (c->ssh) return ssh_matvec(c->ssh, FPH_OP_MT, nr, in, out, stream);
  return fermion_matvec(c->h, FPH_OP_MT, FPH_F64, nr, in, out, stream);
}

int op_solve(const fph_hmc_s* c, int nr, const double* b, double* u, const fph_pcg_opts_t* o,
             fph_pcg_stats_t* st, void* stream) {
  if (c->ssh) return ssh_solve(c->ssh, nr, b, u, o, st, stream);
  return pcg_solve_sync(c->h, nr, b, u, o, st, stream);
}

int op_force(const fph_hmc_s* c, int nr, const double* u, double* grad, double scale, void* stream) {
  if (c->ssh) return ssh_force(c->ssh, nr, u, grad, scale, nullptr, stream);
  return fermion_force(c->h, nr, u, grad, scale, nullptr, stream);
}

}  // namespace

#define HMC_CHECK(call)                                         \
  do {                                                          \
    hipError_t e_ = (call);                                     \
    if (e_ != hipSuccess) return fph::record_hip_error(e_);     \
  } while (0)

#define HMC_CALL(call)                 \
  do {                                 \
    int rc_ = (call);                  \
    if (rc_ != FPH_OK) return rc_;     \
  } while (0)

extern "C" {

int fph_hmc_destroy(fph_hmc_t c) {
  if (c == nullptr) return FPH_E_NULL;
  (void)hipDeviceSynchronize();
  void* ptrs[] = {c->tab, c->vals, c->cst, c->xi, c->xa, c->xb, c->pa, c->pb,
                  c->tmp, c->Phi, c->u, c->uold, c->bvec, c->part, c->en};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (c->en_host) (void)hipHostFree(c->en_host);
  delete c;
  return FPH_OK;
}

// The context on a Holstein handle h or an SSH context ssh (the other NULL).
static int create_impl(fph_hmc_t* out, fph_handle_t h, fph_ssh_t ssh, fph_lattice_t lat, int32_t max_rhs,
                       const fph_hmc_opts_t* o, void* stream) {
  *out = nullptr;
  if (!(std::isfinite(o->omega0) && o->omega0 > 0.0) || !(std::isfinite(o->dt) && o->dt > 0.0) ||
      std::isnan(o->m_reg) || o->Nt < 1 || o->nt < 1 || !std::isfinite(o->a1) ||
      !std::isfinite(o->a2) || o->guess < 0 || o->guess > 2 || o->lambda_action < 0 ||
      o->lambda_action > 1 || !opts_ok(o->force_solve) || !opts_ok(o->action_solve) ||
      o->nchains < 0 || o->nchains > 64)
    return FPH_E_ARG;
  const int K = o->nchains > 0 ? o->nchains : 1;
  if (o->nfields < 1 || (long)o->nfields * K > max_rhs || K > max_rhs) return FPH_E_NRHS;
  fph_hmc_s* c = new fph_hmc_s();
  std::memset(c, 0, sizeof(*c));
  c->h = h;
  c->ssh = ssh;
  c->lat = lat;
  c->max_rhs = max_rhs;
  c->N = lat.L * lat.L;
  c->Ltau = lat.Ltau;
  c->d = (long)c->N * lat.Ltau;
  c->off = lat.Ltau + kRows;
  c->ts = 2 * c->off;
  c->o = *o;
  c->K = K;
  if (!std::isfinite(c->o.m_reg)) c->o.m_reg = -1.0;
  const long d = c->d * K;  // per-chain vectors, chain-major
  const int nf = o->nfields;
  hipError_t e = hipSuccess;
#define ALLOC(ptr, n)                                        \
  if (e == hipSuccess) e = hipMalloc((void**)&(ptr), (size_t)(n) * sizeof(double));
  ALLOC(c->tab, (long)kNTab * c->ts);
  ALLOC(c->vals, (long)kNTab * c->Ltau);
  ALLOC(c->cst, 2);
  ALLOC(c->xi, d);
  ALLOC(c->xa, d);
  ALLOC(c->xb, d);
  ALLOC(c->pa, d);
  ALLOC(c->pb, d);
  ALLOC(c->tmp, d);
  ALLOC(c->Phi, nf * d);
  ALLOC(c->u, nf * d);
  if (o->guess == 2) ALLOC(c->uold, nf * d);
  ALLOC(c->bvec, nf * d);
  ALLOC(c->part, 2 * kRedBlocks);
  ALLOC(c->en, (long)kEn * K);
#undef ALLOC
  if (e == hipSuccess)
    e = hipHostMalloc((void**)&c->en_host, (size_t)kEn * K * sizeof(double), hipHostMallocDefault);
  hipStream_t s = (hipStream_t)stream;
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_hmc_modes, dim3((c->Ltau + 63) / 64), dim3(64), 0, s, c->Ltau, lat.dtau,
                       c->o.omega0, c->o.m_reg, c->o.dt / c->o.nt, c->o.nt,
                       c->o.lambda_action ? 0.0 : lat.dtau * lat.alpha, c->vals, c->cst);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_hmc_tables, dim3((c->ts + 63) / 64, kNTab), dim3(64), 0, s, c->Ltau, c->ts,
                       c->off, (const double*)c->vals, c->tab);
    e = hipGetLastError();
  }
  if (e != hipSuccess) {
    fph_hmc_destroy(c);
    return fph::record_hip_error(e);
  }
  *out = c;
  return FPH_OK;
}

int fph_hmc_create(fph_hmc_t* out, fph_handle_t h, const fph_hmc_opts_t* o, void* stream) {
  if (out == nullptr || h == nullptr || o == nullptr) return FPH_E_NULL;
  *out = nullptr;
  fph_lattice_t lat;
  int32_t max_rhs = 0;
  HMC_CALL(fph_get_lattice(h, &lat, &max_rhs));
  return create_impl(out, h, nullptr, lat, max_rhs, o, stream);
}

int fph_hmc_create_ssh(fph_hmc_t* out, fph_ssh_t ssh, const fph_hmc_opts_t* o, void* stream) {
  if (out == nullptr || ssh == nullptr || o == nullptr) return FPH_E_NULL;
  *out = nullptr;
  fph_lattice_t lat;
  int32_t max_rhs = 0;
  HMC_CALL(fph::ssh_info(ssh, &lat, &max_rhs, nullptr));
  if (o->lambda_action != 0 || o->nchains > 1) return FPH_E_ARG;
  auto ssh_prec = [](int32_t p) { return p == FPH_F64 || p == FPH_F32_REFINED; };
  if (!ssh_prec(o->force_solve.prec) || !ssh_prec(o->action_solve.prec)) return FPH_E_PREC;
  return create_impl(out, nullptr, ssh, lat, max_rhs, o, stream);
}

int bosonic_action(fph_hmc_t c, const double* x_dev, double* out_dev, void* stream) {
  if (c == nullptr || x_dev == nullptr || out_dev == nullptr) return FPH_E_NULL;
  HMC_CHECK(sb_into(c, x_dev, out_dev, out_dev + 1, (hipStream_t)stream));
  return FPH_OK;
}

int bosonic_force(fph_hmc_t c, const double* x_dev, double* grad_dev, double scale, void* stream) {
  if (c == nullptr || x_dev == nullptr || grad_dev == nullptr) return FPH_E_NULL;
  if (!std::isfinite(scale)) return FPH_E_ARG;
  hipLaunchKernelGGL(k_sb_force, dim3(grid_for(c->d)), dim3(256), 0, (hipStream_t)stream, c->N,
                     c->Ltau, x_dev, c->o.omega0, c->lat.dtau,
                     c->o.lambda_action ? 0.0 : c->lat.alpha, scale, grad_dev);
  HMC_CHECK(hipGetLastError());
  return FPH_OK;
}

int hmc_mass_apply(fph_hmc_t c, int32_t op, int32_t nvec, const double* in_dev, double* out_dev,
                   void* stream) {
  if (c == nullptr || in_dev == nullptr || out_dev == nullptr) return FPH_E_NULL;
  if (op < FPH_MASS_INV || op > FPH_MASS) return FPH_E_PREC;
  if (nvec < 1 || nvec > 65535) return FPH_E_ARG;
  const long bytes = (long)nvec * c->d * 8;
  const char *a = (const char*)in_dev, *b = (const char*)out_dev;
  if (a < b + bytes && b < a + bytes) return FPH_E_ARG;
  const int k = (op == FPH_MASS_INV) ? TAB_MINV : (op == FPH_MASS_SQRT) ? TAB_MSQRT : TAB_MASS;
  HMC_CHECK(circ1(c, k, nvec, in_dev, out_dev, (hipStream_t)stream));
  return FPH_OK;
}

int hmc_boson_steps(fph_hmc_t c, double* x_dev, double* p_dev, void* stream) {
  if (c == nullptr || x_dev == nullptr || p_dev == nullptr) return FPH_E_NULL;
  hipStream_t s = (hipStream_t)stream;
  HMC_CHECK(step_map(c, x_dev, p_dev, c->xb, c->pb, s));
  HMC_CHECK(hipMemcpyAsync(x_dev, c->xb, c->d * 8, hipMemcpyDeviceToDevice, s));
  HMC_CHECK(hipMemcpyAsync(p_dev, c->pb, c->d * 8, hipMemcpyDeviceToDevice, s));
  return FPH_OK;
}

}  // extern "C"

namespace {

// Algorithm 1 for the context's K chains at once: chain k's field is
// x_dev + k d, its pseudofermions are right-hand sides k nf .. k nf + nf - 1
// of every solve (per-right-hand-side fields when K > 1), its momentum
// p + k d; energies and the Metropolis test are per chain.
int traj_impl(fph_hmc_s* c, double* x_dev, const double* R_fields_dev, const double* R_mom_dev,
              const double* r_uniform, double* p_out_dev, fph_hmc_stats_t* st, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  const fph_hmc_opts_t& o = c->o;
  const int K = c->K;
  const long d = c->d;
  const int nf = o.nfields;
  const int NR = nf * K;
  const bool lam = o.lambda_action != 0;
  std::vector<fph_hmc_stats_t> S(K);
  for (auto& v : S) std::memset(&v, 0, sizeof(v));
  std::vector<fph_pcg_stats_t> ps(NR);
  int nsolves = 0;

  auto set_fields = [&](const double* x) -> int {
    return op_set_fields(c, K, x, stream);
  };
  const double* rhs = lam ? c->bvec : c->Phi;  // b = Lambda(x)^{-T} Phi, or Phi
  auto solve = [&](const fph_pcg_opts_t& so, int zero_guess) -> int {
    fph_pcg_opts_t oo = so;
    oo.zero_guess = zero_guess;
    int rc = op_solve(c, NR, rhs, c->u, &oo, ps.data(), stream);
    if (rc != FPH_OK) return rc;
    ++nsolves;
    for (int r = 0; r < NR; ++r) {
      fph_hmc_stats_t& v = S[r / nf];
      v.status |= ps[r].status;
      v.cg_iters += ps[r].iters;
      v.matvecs += ps[r].matvecs;
    }
    return FPH_OK;
  };
  // The fermion force at the current fields c->xa into p (scale per field
  // times 1/2: S_F = 1/2 sum_sigma b_sigma . u_sigma).
  auto kick = [&](double scale, int zero_guess) -> int {
    if (lam) {
      hipError_t e = lambda_into(c, 3, NR, c->xa, c->Phi, c->bvec, s, nf);
      if (e != hipSuccess) return fph::record_hip_error(e);
    }
    int rc = solve(o.force_solve, zero_guess);
    if (rc != FPH_OK) return rc;
    rc = op_force(c, NR, c->u, c->pa, 0.5 * scale, stream);
    if (rc != FPH_OK || !lam) return rc;
    hipError_t e = lambda_force_into(c, nf, c->bvec, c->u, c->pa, 0.5 * scale, s, K);
    return e == hipSuccess ? FPH_OK : fph::record_hip_error(e);
  };
  auto energies = [&](int sb_slot, int lin_slot, int k_slot) -> hipError_t {
    hipError_t e = circ1(c, TAB_MINV, K, c->pa, c->tmp, s);
    for (int k = 0; k < K && e == hipSuccess; ++k) {
      double* en = c->en + (long)k * kEn;
      e = sb_into(c, c->xa + k * d, en + sb_slot, en + lin_slot, s);
      if (e == hipSuccess) e = dot_into(c, d, c->pa + k * d, c->tmp + k * d, 0.5, en + k_slot, s);
    }
    return e;
  };

  // Initial state: x_i, Phi_sigma = A(x_i)^T R_sigma, p = sqrt(Mass) R.
  HMC_CHECK(hipMemcpyAsync(c->xi, x_dev, K * d * 8, hipMemcpyDeviceToDevice, s));
  HMC_CHECK(hipMemcpyAsync(c->xa, x_dev, K * d * 8, hipMemcpyDeviceToDevice, s));
  HMC_CALL(set_fields(c->xa));
  if (lam) {
    HMC_CALL(op_MT(c, NR, R_fields_dev, c->bvec, stream));
    HMC_CHECK(lambda_into(c, 2, NR, c->xa, c->bvec, c->Phi, s, nf));
  } else {
    HMC_CALL(op_MT(c, NR, R_fields_dev, c->Phi, stream));
  }
  HMC_CHECK(circ1(c, TAB_MSQRT, K, R_mom_dev, c->pa, s));
  for (int k = 0; k < K; ++k)
    HMC_CHECK(dot_into(c, (long)nf * d, R_fields_dev + (long)k * nf * d, R_fields_dev + (long)k * nf * d,
                       0.5, c->en + (long)k * kEn + EN_R2, s));
  HMC_CHECK(energies(EN_SB_I, EN_LIN_I, EN_K_I));

  // Leapfrog with time-step splitting; the two half kicks between steps
  // share one force evaluation (same x) and are applied as one kick of dt.
  HMC_CHECK(hipMemsetAsync(c->u, 0, (size_t)NR * d * 8, s));
  HMC_CALL(kick(-0.5 * o.dt, 1));
  for (int t = 0; t < o.Nt; ++t) {
    HMC_CHECK(step_map(c, c->xa, c->pa, c->xb, c->pb, s, K));
    std::swap(c->xa, c->xb);
    std::swap(c->pa, c->pb);
    HMC_CALL(set_fields(c->xa));
    if (o.guess == 2) {
      if (t == 0) {
        HMC_CHECK(hipMemcpyAsync(c->uold, c->u, (size_t)NR * d * 8, hipMemcpyDeviceToDevice, s));
      } else {
        hipLaunchKernelGGL(k_extrapolate, dim3(grid_for((long)NR * d)), dim3(256), 0, s,
                           (long)NR * d, c->u, c->uold);
        HMC_CHECK(hipGetLastError());
      }
    }
    HMC_CALL(kick((t + 1 < o.Nt ? -1.0 : -0.5) * o.dt, o.guess == 0 ? 1 : 0));
  }
  std::vector<int> force_status(K);
  for (int k = 0; k < K; ++k) force_status[k] = S[k].status;

  // Final energies; S_F(x_f) from a tight solve started at the last solution
  // (b of x_f is already in place).
  HMC_CALL(solve(o.action_solve, 0));
  std::vector<double> sf_f(K, 0.0);
  std::vector<int> action_ok(K, 1);
  for (int r = 0; r < NR; ++r) {
    sf_f[r / nf] += 0.5 * ps[r].action;
    if (!(ps[r].status & FPH_ST_CONVERGED)) action_ok[r / nf] = 0;
  }
  HMC_CHECK(energies(EN_SB_F, EN_LIN_F, EN_K_F));
  HMC_CHECK(hipMemcpyAsync(c->en_host, c->en, (size_t)kEn * K * 8, hipMemcpyDeviceToHost, s));
  HMC_CHECK(hipStreamSynchronize(s));
  bool any_rejected = false;
  for (int k = 0; k < K; ++k) {
    const double* en = c->en_host + (long)k * kEn;
    fph_hmc_stats_t& v = S[k];
    v.solves = nsolves;
    v.SB_i = en[EN_SB_I] + (lam ? 0.0 : en[EN_LIN_I]);
    v.SB_f = en[EN_SB_F] + (lam ? 0.0 : en[EN_LIN_F]);
    v.SF_i = en[EN_R2];
    v.SF_f = sf_f[k];
    v.K_i = en[EN_K_I];
    v.K_f = en[EN_K_F];
    v.H_i = v.SB_i + v.SF_i + v.K_i;
    v.H_f = v.SB_f + v.SF_f + v.K_f;
    const double dH = v.H_f - v.H_i;
    const bool bad = !std::isfinite(dH) ||
                     ((v.status | force_status[k]) & (FPH_ST_BREAKDOWN | FPH_ST_NONFINITE)) || !action_ok[k];
    v.accept_prob = bad ? 0.0 : (dH <= 0.0 ? 1.0 : std::exp(-dH));
    v.accepted = (!bad && r_uniform[k] < v.accept_prob) ? 1 : 0;
    if (v.accepted)
      HMC_CHECK(hipMemcpyAsync(x_dev + k * d, c->xa + k * d, d * 8, hipMemcpyDeviceToDevice, s));
    else
      any_rejected = true;
  }
  if (p_out_dev) HMC_CHECK(hipMemcpyAsync(p_out_dev, c->pa, K * d * 8, hipMemcpyDeviceToDevice, s));
  if (any_rejected) HMC_CALL(set_fields(x_dev));
  HMC_CHECK(hipStreamSynchronize(s));
  if (st)
    for (int k = 0; k < K; ++k) st[k] = S[k];
  return FPH_OK;
}

}  // namespace

extern "C" {

int hmc_trajectory(fph_hmc_t c, double* x_dev, const double* R_fields_dev, const double* R_mom_dev,
                   double r_uniform, double* p_out_dev, fph_hmc_stats_t* st, void* stream) {
  if (c == nullptr || x_dev == nullptr || R_fields_dev == nullptr || R_mom_dev == nullptr)
    return FPH_E_NULL;
  if (!(r_uniform >= 0.0 && r_uniform <= 1.0) || c->K != 1) return FPH_E_ARG;
  return traj_impl(c, x_dev, R_fields_dev, R_mom_dev, &r_uniform, p_out_dev, st, stream);
}

int hmc_trajectories(fph_hmc_t c, double* x_dev, const double* R_fields_dev, const double* R_mom_dev,
                     const double* r_uniform_host, double* p_out_dev, fph_hmc_stats_t* stats_host,
                     void* stream) {
  if (c == nullptr || x_dev == nullptr || R_fields_dev == nullptr || R_mom_dev == nullptr ||
      r_uniform_host == nullptr)
    return FPH_E_NULL;
  for (int k = 0; k < c->K; ++k)
    if (!(r_uniform_host[k] >= 0.0 && r_uniform_host[k] <= 1.0)) return FPH_E_ARG;
  return traj_impl(c, x_dev, R_fields_dev, R_mom_dev, r_uniform_host, p_out_dev, stats_host, stream);
}

int lambda_apply(fph_hmc_t c, int32_t op, const double* x_dev, int32_t nvec, const double* in_dev,
                 double* out_dev, void* stream) {
  if (c == nullptr || x_dev == nullptr || in_dev == nullptr || out_dev == nullptr) return FPH_E_NULL;
  if (op < FPH_LAMBDA || op > FPH_LAMBDA_INV_T) return FPH_E_PREC;
  if (nvec < 1 || nvec > 65535) return FPH_E_ARG;
  const long bytes = (long)nvec * c->d * 8;
  const char *a = (const char*)in_dev, *b = (const char*)out_dev;
  if (a < b + bytes && b < a + bytes) return FPH_E_ARG;
  HMC_CHECK(lambda_into(c, op, nvec, x_dev, in_dev, out_dev, (hipStream_t)stream));
  return FPH_OK;
}

int lambda_force(fph_hmc_t c, int32_t nrhs, const double* b_dev, const double* u_dev,
                 double* grad_dev, double scale, void* stream) {
  if (c == nullptr || b_dev == nullptr || u_dev == nullptr || grad_dev == nullptr) return FPH_E_NULL;
  if (nrhs < 1) return FPH_E_NRHS;
  if (!std::isfinite(scale)) return FPH_E_ARG;
  HMC_CHECK(lambda_force_into(c, nrhs, b_dev, u_dev, grad_dev, scale, (hipStream_t)stream));
  return FPH_OK;
}

int hmc_global_update(fph_hmc_t c, int32_t kind, int32_t i, int32_t j, double* x_dev,
                      const double* R_fields_dev, double r_uniform, fph_update_stats_t* st,
                      void* stream) {
  if (c == nullptr || x_dev == nullptr || R_fields_dev == nullptr) return FPH_E_NULL;
  if (c->K != 1 || (kind != FPH_MOVE_REFLECT && kind != FPH_MOVE_SWAP) || i < 0 || i >= c->N ||
      (kind == FPH_MOVE_SWAP && (j < 0 || j >= c->N || j == i)) ||
      !(r_uniform >= 0.0 && r_uniform <= 1.0))
    return FPH_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  const fph_hmc_opts_t& o = c->o;
  const long d = c->d;
  const int nf = o.nfields;
  const bool lam = o.lambda_action != 0;
  fph_update_stats_t S;
  std::memset(&S, 0, sizeof(S));
  fph_pcg_stats_t ps[64];
  if (nf > 64) return FPH_E_NRHS;

  // Phi = A(x)^T R at the current field, S_F(x) = 1/2 |R|^2, the x-only action.
  HMC_CALL(op_set_fields(c, 1, x_dev, stream));
  if (lam) {
    HMC_CALL(op_MT(c, nf, R_fields_dev, c->bvec, stream));
    HMC_CHECK(lambda_into(c, 2, nf, x_dev, c->bvec, c->Phi, s));
  } else {
    HMC_CALL(op_MT(c, nf, R_fields_dev, c->Phi, stream));
  }
  HMC_CHECK(dot_into(c, (long)nf * d, R_fields_dev, R_fields_dev, 0.5, c->en + EN_R2, s));
  HMC_CHECK(sb_into(c, x_dev, c->en + EN_SB_I, c->en + EN_LIN_I, s));
  // Proposal x' in c->xa; its x-only action; S_F(x') from a solve to the action tolerance.
  HMC_CHECK(hipMemcpyAsync(c->xa, x_dev, d * 8, hipMemcpyDeviceToDevice, s));
  hipLaunchKernelGGL(k_global_move, dim3((c->Ltau + 255) / 256), dim3(256), 0, s, c->N, c->Ltau,
                     (int)kind, (int)i, (int)j, c->xa);
  HMC_CHECK(hipGetLastError());
  HMC_CHECK(sb_into(c, c->xa, c->en + EN_SB_F, c->en + EN_LIN_F, s));
  HMC_CALL(op_set_fields(c, 1, c->xa, stream));
  const double* rhs = c->Phi;
  if (lam) {
    HMC_CHECK(lambda_into(c, 3, nf, c->xa, c->Phi, c->bvec, s));
    rhs = c->bvec;
  }
  fph_pcg_opts_t oo = o.action_solve;
  oo.zero_guess = 1;
  HMC_CALL(op_solve(c, nf, rhs, c->u, &oo, ps, stream));
  bool ok = true;
  double sf_new = 0.0;
  for (int r = 0; r < nf; ++r) {
    S.status |= ps[r].status;
    S.cg_iters += ps[r].iters;
    ok = ok && (ps[r].status & FPH_ST_CONVERGED);
    sf_new += 0.5 * ps[r].action;
  }
  HMC_CHECK(hipMemcpyAsync(c->en_host, c->en, kEn * 8, hipMemcpyDeviceToHost, s));
  HMC_CHECK(hipStreamSynchronize(s));
  const double* en = c->en_host;
  S.dS_B = (en[EN_SB_F] - en[EN_SB_I]) + (lam ? 0.0 : en[EN_LIN_F] - en[EN_LIN_I]);
  S.SF_old = en[EN_R2];
  S.SF_new = sf_new;
  S.dS = S.dS_B + S.SF_new - S.SF_old;
  const bool bad = !ok || !std::isfinite(S.dS);
  S.accept_prob = bad ? 0.0 : (S.dS <= 0.0 ? 1.0 : std::exp(-S.dS));
  S.accepted = (!bad && r_uniform < S.accept_prob) ? 1 : 0;
  if (S.accepted) {
    HMC_CHECK(hipMemcpyAsync(x_dev, c->xa, d * 8, hipMemcpyDeviceToDevice, s));
  } else {
    HMC_CALL(op_set_fields(c, 1, x_dev, stream));
  }
  HMC_CHECK(hipStreamSynchronize(s));
  if (st) *st = S;
  return FPH_OK;
}

}  // extern "C"
