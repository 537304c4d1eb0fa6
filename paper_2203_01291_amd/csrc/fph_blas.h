// Setup, vector and CG-update kernels.
//
// Every reduction is deterministic: each block writes one partial sum, the
// last block to arrive (per right-hand side) adds the partials in block
// order and updates RhsState.  All dot products accumulate in FP64.
#pragma once

#include "fph_common.h"

namespace fph {

// E = exp(-dtau (alpha x - mu)) in FP64 and its FP32 rounding (Eq. B_def).
__global__ void k_set_field(long n, const double* __restrict__ x, double dtau,
                            double alpha, double mu, double* __restrict__ E64,
                            float* __restrict__ E32) {
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n;
       k += (long)gridDim.x * blockDim.x) {
    const double e = exp(-dtau * (alpha * x[k] - mu));
    E64[k] = e;
    E32[k] = (float)e;
  }
}

// dbar_i = (1/Ltau) sum_tau E[tau][i] (Eq. expnVbar), summed in tau order.
__global__ void k_dbar(int N, int Ltau, const double* __restrict__ E64,
                       double* __restrict__ dbar64, float* __restrict__ dbar32) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double s = 0.0;
  for (int tau = 0; tau < Ltau; ++tau) s += E64[(long)tau * N + i];
  s /= (double)Ltau;
  dbar64[i] = s;
  dbar32[i] = (float)s;
}

// Zero-initialise the solver state and set bb = |b|^2 for each rhs.
// Launch: grid (nblk, nrhs), 256 threads.
template <typename T>
__global__ void __launch_bounds__(256)
k_norm2(long d, const T* __restrict__ b, double* partial, unsigned* counter,
        RhsState* st, double tol, int maxiter, int mode) {
  __shared__ double red_sh[4];
  __shared__ int flag_sh;
  const int r = blockIdx.y;
  const T* br = b + (long)r * d;
  double acc = 0.0;
  for (long k = blockIdx.x * 256L + threadIdx.x; k < d; k += (long)gridDim.x * 256) {
    const double v = (double)br[k];
    acc += v * v;
  }
  const double bs = block_sum<256>(acc, red_sh);
  if (threadIdx.x == 0) partial[(long)r * gridDim.x + blockIdx.x] = bs;
  if (last_block(counter + r, gridDim.x, &flag_sh)) {
    const double tot = reduce_partials<256>(partial + (long)r * gridDim.x, gridDim.x, red_sh);
    if (threadIdx.x == 0) {
      RhsState& s = st[r];
      if (mode == 0) {  // initialise a solve with |b|^2
        s.bb = tot;
        s.rr = tot;
        s.rz = tot;
        s.rz_prev = tot;
        s.pAp = 0.0;
        s.alpha = 0.0;
        s.beta = 0.0;
        s.rr_ref = tot;
        s.rr_true = tot;
        s.tol2 = tol * tol * tot;
        s.ru_thresh = 0.0;
        s.iter = 0;
        s.done = (tot == 0.0) ? 1 : 0;
        s.status = (tot == 0.0) ? 1 : (isfinite(tot) ? 0 : 8);
        if (!isfinite(tot)) s.done = 1;
        s.fresh = 1;
        s.matvecs = 0;
        s.maxiter = maxiter;
      } else {  // |r|^2 of a replaced residual; without preconditioner rz = rr
        s.rr = tot;
        s.rz = tot;
        s.rr_ref = tot;
        s.beta = tot / s.rz_prev;
        if (tot <= s.tol2) s.done = 1;
      }
      __threadfence();
      atomicExch(counter + r, 0u);
    }
  }
}

// out_r = sum_k a_r[k] * b_r[k] (FP64).  Launch: grid (nblk, nrhs).
__global__ void __launch_bounds__(256)
k_dot_out(long d, const double* __restrict__ a, const double* __restrict__ b,
          double* partial, unsigned* counter, double* out) {
  __shared__ double red_sh[4];
  __shared__ int flag_sh;
  const int r = blockIdx.y;
  const double* ar = a + (long)r * d;
  const double* br = b + (long)r * d;
  double acc = 0.0;
  for (long k = blockIdx.x * 256L + threadIdx.x; k < d; k += (long)gridDim.x * 256)
    acc += ar[k] * br[k];
  const double bs = block_sum<256>(acc, red_sh);
  if (threadIdx.x == 0) partial[(long)r * gridDim.x + blockIdx.x] = bs;
  if (last_block(counter + r, gridDim.x, &flag_sh)) {
    const double tot = reduce_partials<256>(partial + (long)r * gridDim.x, gridDim.x, red_sh);
    if (threadIdx.x == 0) {
      out[r] = tot;
      __threadfence();
      atomicExch(counter + r, 0u);
    }
  }
}

// dst = (TD) src, elementwise over n values.
template <typename TS, typename TD>
__global__ void k_cast(long n, const TS* __restrict__ src, TD* __restrict__ dst) {
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n;
       k += (long)gridDim.x * blockDim.x)
    dst[k] = (TD)src[k];
}

// u64 += u32 (FP64 accumulation of the FP32 correction); u32 = 0.
// Skips right-hand sides with done set.  Launch: grid (nblk, nrhs).
__global__ void k_flush(long d, float* __restrict__ u32, double* __restrict__ u64,
                        const RhsState* st) {
  const int r = blockIdx.y;
  if (st[r].done) return;
  float* a = u32 + (long)r * d;
  double* b = u64 + (long)r * d;
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < d;
       k += (long)gridDim.x * blockDim.x) {
    b[k] += (double)a[k];
    a[k] = 0.0f;
  }
}

// CG update without preconditioner: u += alpha p, r -= alpha Ap, then
// |r|^2; the last block sets rz = |r|^2, beta = rz / rz_prev and tests
// convergence (|r|^2 <= tol^2 |b|^2) and the iteration cap.
// Launch: grid (nblk, nrhs), 256 threads; d multiple of 4.
// The direction written by this iteration's operator kernel is pb when the
// iteration count is even, pa when odd (see InPUpdate).
template <typename T>
__global__ void __launch_bounds__(256)
k_cg_update(long d, T* __restrict__ u, const T* pa, const T* pb,
            T* __restrict__ r, const T* __restrict__ Ap, RhsState* st,
            double* partial, unsigned* counter) {
  __shared__ double red_sh[4];
  __shared__ int flag_sh;
  const int rh = blockIdx.y;
  if (st[rh].done) return;
  const T* __restrict__ p = (st[rh].iter & 1) ? pa : pb;
  const T a = (T)st[rh].alpha;
  const long off = (long)rh * d;
  double acc = 0.0;
  for (long k = blockIdx.x * 256L + threadIdx.x; k < d; k += (long)gridDim.x * 256) {
    const T pk = p[off + k];
    const T rk = r[off + k] - a * Ap[off + k];
    u[off + k] += a * pk;
    r[off + k] = rk;
    acc += (double)rk * (double)rk;
  }
  const double bs = block_sum<256>(acc, red_sh);
  if (threadIdx.x == 0) partial[(long)rh * gridDim.x + blockIdx.x] = bs;
  if (last_block(counter + rh, gridDim.x, &flag_sh)) {
    const double tot = reduce_partials<256>(partial + (long)rh * gridDim.x, gridDim.x, red_sh);
    if (threadIdx.x == 0) {
      RhsState& s = st[rh];
      s.rr = tot;
      s.rz_prev = s.rz;
      s.rz = tot;
      s.beta = tot / s.rz_prev;
      s.fresh = 0;
      s.iter += 1;
      if (!isfinite(tot)) {
        s.status |= 8;
        s.done = 1;
      } else if (tot <= s.tol2) {
        s.done = 1;
      } else if (s.iter >= s.maxiter) {
        s.status |= 2;
        s.done = 1;
      } else if (tot < s.ru_thresh) {
        s.done = 1;  // pause for an FP64 residual replacement
      }
      __threadfence();
      atomicExch(counter + rh, 0u);
    }
  }
}

}  // namespace fph
