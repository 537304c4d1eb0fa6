// Setup, vector and CG-update kernels.
//
// Reductions never synchronise blocks: each block writes one partial sum
// and the next state-aware kernel folds them (see state_begin).  All dot
// products accumulate in FP64.  Elementwise kernels move 4 elements per
// thread per step (N = L^2 with even L is a multiple of 4).
#pragma once

#include "fph_common.h"

namespace fph {

// ------------------------------------------------------ 4-wide accessors

template <typename T> struct Vec4;
template <> struct Vec4<float> {
  using V = float4;
  static FPH_DEVINL V ld(const float* p) { return *reinterpret_cast<const float4*>(p); }
  static FPH_DEVINL void st(float* p, V v) { *reinterpret_cast<float4*>(p) = v; }
};
template <> struct Vec4<double> {
  struct V { double x, y, z, w; };
  static FPH_DEVINL V ld(const double* p) {
    const double2 a = *reinterpret_cast<const double2*>(p);
    const double2 b = *reinterpret_cast<const double2*>(p + 2);
    return V{a.x, a.y, b.x, b.y};
  }
  static FPH_DEVINL void st(double* p, V v) {
    *reinterpret_cast<double2*>(p) = make_double2(v.x, v.y);
    *reinterpret_cast<double2*>(p + 2) = make_double2(v.z, v.w);
  }
};

// ------------------------------------------------------------- set field

// E = exp(-dtau (alpha x - mu)) (Eq. B_def) times c4 = cosh(dtau t)^4, the
// factor the operator kernels take out of the checkerboard, in FP64 and its
// FP32 rounding.
__global__ void k_set_field(long n, const double* __restrict__ x, double dtau,
                            double alpha, double mu, double c4, double* __restrict__ E64,
                            float* __restrict__ E32) {
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n;
       k += (long)gridDim.x * blockDim.x) {
    const double e = c4 * exp(-dtau * (alpha * x[k] - mu));
    E64[k] = e;
    E32[k] = (float)e;
  }
}

// dbar_i = (1/Ltau) sum_tau E[tau][i] (Eq. expnVbar) from the stored c4 E.
// Block (64, 16): 64 sites, 16 interleaved groups of time slices, whose sums
// are added in group order.  Launch: grid (ceil(N/64), fields); field y
// reads E64 + y N Ltau and writes dbar + y N.
__global__ void __launch_bounds__(1024)
k_dbar(int N, int Ltau, const double* __restrict__ E64, double c4, double* __restrict__ dbar64,
       float* __restrict__ dbar32) {
  __shared__ double part[16][64];
  E64 += (long)blockIdx.y * N * Ltau;
  dbar64 += (long)blockIdx.y * N;
  dbar32 += (long)blockIdx.y * N;
  const int i = blockIdx.x * 64 + threadIdx.x;
  double s = 0.0;
  if (i < N)
    for (int tau = threadIdx.y; tau < Ltau; tau += 16) s += E64[(long)tau * N + i];
  part[threadIdx.y][threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.y != 0 || i >= N) return;
  double t = 0.0;
  for (int g = 0; g < 16; ++g) t += part[g][threadIdx.x];
  t /= (double)Ltau * c4;
  dbar64[i] = t;
  dbar32[i] = (float)t;
}

// ------------------------------------------------------- CG update ------

// CG update without preconditioner: alpha = rz / pAp (from the pending
// P_PAP partials), u += alpha p, r -= alpha Ap, and |r|^2 as P_RR partials.
// The direction written by this iteration's operator kernel is pb when the
// iteration count is even, pa when odd (see InPUpdate).  After an FP64
// residual evaluation (the pending partials were P_RES) the kernel only
// folds the decision.  FP32-refined: u is the FP32 correction, read as zero
// while the state says it is zero.  Launch: grid (nblk, nrhs), 256 threads.
template <typename T>
__global__ void __launch_bounds__(256)
k_cg_update(long d, T* __restrict__ u, const T* pa, const T* pb, T* __restrict__ r,
            const T* __restrict__ Ap, StIO io) {
  __shared__ double red_sh[4];
  __shared__ RhsState s_sh;
  const int rh = blockIdx.y;
  const long off = (long)rh * d;
  // The thread's first four elements are loaded (with both direction
  // buffers) while the state is read.
  const long k0 = 4 * (blockIdx.x * 256L + threadIdx.x);
  using V = typename Vec4<T>::V;
  V u0{}, r0{}, pa0{}, pb0{}, a0{};
  if (k0 < d) {
    u0 = Vec4<T>::ld(u + off + k0);
    r0 = Vec4<T>::ld(r + off + k0);
    pa0 = Vec4<T>::ld(pa + off + k0);
    pb0 = Vec4<T>::ld(pb + off + k0);
    a0 = Vec4<T>::ld(Ap + off + k0);
  }
  state_begin<256>(io, rh, &s_sh, red_sh);
  if (s_sh.done || s_sh.folded != P_PAP) {
    state_end(io, rh, &s_sh, P_NONE, 0.0, blockIdx.x, gridDim.x, blockIdx.x == 0);
    return;
  }
  const bool odd = (s_sh.iter & 1) != 0;
  const bool uz = s_sh.u32z != 0;
  const T* __restrict__ p = odd ? pa : pb;
  const T a = (T)s_sh.alpha;
  double acc = 0.0;
  for (long k = k0; k < d; k += 4L * gridDim.x * 256) {
    const long o = off + k;
    V uu, rr, pp, aa;
    if (k == k0) {
      uu = u0;
      rr = r0;
      pp = odd ? pa0 : pb0;
      aa = a0;
    } else {
      uu = Vec4<T>::ld(u + o);
      rr = Vec4<T>::ld(r + o);
      pp = Vec4<T>::ld(p + o);
      aa = Vec4<T>::ld(Ap + o);
    }
    if (uz) uu = V{};
    uu.x += a * pp.x; uu.y += a * pp.y; uu.z += a * pp.z; uu.w += a * pp.w;
    rr.x -= a * aa.x; rr.y -= a * aa.y; rr.z -= a * aa.z; rr.w -= a * aa.w;
    Vec4<T>::st(u + o, uu);
    Vec4<T>::st(r + o, rr);
    acc += (double)rr.x * (double)rr.x + (double)rr.y * (double)rr.y +
           (double)rr.z * (double)rr.z + (double)rr.w * (double)rr.w;
  }
  const double bs = block_sum<256, true>(acc, red_sh);
  if (threadIdx.x == 0) s_sh.u32z = 0;
  state_end(io, rh, &s_sh, P_RR, bs, blockIdx.x, gridDim.x, blockIdx.x == 0);
}

// ------------------------------------------------------------ plain BLAS

// part[r * stride + block] = partial sums of a_r . b_r (FP64).  Launch:
// grid (nblk, nrhs), nblk <= stride.
__global__ void __launch_bounds__(256)
k_dot_partials(long d, const double* __restrict__ a, const double* __restrict__ b,
               double* __restrict__ part, long stride) {
  __shared__ double red_sh[4];
  const int r = blockIdx.y;
  const double* ar = a + (long)r * d;
  const double* br = b + (long)r * d;
  double acc = 0.0;
  for (long k = 4 * (blockIdx.x * 256L + threadIdx.x); k < d; k += 4L * gridDim.x * 256) {
    const auto x = Vec4<double>::ld(ar + k);
    const auto y = Vec4<double>::ld(br + k);
    acc += x.x * y.x + x.y * y.y + x.z * y.z + x.w * y.w;
  }
  const double bs = block_sum<256>(acc, red_sh);
  if (threadIdx.x == 0) part[(long)r * stride + blockIdx.x] = bs;
}

// out[r] = sum of the nb partials of rhs r (at part + r * stride), in block
// order.  One block per rhs.
__global__ void __launch_bounds__(256)
k_sum_partials(int nb, const double* __restrict__ part, long stride, double* __restrict__ out) {
  __shared__ double red_sh[4];
  const int r = blockIdx.x;
  const double tot = reduce_partials<256>(part + (long)r * stride, nb, red_sh);
  if (threadIdx.x == 0) out[r] = tot;
}

// dst = (TD) src, elementwise over n values (n multiple of 4).
template <typename TS, typename TD>
__global__ void k_cast(long n, const TS* __restrict__ src, TD* __restrict__ dst) {
  for (long k = 4 * (blockIdx.x * (long)blockDim.x + threadIdx.x); k < n;
       k += 4L * gridDim.x * blockDim.x) {
    const auto x = Vec4<TS>::ld(src + k);
    typename Vec4<TD>::V y;
    y.x = (TD)x.x; y.y = (TD)x.y; y.z = (TD)x.z; y.w = (TD)x.w;
    Vec4<TD>::st(dst + k, y);
  }
}

}  // namespace fph
