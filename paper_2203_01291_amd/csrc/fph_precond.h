// Adiabatic preconditioner of Sec. V and App. C of the paper.
//
// F ~ P^{-1} = U^dagger Ptilde^{-1} U (Eq. P_change_basis), with
// U_{w,tau} = exp(-2 pi i tau (w + 1/2)/Ltau)/sqrt(Ltau) (Eq. U_omega) and
// Ptilde^{-1} block diagonal: block w is (I - e^{-i phi_w} Bbar)^{-1},
// phi_w = 2 pi (w + 1/2)/Ltau (Eq. Mww), approximated by the truncated
// Chebyshev series sum_{m < N_P(w)} c_m(w) T_m(A), A = s Bbar - c with
// s = 2/db, c = 1 + 2 bmin/db (Eqs. A_def, f_A_approx, alpha_recur).
//
// Real input, half spectrum.  For real r, (U r)_{Ltau-1-w} = conj((U r)_w)
// and the blocks obey f_{Ltau-1-w} = conj(f_w), so the even frequencies
// w = 2k (k < H = Ltau/2) carry everything:
//   Z_k = (U r)_{2k} = (1/sqrt Ltau) sum_{tau < H} W_H^{k tau}
//                      e^{-i pi tau/Ltau} (r_tau - i r_{tau+H}),
// a length-H complex DFT (W_H = e^{-2 pi i/H}).  The inverse maps the
// block outputs Zh_k back by S_tau = e^{+i pi tau/Ltau} sum_k W_H^{-k tau}
// Zh_k and out_tau = (2/sqrt Ltau) Re S_tau, out_{tau+H} = -(2/sqrt Ltau)
// Im S_tau.  The length-H DFTs use one Cooley-Tukey split H = H1 * H2.
//
// F^T = U^dagger D^H U (F is real), so the CG preconditioner
// F F^T = U^dagger (D D^H) U needs one forward and one inverse transform:
// per block, first sum conj(c_m) T_m(A^T), then sum c_m T_m(A)
// (A^T = s C^T diag(dbar) - c, C^T = P_B P_A).
#pragma once

#include <cstring>

#include "fph_common.h"

namespace fph {

constexpr int kNPMax = 1024;   // cap on the Chebyshev order N_P(w)
constexpr int kSites = 16;     // sites per transform block (one 128-byte row in FP64)

template <typename T> struct Cplx;
template <> struct Cplx<double> { using type = double2; };
template <> struct Cplx<float> { using type = float2; };

struct PcTables {
  int H, H1, H2;
  double2* tw64;   // e^{-i pi tau / Ltau}, tau < H
  double2* W64;    // e^{-2 pi i k / H}, k < H
  float2* tw32;
  float2* W32;
  PcInfo* info;    // bounds and series constants (device)
  int* np;         // N_P(w) for w < Ltau (device)
  double2* coef64; // [H][kNPMax]: c_m(2k)
  float2* coef32;
  void* Z;         // complex workspace, max_rhs * H * N (double2)
  void* Z2;
  double ch, sh;   // checkerboard rotation cosh(dtau t), sinh(dtau t)
};

inline int pick_h1(int H) {
  static const int cand[] = {20, 16, 10, 8, 5, 4, 3, 2, 1};
  for (int h1 : cand)
    if (H % h1 == 0 && H / h1 <= 32) return h1;
  return 0;
}

inline bool pc_supported(int Ltau) { return Ltau >= 2 && Ltau % 2 == 0 && pick_h1(Ltau / 2) > 0; }

// ----------------------------------------------------------- setup kernels

__global__ void k_pc_twiddles(int H, int Ltau, double2* tw64, double2* W64, float2* tw32,
                              float2* W32) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < H; k += gridDim.x * blockDim.x) {
    const double a = (double)k / (double)Ltau;      // twist angle / pi
    const double b = 2.0 * (double)k / (double)H;   // DFT angle / pi
    const double2 t = make_double2(cospi(a), -sinpi(a));
    const double2 w = make_double2(cospi(b), -sinpi(b));
    tw64[k] = t;
    W64[k] = w;
    tw32[k] = make_float2((float)t.x, (float)t.y);
    W32[k] = make_float2((float)w.x, (float)w.y);
  }
}

// Bounds of the spectrum of Bbar = diag(dbar) C and N_P(w).  One block.
//   bmin = min(dbar) e^{-4 dtau |t|}, bmax = max(dbar) e^{+4 dtau |t|}
//   N_P(w) = max(1, floor(db (a1/phi_w' + a2))), w' = min(w, Ltau-1-w)
__global__ void __launch_bounds__(256)
k_pc_bounds(int N, int Ltau, const double* __restrict__ dbar, double dtau, double t, double a1,
            double a2, PcInfo* info, int* np) {
  __shared__ double smin[256], smax[256];
  __shared__ int snp[256];
  double lo = 1e300, hi = -1e300;
  for (int i = threadIdx.x; i < N; i += 256) {
    lo = fmin(lo, dbar[i]);
    hi = fmax(hi, dbar[i]);
  }
  smin[threadIdx.x] = lo;
  smax[threadIdx.x] = hi;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + off]);
      smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + off]);
    }
    __syncthreads();
  }
  const double g = exp(4.0 * dtau * fabs(t));
  const double bmin = smin[0] / g, bmax = smax[0] * g;
  const double db = bmax - bmin;
  int mx = 1;
  for (int w = threadIdx.x; w < Ltau; w += 256) {
    const int wp = min(w, Ltau - 1 - w);
    const double phi = 2.0 * M_PI * ((double)wp + 0.5) / (double)Ltau;
    double v = floor(db * (a1 / phi + a2));
    int n = (v < 1.0) ? 1 : (v > (double)kNPMax ? kNPMax : (int)v);
    np[w] = n;
    mx = max(mx, n);
  }
  snp[threadIdx.x] = mx;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) snp[threadIdx.x] = max(snp[threadIdx.x], snp[threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    info->bmin = bmin;
    info->bmax = bmax;
    info->s = db > 0.0 ? 2.0 / db : 0.0;
    info->c = db > 0.0 ? 1.0 + 2.0 * bmin / db : 0.0;
    info->maxnp = snp[0];
  }
}

// Chebyshev-Gauss coefficients (Eq. Cheby-Gauss, N_Q = 2 N_P) of
// f_w(y) = 1/(1 - e^{-i phi_w} b(y)), b(y) = bmin + (y + 1) db/2, for the
// even frequencies w = 2k.  Grid: H blocks.
__global__ void __launch_bounds__(256)
k_pc_coef(int Ltau, const PcInfo* info, const int* np, double2* coef64, float2* coef32) {
  const int k = blockIdx.x;
  const int w = 2 * k;
  const int NP = np[w];
  const int NQ = 2 * NP;
  const double bmin = info->bmin, db = info->bmax - info->bmin;
  const double er = cospi((2.0 * w + 1.0) / (double)Ltau);    // Re e^{-i phi}
  const double ei = -sinpi((2.0 * w + 1.0) / (double)Ltau);   // Im e^{-i phi}
  for (int m = threadIdx.x; m < NP; m += 256) {
    double sr = 0.0, si = 0.0;
    for (int n = 0; n < NQ; ++n) {
      const double y = cospi((2.0 * n + 1.0) / (2.0 * NQ));
      const long arg = ((long)m * (2 * n + 1)) % (4L * NQ);
      const double cm = cospi((double)arg / (2.0 * NQ));
      const double b = bmin + (y + 1.0) * 0.5 * db;
      const double dr = 1.0 - er * b, di = -ei * b;   // 1 - e^{-i phi} b
      const double den = dr * dr + di * di;
      sr += cm * (dr / den);
      si += cm * (-di / den);
    }
    const double scale = (m == 0 ? 1.0 : 2.0) / (double)NQ;
    const double2 c = make_double2(sr * scale, si * scale);
    coef64[(long)k * kNPMax + m] = c;
    coef32[(long)k * kNPMax + m] = make_float2((float)c.x, (float)c.y);
  }
}

// ------------------------------------------------------ transform kernels

template <typename T2, typename T>
FPH_DEVINL T2 cmul(T2 a, T2 b) {
  T2 r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}

template <typename T2, typename T>
FPH_DEVINL T2 cmulc(T2 a, T2 b) {  // a * conj(b)
  T2 r;
  r.x = a.x * b.x + a.y * b.y;
  r.y = a.y * b.x - a.x * b.y;
  return r;
}

// Forward transform of KSITES sites per block: Z[r][k][i] = (U in)_{2k}.
// With CGUPD, first the CG update of the tile: u += alpha p,
// r -= alpha Ap (r is `in`, updated in place) and |r|^2, after which the
// last block sets rr, advances the iteration count and tests convergence.
// The direction is pb on even iteration counts, pa on odd (see InPUpdate).
// Launch: grid (ceil(N / kSites), nrhs), NT threads, LDS H * kSites complex.
template <typename T, int H1, int NT, bool CGUPD>
__global__ void __launch_bounds__(NT)
k_tfwd(Geom g, int H2, const typename Cplx<T>::type* __restrict__ tw,
       const typename Cplx<T>::type* __restrict__ W, T* in, typename Cplx<T>::type* __restrict__ Z,
       T* __restrict__ u, const T* pa, const T* pb, const T* __restrict__ Ap, RhsState* st,
       double* partial, unsigned* counter) {
  using T2 = typename Cplx<T>::type;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T2* Y = reinterpret_cast<T2*>(smem_raw);
  __shared__ double red_sh[NT / 64];
  __shared__ int flag_sh;
  const int r = blockIdx.y;
  if (st != nullptr && st[r].done) return;
  const int H = H1 * H2;
  const int i0 = blockIdx.x * kSites;
  const long base = (long)r * g.d;
  const T scale = (T)(1.0 / sqrt((double)g.Ltau));
  T alpha = (T)0;
  const T* __restrict__ p = pa;
  if (CGUPD) {
    alpha = (T)st[r].alpha;
    p = (st[r].iter & 1) ? pa : pb;  // direction written by this iteration
  }
  double acc_rr = 0.0;

  // Step 1: per (site, n2), H1-point DFT over n1 of the twisted input.
  for (int it = threadIdx.x; it < kSites * H2; it += NT) {
    const int s = it % kSites, n2 = it / kSites;
    if (i0 + s >= g.N) continue;
    T2 acc[H1];
#pragma unroll
    for (int k1 = 0; k1 < H1; ++k1) acc[k1] = T2{(T)0, (T)0};
#pragma unroll
    for (int n1 = 0; n1 < H1; ++n1) {
      const int tau = H2 * n1 + n2;
      const long oa = base + (long)tau * g.N + i0 + s;
      const long ob = oa + (long)H * g.N;
      T a = in[oa], b = in[ob];
      if (CGUPD) {
        a -= alpha * Ap[oa];
        b -= alpha * Ap[ob];
        in[oa] = a;
        in[ob] = b;
        u[oa] += alpha * p[oa];
        u[ob] += alpha * p[ob];
        acc_rr += (double)a * (double)a + (double)b * (double)b;
      }
      const T2 y = cmul<T2, T>(tw[tau], T2{a, -b});
#pragma unroll
      for (int k1 = 0; k1 < H1; ++k1) {
        const T2 wv = W[(H2 * n1 * k1) % H];
        acc[k1].x += wv.x * y.x - wv.y * y.y;
        acc[k1].y += wv.x * y.y + wv.y * y.x;
      }
    }
#pragma unroll
    for (int k1 = 0; k1 < H1; ++k1)
      Y[(n2 * H1 + k1) * kSites + s] = cmul<T2, T>(acc[k1], W[(n2 * k1) % H]);
  }
  __syncthreads();
  // Step 2: per (site, k1, k2), H2-point DFT over n2.
  for (int it = threadIdx.x; it < kSites * H; it += NT) {
    const int s = it % kSites;
    const int kk = it / kSites;
    const int k1 = kk % H1, k2 = kk / H1;
    if (i0 + s >= g.N) continue;
    T2 x = T2{(T)0, (T)0};
    for (int n2 = 0; n2 < H2; ++n2) {
      const T2 wv = W[(H1 * n2 * k2) % H];
      const T2 yv = Y[(n2 * H1 + k1) * kSites + s];
      x.x += wv.x * yv.x - wv.y * yv.y;
      x.y += wv.x * yv.y + wv.y * yv.x;
    }
    const int k = k1 + H1 * k2;
    Z[((long)r * H + k) * g.N + i0 + s] = T2{x.x * scale, x.y * scale};
  }

  if (CGUPD) {
    const double bs = block_sum<NT>(acc_rr, red_sh);
    if (threadIdx.x == 0) partial[(long)r * gridDim.x + blockIdx.x] = bs;
    if (last_block(counter + r, gridDim.x, &flag_sh)) {
      const double tot = reduce_partials<NT>(partial + (long)r * gridDim.x, gridDim.x, red_sh);
      if (threadIdx.x == 0) {
        RhsState& sst = st[r];
        sst.rr = tot;
        sst.rz_prev = sst.rz;  // r.z of the residual before this update
        sst.fresh = 0;
        sst.iter += 1;
        if (!isfinite(tot)) {
          sst.status |= 8;
          sst.done = 1;
        } else if (tot <= sst.tol2) {
          sst.done = 1;
        } else if (sst.iter >= sst.maxiter) {
          sst.status |= 2;
          sst.done = 1;
        } else if (tot < sst.ru_thresh) {
          sst.done = 1;  // pause for an FP64 residual replacement
        }
        __threadfence();
        atomicExch(counter + r, 0u);
      }
    }
  }
}

// Inverse transform: out[r][tau][i] from Zh[r][k][i].  With dot != 0 also
// accumulates rdot . out; the last block then sets rz = r.z and
// beta = rz / rz_prev (rz_prev holds r.z of the previous residual: the CG
// update shifts it, a residual replacement keeps it).
template <typename T, int H1, int NT>
__global__ void __launch_bounds__(NT)
k_tinv(Geom g, int H2, const typename Cplx<T>::type* __restrict__ tw,
       const typename Cplx<T>::type* __restrict__ W, const typename Cplx<T>::type* __restrict__ Zh,
       T* __restrict__ out, int dot, const T* __restrict__ rdot, RhsState* st, double* partial,
       unsigned* counter) {
  using T2 = typename Cplx<T>::type;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T2* Y = reinterpret_cast<T2*>(smem_raw);
  __shared__ double red_sh[NT / 64];
  __shared__ int flag_sh;
  const int r = blockIdx.y;
  if (st != nullptr && st[r].done) return;
  const int H = H1 * H2;
  const int i0 = blockIdx.x * kSites;
  const long base = (long)r * g.d;
  const T scale = (T)(2.0 / sqrt((double)g.Ltau));
  double acc_dot = 0.0;

  for (int it = threadIdx.x; it < kSites * H2; it += NT) {
    const int s = it % kSites, n2 = it / kSites;
    if (i0 + s >= g.N) continue;
    T2 acc[H1];
#pragma unroll
    for (int k1 = 0; k1 < H1; ++k1) acc[k1] = T2{(T)0, (T)0};
#pragma unroll
    for (int n1 = 0; n1 < H1; ++n1) {
      const int kin = H2 * n1 + n2;
      const T2 y = Zh[((long)r * H + kin) * g.N + i0 + s];
#pragma unroll
      for (int k1 = 0; k1 < H1; ++k1) {
        const T2 wv = W[(H2 * n1 * k1) % H];   // used conjugated
        acc[k1].x += wv.x * y.x + wv.y * y.y;
        acc[k1].y += wv.x * y.y - wv.y * y.x;
      }
    }
#pragma unroll
    for (int k1 = 0; k1 < H1; ++k1)
      Y[(n2 * H1 + k1) * kSites + s] = cmulc<T2, T>(acc[k1], W[(n2 * k1) % H]);
  }
  __syncthreads();
  for (int it = threadIdx.x; it < kSites * H; it += NT) {
    const int s = it % kSites;
    const int kk = it / kSites;
    const int k1 = kk % H1, k2 = kk / H1;
    if (i0 + s >= g.N) continue;
    T2 x = T2{(T)0, (T)0};
    for (int n2 = 0; n2 < H2; ++n2) {
      const T2 wv = W[(H1 * n2 * k2) % H];
      const T2 yv = Y[(n2 * H1 + k1) * kSites + s];
      x.x += wv.x * yv.x + wv.y * yv.y;
      x.y += wv.x * yv.y - wv.y * yv.x;
    }
    const int tau = k1 + H1 * k2;
    const T2 sv = cmulc<T2, T>(x, tw[tau]);
    const long oa = base + (long)tau * g.N + i0 + s;
    const long ob = oa + (long)H * g.N;
    const T va = scale * sv.x, vb = -scale * sv.y;
    out[oa] = va;
    out[ob] = vb;
    if (dot) acc_dot += (double)rdot[oa] * (double)va + (double)rdot[ob] * (double)vb;
  }

  if (dot) {
    const double bs = block_sum<NT>(acc_dot, red_sh);
    if (threadIdx.x == 0) partial[(long)r * gridDim.x + blockIdx.x] = bs;
    if (last_block(counter + r, gridDim.x, &flag_sh)) {
      const double tot = reduce_partials<NT>(partial + (long)r * gridDim.x, gridDim.x, red_sh);
      if (threadIdx.x == 0) {
        RhsState& sst = st[r];
        sst.rz = tot;
        sst.beta = tot / sst.rz_prev;
        if (!(tot > 0.0) || !isfinite(tot)) {
          sst.status |= isfinite(tot) ? 4 : 8;
          sst.done = 1;
        }
        __threadfence();
        atomicExch(counter + r, 0u);
      }
    }
  }
}

// ------------------------------------------------------------ KPM kernel

// Bbar x (TRANS = false: dbar * P_A (P_B x)) or Bbar^T x (TRANS = true:
// P_B (P_A (dbar * x))) for a complex vector held on even plaquettes.
template <typename T, int NT, int MS, bool TRANS>
FPH_DEVINL void bbar_apply(const Geom& g, int nslot, T (&xr)[MS][4], T (&xi)[MS][4],
                           const T (&db)[MS][4], T* lr, T* li, T ch, T sh) {
  // (1) even layout: TRANS -> dbar*, P_A ; write
#pragma unroll
  for (int k = 0; k < MS; ++k) {
    const int q = threadIdx.x + k * NT;
    if (k < nslot && q < g.Q) {
      if (TRANS) {
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          xr[k][m] *= db[k][m];
          xi[k][m] *= db[k][m];
        }
        plaq_rot(xr[k], ch, sh);
        plaq_rot(xi[k], ch, sh);
      }
      int s[4];
      even_sites(g, q, s);
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        lr[s[m]] = xr[k][m];
        li[s[m]] = xi[k][m];
      }
    }
  }
  __syncthreads();
  // (2) odd layout: P_B in place
#pragma unroll
  for (int k = 0; k < MS; ++k) {
    const int q = threadIdx.x + k * NT;
    if (k < nslot && q < g.Q) {
      int s[4];
      odd_sites(g, q, s);
      T tr[4], ti[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        tr[m] = lr[s[m]];
        ti[m] = li[s[m]];
      }
      plaq_rot(tr, ch, sh);
      plaq_rot(ti, ch, sh);
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        lr[s[m]] = tr[m];
        li[s[m]] = ti[m];
      }
    }
  }
  __syncthreads();
  // (3) even layout: read; !TRANS -> P_A, dbar*
#pragma unroll
  for (int k = 0; k < MS; ++k) {
    const int q = threadIdx.x + k * NT;
    if (k < nslot && q < g.Q) {
      int s[4];
      even_sites(g, q, s);
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        xr[k][m] = lr[s[m]];
        xi[k][m] = li[s[m]];
      }
      if (!TRANS) {
        plaq_rot(xr[k], ch, sh);
        plaq_rot(xi[k], ch, sh);
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          xr[k][m] *= db[k][m];
          xi[k][m] *= db[k][m];
        }
      }
    }
  }
}

// acc = sum_{m < NP} c'_m T_m(A') x with A' = A (TRANS false, c' = c) or
// A' = A^T (TRANS true, c' = conj(c)); three-term recurrence of Eq.
// alpha_recur.  x is consumed.
template <typename T, int NT, int MS, bool TRANS>
FPH_DEVINL void cheb_series(const Geom& g, int nslot, int NP, const typename Cplx<T>::type* cf,
                            T sA, T cA, T (&xr)[MS][4], T (&xi)[MS][4], const T (&db)[MS][4],
                            T* lr, T* li, T ch, T sh, T (&ar)[MS][4], T (&ai)[MS][4]) {
  const T cj = TRANS ? (T)-1 : (T)1;
  T pr[MS][4], pi_[MS][4];  // alpha_{m-1}
  {
    const auto c0 = cf[0];
#pragma unroll
    for (int k = 0; k < MS; ++k)
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        ar[k][m] = c0.x * xr[k][m] - cj * c0.y * xi[k][m];
        ai[k][m] = c0.x * xi[k][m] + cj * c0.y * xr[k][m];
        pr[k][m] = xr[k][m];
        pi_[k][m] = xi[k][m];
      }
  }
  for (int m = 1; m < NP; ++m) {
    // x <- (m == 1 ? A x : 2 A x - prev), with x = alpha_{m-1} on entry
    T cr[MS][4], ci[MS][4];
#pragma unroll
    for (int k = 0; k < MS; ++k)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        cr[k][q] = xr[k][q];
        ci[k][q] = xi[k][q];
      }
    bbar_apply<T, NT, MS, TRANS>(g, nslot, xr, xi, db, lr, li, ch, sh);
    const T two = (m == 1) ? (T)1 : (T)2;
    const auto cm = cf[m];
#pragma unroll
    for (int k = 0; k < MS; ++k)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        T nr = two * (sA * xr[k][q] - cA * cr[k][q]);
        T ni = two * (sA * xi[k][q] - cA * ci[k][q]);
        if (m > 1) {
          nr -= pr[k][q];
          ni -= pi_[k][q];
        }
        pr[k][q] = cr[k][q];
        pi_[k][q] = ci[k][q];
        xr[k][q] = nr;
        xi[k][q] = ni;
        ar[k][q] += cm.x * nr - cj * cm.y * ni;
        ai[k][q] += cm.x * ni + cj * cm.y * nr;
      }
  }
}

// Per-block Chebyshev apply.  op 0: F (series in A), 1: F^T (conjugate
// series in A^T), 2: F F^T (conjugate series, then series).  Block b
// serves frequency order b / nrhs (longest series first: k = 0, H-1, 1,
// H-2, ...) and right-hand side b % nrhs.  LDS: 2 * N * sizeof(T).
template <typename T, int NT, int MS>
__global__ void __launch_bounds__(NT)
k_kpm(Geom g, int H, int nrhs, int op, const PcInfo* __restrict__ info,
      const int* __restrict__ np, const typename Cplx<T>::type* __restrict__ coef,
      const T* __restrict__ dbar, T ch, T sh, const typename Cplx<T>::type* __restrict__ Z,
      typename Cplx<T>::type* __restrict__ Zo, const RhsState* st) {
  using T2 = typename Cplx<T>::type;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* lr = reinterpret_cast<T*>(smem_raw);
  T* li = lr + g.N;
  const int ko = blockIdx.x / nrhs;
  const int r = blockIdx.x % nrhs;
  if (st != nullptr && st[r].done) return;
  const int k = (ko % 2 == 0) ? ko / 2 : H - 1 - ko / 2;
  const int NP = np[2 * k];
  const T2* cf = coef + (long)k * kNPMax;
  const T sA = (T)info->s, cA = (T)info->c;
  const int nslot = (g.Q + NT - 1) / NT;

  T xr[MS][4], xi[MS][4], db[MS][4], ar[MS][4], ai[MS][4];
  const T2* Zin = Z + ((long)r * H + k) * g.N;
#pragma unroll
  for (int kk = 0; kk < MS; ++kk) {
    const int q = threadIdx.x + kk * NT;
    int s[4];
    if (kk < nslot && q < g.Q) {
      even_sites(g, q, s);
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const T2 v = Zin[s[m]];
        xr[kk][m] = v.x;
        xi[kk][m] = v.y;
        db[kk][m] = dbar[s[m]];
      }
    } else {
#pragma unroll
      for (int m = 0; m < 4; ++m) xr[kk][m] = xi[kk][m] = db[kk][m] = (T)0;
    }
  }
  if (op == 0) {
    cheb_series<T, NT, MS, false>(g, nslot, NP, cf, sA, cA, xr, xi, db, lr, li, ch, sh, ar, ai);
  } else {
    cheb_series<T, NT, MS, true>(g, nslot, NP, cf, sA, cA, xr, xi, db, lr, li, ch, sh, ar, ai);
    if (op == 2) {
#pragma unroll
      for (int kk = 0; kk < MS; ++kk)
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          xr[kk][m] = ar[kk][m];
          xi[kk][m] = ai[kk][m];
        }
      cheb_series<T, NT, MS, false>(g, nslot, NP, cf, sA, cA, xr, xi, db, lr, li, ch, sh, ar, ai);
    }
  }
  T2* Zout = Zo + ((long)r * H + k) * g.N;
#pragma unroll
  for (int kk = 0; kk < MS; ++kk) {
    const int q = threadIdx.x + kk * NT;
    if (kk < nslot && q < g.Q) {
      int s[4];
      even_sites(g, q, s);
#pragma unroll
      for (int m = 0; m < 4; ++m) Zout[s[m]] = T2{ar[kk][m], ai[kk][m]};
    }
  }
}

// ----------------------------------------------------------------- host

inline hipError_t pc_create(PcTables* pc, const Geom& g, int max_rhs) {
  std::memset(pc, 0, sizeof(*pc));
  pc->H = g.Ltau / 2;
  pc->H1 = pick_h1(pc->H);
  pc->H2 = pc->H1 ? pc->H / pc->H1 : 0;
  const int H = pc->H;
  hipError_t e = hipSuccess;
#define PCALLOC(ptr, bytes) \
  if (e == hipSuccess) e = hipMalloc((void**)&(ptr), (bytes));
  PCALLOC(pc->tw64, H * sizeof(double2));
  PCALLOC(pc->W64, H * sizeof(double2));
  PCALLOC(pc->tw32, H * sizeof(float2));
  PCALLOC(pc->W32, H * sizeof(float2));
  PCALLOC(pc->info, sizeof(PcInfo));
  PCALLOC(pc->np, g.Ltau * sizeof(int));
  PCALLOC(pc->coef64, (size_t)H * kNPMax * sizeof(double2));
  PCALLOC(pc->coef32, (size_t)H * kNPMax * sizeof(float2));
  PCALLOC(pc->Z, (size_t)max_rhs * H * g.N * sizeof(double2));
  PCALLOC(pc->Z2, (size_t)max_rhs * H * g.N * sizeof(double2));
#undef PCALLOC
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_pc_twiddles, dim3((H + 255) / 256), dim3(256), 0, 0, H, g.Ltau, pc->tw64,
                     pc->W64, pc->tw32, pc->W32);
  return hipGetLastError();
}

inline void pc_destroy(PcTables* pc) {
  void* ptrs[] = {pc->tw64, pc->W64, pc->tw32, pc->W32, pc->info, pc->np,
                  pc->coef64, pc->coef32, pc->Z, pc->Z2};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  std::memset(pc, 0, sizeof(*pc));
}

inline hipError_t pc_set_field(PcTables* pc, const Geom& g, const double* dbar64, double dtau,
                               double t, double a1, double a2, hipStream_t s) {
  hipLaunchKernelGGL(k_pc_bounds, dim3(1), dim3(256), 0, s, g.N, g.Ltau, dbar64, dtau, t, a1, a2,
                     pc->info, pc->np);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_pc_coef, dim3(pc->H), dim3(256), 0, s, g.Ltau, pc->info, pc->np,
                     pc->coef64, pc->coef32);
  return hipGetLastError();
}

template <typename T, int H1>
hipError_t pc_launch_fwd(const PcTables* pc, const Geom& g, int nrhs, T* in,
                         typename Cplx<T>::type* Z, T* u, const T* pa, const T* pb, const T* Ap, RhsState* st,
                         double* partial, unsigned* counter, bool cgupd, hipStream_t s) {
  const size_t lds = (size_t)pc->H * kSites * sizeof(typename Cplx<T>::type);
  const auto* tw = (const typename Cplx<T>::type*)(sizeof(T) == 8 ? (const void*)pc->tw64 : (const void*)pc->tw32);
  const auto* W = (const typename Cplx<T>::type*)(sizeof(T) == 8 ? (const void*)pc->W64 : (const void*)pc->W32);
  dim3 grid((g.N + kSites - 1) / kSites, nrhs);
  if (cgupd) {
    auto kern = k_tfwd<T, H1, 256, true>;
    if (lds > 48 * 1024) (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(kern, grid, dim3(256), lds, s, g, pc->H2, tw, W, in, Z, u, pa, pb, Ap, st, partial, counter);
  } else {
    auto kern = k_tfwd<T, H1, 256, false>;
    if (lds > 48 * 1024) (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(kern, grid, dim3(256), lds, s, g, pc->H2, tw, W, in, Z, u, pa, pb, Ap, st, partial, counter);
  }
  return hipGetLastError();
}

template <typename T, int H1>
hipError_t pc_launch_inv(const PcTables* pc, const Geom& g, int nrhs,
                         const typename Cplx<T>::type* Zh, T* out, int dot, const T* rdot,
                         RhsState* st, double* partial, unsigned* counter, hipStream_t s) {
  const size_t lds = (size_t)pc->H * kSites * sizeof(typename Cplx<T>::type);
  const auto* tw = (const typename Cplx<T>::type*)(sizeof(T) == 8 ? (const void*)pc->tw64 : (const void*)pc->tw32);
  const auto* W = (const typename Cplx<T>::type*)(sizeof(T) == 8 ? (const void*)pc->W64 : (const void*)pc->W32);
  auto kern = k_tinv<T, H1, 256>;
  if (lds > 48 * 1024) (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(kern, dim3((g.N + kSites - 1) / kSites, nrhs), dim3(256), lds, s, g, pc->H2, tw, W, Zh, out,
                     dot, rdot, st, partial, counter);
  return hipGetLastError();
}

template <typename T>
hipError_t pc_fwd(const PcTables* pc, const Geom& g, int nrhs, T* in, typename Cplx<T>::type* Z,
                  T* u, const T* pa, const T* pb, const T* Ap, RhsState* st, double* partial,
                  unsigned* counter, bool cgupd, hipStream_t s) {
  switch (pc->H1) {
#define FPH_FWD_CASE(h1) \
  case h1: return pc_launch_fwd<T, h1>(pc, g, nrhs, in, Z, u, pa, pb, Ap, st, partial, counter, cgupd, s);
    FPH_FWD_CASE(1) FPH_FWD_CASE(2) FPH_FWD_CASE(3) FPH_FWD_CASE(4) FPH_FWD_CASE(5)
    FPH_FWD_CASE(8) FPH_FWD_CASE(10) FPH_FWD_CASE(16) FPH_FWD_CASE(20)
#undef FPH_FWD_CASE
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t pc_inv(const PcTables* pc, const Geom& g, int nrhs, const typename Cplx<T>::type* Zh,
                  T* out, int dot, const T* rdot, RhsState* st, double* partial,
                  unsigned* counter, hipStream_t s) {
  switch (pc->H1) {
#define FPH_INV_CASE(h1) \
  case h1: return pc_launch_inv<T, h1>(pc, g, nrhs, Zh, out, dot, rdot, st, partial, counter, s);
    FPH_INV_CASE(1) FPH_INV_CASE(2) FPH_INV_CASE(3) FPH_INV_CASE(4) FPH_INV_CASE(5)
    FPH_INV_CASE(8) FPH_INV_CASE(10) FPH_INV_CASE(16) FPH_INV_CASE(20)
#undef FPH_INV_CASE
    default: return hipErrorInvalidValue;
  }
}

template <typename T, int NT, int MS>
hipError_t pc_launch_kpm(const PcTables* pc, const Geom& g, const T* dbar, int op, int nrhs,
                         const typename Cplx<T>::type* Z, typename Cplx<T>::type* Zo,
                         const RhsState* st, T ch, T sh, hipStream_t s) {
  const size_t lds = 2 * (size_t)g.N * sizeof(T);
  auto kern = k_kpm<T, NT, MS>;
  if (lds > 48 * 1024) (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  const auto* cf = (const typename Cplx<T>::type*)(sizeof(T) == 8 ? (const void*)pc->coef64 : (const void*)pc->coef32);
  hipLaunchKernelGGL(kern, dim3(pc->H * nrhs), dim3(NT), lds, s, g, pc->H, nrhs, op, pc->info,
                     pc->np, cf, dbar, ch, sh, Z, Zo, st);
  return hipGetLastError();
}

template <typename T>
hipError_t pc_kpm(const PcTables* pc, const Geom& g, const T* dbar, int op, int nrhs,
                  const typename Cplx<T>::type* Z, typename Cplx<T>::type* Zo, const RhsState* st,
                  T ch, T sh, hipStream_t s) {
  if (g.Q <= 64) return pc_launch_kpm<T, 64, 1>(pc, g, dbar, op, nrhs, Z, Zo, st, ch, sh, s);
  if (g.Q <= 256) return pc_launch_kpm<T, 256, 1>(pc, g, dbar, op, nrhs, Z, Zo, st, ch, sh, s);
  if (g.Q <= 512) return pc_launch_kpm<T, 512, 1>(pc, g, dbar, op, nrhs, Z, Zo, st, ch, sh, s);
  return pc_launch_kpm<T, 1024, 1>(pc, g, dbar, op, nrhs, Z, Zo, st, ch, sh, s);
}

// out = op(in) (op: 0 F, 1 F^T, 2 F F^T).  With rdot != nullptr the inverse
// transform also forms rdot . out and updates rz / beta (residual replaced).
template <typename T>
hipError_t pc_apply(const PcTables* pc, const Geom& g, const T* dbar, int op, int nrhs,
                    const T* in, T* out, RhsState* st, const T* rdot, void* /*reserved*/,
                    double* partial, unsigned* counter, hipStream_t s) {
  using T2 = typename Cplx<T>::type;
  T2* Z = reinterpret_cast<T2*>(pc->Z);
  T2* Z2 = reinterpret_cast<T2*>(pc->Z2);
  hipError_t e = pc_fwd<T>(pc, g, nrhs, const_cast<T*>(in), Z, nullptr, nullptr, nullptr,
                           nullptr, st, partial, counter, false, s);
  if (e != hipSuccess) return e;
  e = pc_kpm<T>(pc, g, dbar, op, nrhs, Z, Z2, st, (T)pc->ch, (T)pc->sh, s);
  if (e != hipSuccess) return e;
  return pc_inv<T>(pc, g, nrhs, Z2, out, rdot ? 2 : 0, rdot, st, partial, counter, s);
}

// Preconditioned CG update: u += alpha p, r -= alpha Ap (with |r|^2 and the
// convergence test), then z = F F^T r and rz_prev = rz, rz = r.z,
// beta = rz / rz_prev.  Three launches.
template <typename T>
hipError_t pc_cg_update(const PcTables* pc, const Geom& g, const T* dbar, int nrhs, T* u,
                        const T* pa, const T* pb, T* r, const T* Ap, T* z, RhsState* st,
                        double* partial, unsigned* counter, hipStream_t s) {
  using T2 = typename Cplx<T>::type;
  T2* Z = reinterpret_cast<T2*>(pc->Z);
  T2* Z2 = reinterpret_cast<T2*>(pc->Z2);
  hipError_t e = pc_fwd<T>(pc, g, nrhs, r, Z, u, pa, pb, Ap, st, partial, counter, true, s);
  if (e != hipSuccess) return e;
  e = pc_kpm<T>(pc, g, dbar, 2, nrhs, Z, Z2, st, (T)pc->ch, (T)pc->sh, s);
  if (e != hipSuccess) return e;
  return pc_inv<T>(pc, g, nrhs, Z2, z, 1, r, st, partial, counter, s);
}

}  // namespace fph
