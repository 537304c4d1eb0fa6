// The adiabatic preconditioner z = F F^T r of one batch item inside its
// workgroup (Sec. V A, Eqs. CG_precon, P_change_basis; App. C).
//
// The same three steps as the single-system kernels (fph_precond.h), run by
// one workgroup over the item's whole vector:
//   1. forward transform: for every tile of KS sites, the twisted half-
//      spectrum DFT over tau, Z_k[i] = (U r)_{2k}, k < H = Ltau/2, through
//      LDS as a Cooley-Tukey split H = H1 H2, into the item's Z workspace;
//   2. for k = 0 .. H-1 in turn, the conjugate series in A^T and then the
//      series in A on block k (cheb_series, one even plaquette per thread,
//      NT >= Q), in place in Z;
//   3. inverse transform of Z into z, with r . z accumulated.
// Everything is FP32 (the iteration precision of the batch); the tables
// (bounds, N_P, coefficients, twiddles) are per system.
#pragma once

#include "fph_common.h"
#include "fph_precond.h"

namespace fph {

// Preconditioner tables of one system (device pointers).
struct BatchPc {
  const PcInfo* info;   // bounds and series constants
  const int* np;        // N_P(w), w < Ltau
  const float2* coef;   // [H][kNPMax]: c_m(2k)
  const float* dbar;    // [N]
  const float2* tw;     // [H]: e^{-i pi tau / Ltau}
  const float2* W;      // [H]: W_H^k
  const float2* F;      // H1 x H1 then H2 x H2 DFT matrices
  float c4;             // cosh(dtau t)^4 (joins dbar in the series)
  int H, H1, H2;
};

// Tile width of the transforms: 32 sites (or N when smaller).
__host__ __device__ inline int bpc_tile_n(int N) { return N >= 32 ? 32 : N; }
FPH_DEVINL int bpc_tile(const Geom& g) { return bpc_tile_n(g.N); }

// LDS (complex values) of the transforms and of the series.
__host__ __device__ inline long bpc_lds_tf(int H, int H1, int H2, int KS) {
  return (long)H1 * H1 + (long)H2 * H2 + H + 2L * H * KS;
}
__host__ __device__ inline long bpc_lds_series(int L) {
  return 2L * (2L * kpm_row_stride(L / 2) * L + kWinPad);
}

// Forward transform of the item's r (FP32 [Ltau][N]) into Z ([H][N] complex).
template <int NT>
FPH_DEVINL void bpc_forward(const Geom& g, const BatchPc& pc, const float* __restrict__ r,
                            float2* __restrict__ Z, float2* lds) {
  const int H = pc.H, H1 = pc.H1, H2 = pc.H2, KS = bpc_tile(g);
  const int nF = H1 * H1 + H2 * H2;
  float2* Fl = lds;
  float2* Wl = Fl + nF;
  float2* Y0 = Wl + H;
  float2* Y1 = Y0 + H * KS;
  for (int k = threadIdx.x; k < nF; k += NT) Fl[k] = pc.F[k];
  for (int k = threadIdx.x; k < H; k += NT) Wl[k] = pc.W[k];
  const float scale = (float)(1.0 / sqrt((double)g.Ltau));
  const long hN = (long)H * g.N;
  for (int i0 = 0; i0 < g.N; i0 += KS) {
    // stage 0: y_tau = e^{-i pi tau/Ltau} (r_tau - i r_{tau+H})
    for (int e = threadIdx.x; e < H * KS; e += NT) {
      const int tau = e / KS, s = e - tau * KS;
      float a = 0.f, b = 0.f;
      if (i0 + s < g.N) {
        const long o = (long)tau * g.N + i0 + s;
        a = r[o];
        b = r[o + hN];
      }
      const float2 t = pc.tw[tau];
      Y0[e] = make_float2(t.x * a + t.y * b, t.y * a - t.x * b);
    }
    __syncthreads();
    // step 1: H1-point DFTs over n1 of y_{n2 + H2 n1}, times W_H^{n2 k1}
    for (int it = threadIdx.x; it < KS * H; it += NT) {
      const int s = it % KS, rest = it / KS;  // n2 * H1 + k1
      const int n2 = rest / H1, k1 = rest - n2 * H1;
      float2 acc = make_float2(0.f, 0.f);
      for (int n1 = 0; n1 < H1; ++n1) cmac(acc, Fl[k1 * H1 + n1], Y0[(n2 + H2 * n1) * KS + s]);
      Y1[it] = cmul<float2, float>(acc, Wl[(n2 * k1) % H]);
    }
    __syncthreads();
    // step 2: H2-point DFTs over n2 -> Z_{k1 + H1 k2}
    for (int it = threadIdx.x; it < KS * H; it += NT) {
      const int s = it % KS, kk = it / KS;
      const int k2 = kk / H1, k1 = kk - k2 * H1;
      if (i0 + s >= g.N) continue;
      float2 x = make_float2(0.f, 0.f);
      for (int n2 = 0; n2 < H2; ++n2)
        cmac(x, Fl[H1 * H1 + k2 * H2 + n2], Y1[(n2 * H1 + k1) * KS + s]);
      Z[(long)kk * g.N + i0 + s] = make_float2(x.x * scale, x.y * scale);
    }
    __syncthreads();
  }
}

// Inverse transform of Z into z ([Ltau][N]); returns (thread-local)
// partial sums of r . z.
template <int NT>
FPH_DEVINL double bpc_inverse(const Geom& g, const BatchPc& pc, const float2* __restrict__ Z,
                              const float* __restrict__ r, float* __restrict__ z, float2* lds) {
  const int H = pc.H, H1 = pc.H1, H2 = pc.H2, KS = bpc_tile(g);
  const int nF = H1 * H1 + H2 * H2;
  float2* Fl = lds;
  float2* Wl = Fl + nF;
  float2* Zt = Wl + H;
  float2* Y = Zt + H * KS;
  for (int k = threadIdx.x; k < nF; k += NT) Fl[k] = pc.F[k];
  for (int k = threadIdx.x; k < H; k += NT) Wl[k] = pc.W[k];
  const float scale = (float)(2.0 / sqrt((double)g.Ltau));
  const long hN = (long)H * g.N;
  double acc_dot = 0.0;
  for (int i0 = 0; i0 < g.N; i0 += KS) {
    for (int e = threadIdx.x; e < H * KS; e += NT) {
      const int k = e / KS, s = e - k * KS;
      Zt[e] = (i0 + s < g.N) ? Z[(long)k * g.N + i0 + s] : make_float2(0.f, 0.f);
    }
    __syncthreads();
    for (int it = threadIdx.x; it < KS * H; it += NT) {
      const int s = it % KS, rest = it / KS;  // n2 * H1 + k1
      const int n2 = rest / H1, k1 = rest - n2 * H1;
      float2 acc = make_float2(0.f, 0.f);
      for (int n1 = 0; n1 < H1; ++n1) cmacc(acc, Fl[k1 * H1 + n1], Zt[(n2 + H2 * n1) * KS + s]);
      Y[it] = cmulc<float2, float>(acc, Wl[(n2 * k1) % H]);
    }
    __syncthreads();
    for (int it = threadIdx.x; it < KS * H; it += NT) {
      const int s = it % KS, tau = it / KS;  // k1 + H1 k2
      const int k2 = tau / H1, k1 = tau - k2 * H1;
      if (i0 + s >= g.N) continue;
      float2 x = make_float2(0.f, 0.f);
      for (int n2 = 0; n2 < H2; ++n2)
        cmacc(x, Fl[H1 * H1 + k2 * H2 + n2], Y[(n2 * H1 + k1) * KS + s]);
      const float2 sv = cmulc<float2, float>(x, pc.tw[tau]);
      const long oa = (long)tau * g.N + i0 + s;
      const float va = scale * sv.x, vb = -scale * sv.y;
      z[oa] = va;
      z[oa + hN] = vb;
      acc_dot += (double)r[oa] * (double)va + (double)r[oa + hN] * (double)vb;
    }
    __syncthreads();
  }
  return acc_dot;
}

// F F^T on every frequency block of Z, in place: block k gets the
// conjugate series in A^T, then the series in A (as k_kpm with op 2).
// Requires NT >= Q (one even plaquette per thread; the others run the same
// branch-free steps on spare LDS entries).  N_P is uniform over the
// workgroup for each block, so every thread takes the same barriers; a
// block with N_P = 1 takes none.  The coefficients are read from the table
// in global memory (the same address in every thread); consecutive series
// need no barrier between them beyond the one cheb_series itself takes.
// th = tanh(dtau t) (the primed checkerboard factors).
template <int NT>
FPH_DEVINL void bpc_series(const Geom& g, const BatchPc& pc, float th, float2* __restrict__ Z,
                           float2* lds) {
  const int S = kpm_row_stride(g.hL);
  const int nbuf = 2 * S * g.L + kWinPad;
  float2* buf0 = lds;
  float2* buf1 = buf0 + nbuf;
  const int q = threadIdx.x;
  const bool own = q < g.Q;
  const Win w = make_win(g, q, own);
  const int i0 = w.x0 + w.row[1], iL = i0 + g.L;
  const float sA = (float)pc.info->s, cA = (float)pc.info->c;
  float db[4];
  if (own) {
    db[0] = pc.c4 * pc.dbar[i0];
    db[1] = pc.c4 * pc.dbar[i0 + 1];
    db[2] = pc.c4 * pc.dbar[iL];
    db[3] = pc.c4 * pc.dbar[iL + 1];
  } else {
#pragma unroll
    for (int m = 0; m < 4; ++m) db[m] = 1.f;
  }
  for (int k = 0; k < pc.H; ++k) {
    const int NP = pc.np[2 * k];
    float2* Zk = Z + (long)k * g.N;
    float2 x[4], acc[4];
    if (own) {
      ld2c(Zk + i0, x[0], x[1]);
      ld2c(Zk + iL, x[2], x[3]);
    } else {
#pragma unroll
      for (int m = 0; m < 4; ++m) x[m] = make_float2(0.f, 0.f);
    }
    const float2* cfs = pc.coef + (long)k * kNPMax;
    cheb_series<float, true, false>(w, NP, cfs, sA, cA, x, db, buf0, buf1, th, acc, q, g.Q);
#pragma unroll
    for (int m = 0; m < 4; ++m) x[m] = acc[m];
    cheb_series<float, false, false>(w, NP, cfs, sA, cA, x, db, buf0, buf1, th, acc, q, g.Q);
    if (own) {
      st2c(Zk + i0, acc[0], acc[1]);
      st2c(Zk + iL, acc[2], acc[3]);
    }
  }
  __syncthreads();
}

}  // namespace fph
