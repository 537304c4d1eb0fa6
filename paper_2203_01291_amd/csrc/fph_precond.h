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
#include <type_traits>

#include "fph_common.h"

namespace fph {

constexpr int kNPMax = 1024;   // cap on the Chebyshev order N_P(w)

template <typename T> struct Cplx;
template <> struct Cplx<double> { using type = double2; };
template <> struct Cplx<float> { using type = float2; };

struct PcTables {
  int H, H1, H2;
  double2* tw64;   // e^{-i pi tau / Ltau}, tau < H
  double2* W64;    // e^{-2 pi i k / H}, k < H
  double2* F64;    // H1 x H1 then H2 x H2 small-DFT matrices (see k_pc_twiddles)
  float2* tw32;
  float2* W32;
  float2* F32;
  PcInfo* info;    // bounds and series constants (device)
  int* np;         // N_P(w) for w < Ltau (device)
  double2* coef64; // [H][kNPMax]: c_m(2k)
  float2* coef32;
  void* Z;         // complex workspace, max_rhs * H * N (double2)
  void* Z2;
  double th, c4;   // tanh(dtau t) and cosh(dtau t)^4: P_A P_B = c4 P'_A P'_B, C2' = [[1, th], [th, 1]]
};

// First factor of the length-H DFT split H = H1 * H2: at most 10 when
// possible (H1 complex values per thread stay in registers), H2 <= 32.
inline int pick_h1(int H) {
  static const int cand[] = {10, 8, 5, 4, 3, 2, 16, 20, 1};
  for (int h1 : cand)
    if (H % h1 == 0 && H / h1 <= 32) return h1;
  return 0;
}

inline bool pc_supported(int Ltau) { return Ltau >= 2 && Ltau % 2 == 0 && pick_h1(Ltau / 2) > 0; }

// ----------------------------------------------------------- setup kernels

// Twiddles: tw[tau] = e^{-i pi tau/Ltau}, W[k] = W_H^k, and the matrices of
// the two short DFTs, F[k1 H1 + n1] = W_H1^{n1 k1} (H1 x H1) followed by
// F[H1^2 + k2 H2 + n2] = W_H2^{n2 k2} (H2 x H2), so that a thread computing
// one output reads its row with unit stride.
__global__ void k_pc_twiddles(int H, int H1, int H2, int Ltau, double2* tw64, double2* W64,
                              double2* F64, float2* tw32, float2* W32, float2* F32) {
  const int nF = H1 * H1 + H2 * H2;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < H + nF; k += gridDim.x * blockDim.x) {
    if (k < H) {
      const double a = (double)k / (double)Ltau;      // twist angle / pi
      const double b = 2.0 * (double)k / (double)H;   // DFT angle / pi
      const double2 t = make_double2(cospi(a), -sinpi(a));
      const double2 w = make_double2(cospi(b), -sinpi(b));
      tw64[k] = t;
      W64[k] = w;
      tw32[k] = make_float2((float)t.x, (float)t.y);
      W32[k] = make_float2((float)w.x, (float)w.y);
    } else {
      const int f = k - H;
      int n, m;
      if (f < H1 * H1) {
        m = ((f / H1) * (f % H1)) % H1;
        n = H1;
      } else {
        const int g = f - H1 * H1;
        m = ((g / H2) * (g % H2)) % H2;
        n = H2;
      }
      const double c = 2.0 * (double)m / (double)n;
      const double2 w = make_double2(cospi(c), -sinpi(c));
      F64[f] = w;
      F32[f] = make_float2((float)w.x, (float)w.y);
    }
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

// Transform workgroups own a tile of KS = 2^lks consecutive sites (all
// slices of them), as wide as pc_tile_log2 allows.  Workgroups are numbered with
// xcd_contiguous so neighbouring tiles (which share cache lines) run on
// one XCD.  The two short DFTs read their matrix rows (F, see
// k_pc_twiddles) and their inputs with unit and constant strides from LDS.

template <typename T2>
FPH_DEVINL void cmac(T2& acc, T2 w, T2 y) {  // acc += w y
  acc.x = fma(w.x, y.x, fma(-w.y, y.y, acc.x));
  acc.y = fma(w.x, y.y, fma(w.y, y.x, acc.y));
}

template <typename T2>
FPH_DEVINL void cmacc(T2& acc, T2 w, T2 y) {  // acc += conj(w) y
  acc.x = fma(w.x, y.x, fma(w.y, y.y, acc.x));
  acc.y = fma(w.x, y.y, fma(-w.y, y.x, acc.y));
}

// Two outputs of a short DFT of even length n over the values y[j s],
// j < n, from the row fr of its matrix (fr[j] = W_n^{j k}, conjugated with
// CONJ): outputs k and k + n/2 share every product, as
// W_n^{j (k + n/2)} = (-1)^j W_n^{j k}; the even and odd terms summed
// apart give a = e + o (output k) and b = e - o (output k + n/2).
template <bool CONJ, int NU, typename T2>
FPH_DEVINL void dft_pair(const T2* fr, const T2* y, int s, int n, T2& a, T2& b) {
  T2 e = T2{0, 0}, o = T2{0, 0};
#pragma unroll NU
  for (int j = 0; j < n; j += 2) {
    if (CONJ) {
      cmacc(e, fr[j], y[j * s]);
      cmacc(o, fr[j + 1], y[(j + 1) * s]);
    } else {
      cmac(e, fr[j], y[j * s]);
      cmac(o, fr[j + 1], y[(j + 1) * s]);
    }
  }
  a = T2{e.x + o.x, e.y + o.y};
  b = T2{e.x - o.x, e.y - o.y};
}

// Forward transform of one tile of sites: Z[r][k][i] = (U in)_{2k}.
// Stage 0, item (tau < H, site), coalesced: y_tau = e^{-i pi tau/Ltau}
// (in_tau - i in_{tau+H}) into LDS.  With CGUPD both inputs first receive
// the CG update u += alpha p, r -= alpha Ap (r is `in`, updated in place),
// publishing |r|^2 as P_RR partials; the direction is pb on even iteration
// counts, pa on odd.  A right-hand side whose FP64 residual was just
// evaluated (the folded partials were P_RES) is transformed without the
// update; an FP32 correction u the state marks as zero is read as zero.
// The state loads are issued first, then the loads of the first pass (two
// items per thread) other than the direction, which needs the state.
// Step 1, item (site, n2, k1): output k1 of the H1-point DFT over
// n1 of y_{H2 n1 + n2}, times W_H^{n2 k1}.  Step 2, item (site, k1, k2):
// the H2-point DFT over n2 -> Z_{k1 + H1 k2}.
// Launch: grid ntiles * nrhs, NT threads; LDS (H1^2 + H2^2 + H + 2 H KS)
// complex values.  KI stage-0 items per thread and pass: 4 where 2 would
// take a second pass (each pass is one dependent round trip to memory).
template <typename T, int H1, int NT, bool CGUPD, int KI>
__global__ void __launch_bounds__(NT)
k_tfwd(Geom g, int H2, const typename Cplx<T>::type* __restrict__ tw,
       const typename Cplx<T>::type* __restrict__ W, const typename Cplx<T>::type* __restrict__ F,
       T* __restrict__ in, typename Cplx<T>::type* __restrict__ Z, T* __restrict__ u,
       const T* pa, const T* pb, const T* __restrict__ Ap, int lks, int ntiles, StIO io) {
  using T2 = typename Cplx<T>::type;
  constexpr int kI = KI;  // stage-0 items per thread and pass
  const int KS = 1 << lks;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int H = H1 * H2;
  const int nF = H1 * H1 + H2 * H2;
  T2* Fl = reinterpret_cast<T2*>(smem_raw);
  T2* Wl = Fl + nF;
  T2* Y0 = Wl + H;
  T2* Y1 = Y0 + H * KS;
  __shared__ double red_sh[NT / 64];
  __shared__ RhsState s_sh;
  const int logical = xcd_contiguous(blockIdx.x, gridDim.x);
  const int r = logical % (gridDim.x / ntiles);
  const int tile = logical / (gridDim.x / ntiles);
  const int i0 = tile * KS;
  const long base = (long)r * g.d;
  const long hN = (long)H * g.N;
  const int npair = H << lks;

  // Inputs of one pass of stage 0 (kI items per thread): r (and with
  // CGUPD Ap, u, the direction p) at slices tau and tau + H, and the twist.
  struct Pass {
    T ra[kI], rb[kI], aa[kI], ab[kI], ua[kI], ub[kI], pa[kI], pb[kI];
    T2 tw[kI];
  };
  // Items past the last pair, or on a site past the end of a ragged tile,
  // load a valid element instead (slice 0, the last site): the loads stay
  // unconditional, so none waits for the others, and the values are never
  // used (stage 0 skips such items and stores nothing for a ragged site; a
  // ragged site's column of the transforms is not written out).
  auto load = [&](Pass& P, int e0, bool all, bool dir, const T* p) {
#pragma unroll
    for (int j = 0; j < kI; ++j) {
      const int e = e0 + j * NT;
      const int ec = e < npair ? e : 0;
      const int tau = ec >> lks;
      const int site = min(i0 + (ec & (KS - 1)), g.N - 1);
      const long oa = base + (long)tau * g.N + site;
      if (all) {
        P.ra[j] = in[oa];
        P.rb[j] = in[oa + hN];
        P.tw[j] = tw[tau];
      }
      if (CGUPD) {
        if (all) {
          P.aa[j] = Ap[oa];
          P.ab[j] = Ap[oa + hN];
          P.ua[j] = u[oa];
          P.ub[j] = u[oa + hN];
        }
        if (dir) {
          P.pa[j] = p[oa];
          P.pb[j] = p[oa + hN];
        }
      }
    }
  };
  // Issue order: the state (first, so that folding it waits for nothing
  // else), the first pass of inputs, the DFT tables.  In FP32 the tables
  // go to registers and reach LDS after the fold (before the barrier that
  // ends stage 0); in FP64, where the registers would cost occupancy, they
  // are stored before the fold.
  constexpr bool kTabRegs = sizeof(T) == 4;
  StLoad<16> sl;
  if (io.in != nullptr) state_issue(io, r, sl);
  Pass P0;
  load(P0, threadIdx.x, true, false, pa);
  constexpr int kTab = kTabRegs ? 6 : 1;  // (H1^2 + H2^2 + H) <= 6 NT: H1 <= 20, H2 <= 32
  // Entry k of the LDS table is F[k] for k < nF, else W[k - nF]: one load
  // from a selected address (W's index clamped into range), no branch.
  T2 tab[kTab];
  if constexpr (kTabRegs) {
#pragma unroll
    for (int j = 0; j < kTab; ++j) {
      const int k = threadIdx.x + j * NT;
      tab[j] = *(k < nF ? F + k : W + min(max(k - nF, 0), H - 1));
    }
  } else {
    for (int k = threadIdx.x; k < nF; k += NT) Fl[k] = F[k];
    for (int k = threadIdx.x; k < H; k += NT) Wl[k] = W[k];
  }
  if (io.in != nullptr) {
    state_finish<NT>(io, r, sl, &s_sh);
    if (s_sh.done) {
      state_end(io, r, &s_sh, P_NONE, 0.0, tile, ntiles, tile == 0);
      return;
    }
  }
  if constexpr (kTabRegs) {
#pragma unroll
    for (int j = 0; j < kTab; ++j) {
      const int k = threadIdx.x + j * NT;
      if (k < nF + H) Fl[k] = tab[j];  // Wl follows Fl
    }
  }
  const T scale = (T)(1.0 / sqrt((double)g.Ltau));
  double acc_rr = 0.0;
  const bool upd = CGUPD && s_sh.folded == P_PAP;
  const bool uz = CGUPD && s_sh.u32z != 0;

  // Stage 0.  The direction p (the buffer the state names) is used only
  // to update u; for the first pass that update is deferred to the end of
  // the kernel, so the loads of p issued here arrive while the DFT runs.
  T alpha = (T)0;
  const T* p = pa;
  if (CGUPD) {
    alpha = (T)s_sh.alpha;
    p = (s_sh.iter & 1) ? pa : pb;  // direction written by this iteration
    if (upd) load(P0, threadIdx.x, false, true, p);
  }
  auto update_u = [&](const Pass& P, int e0) {
#pragma unroll
    for (int j = 0; j < kI; ++j) {
      const int e = e0 + j * NT;
      const int tau = e >> lks, sidx = e & (KS - 1);
      if (e >= npair || i0 + sidx >= g.N) continue;
      const long oa = base + (long)tau * g.N + i0 + sidx;
      u[oa] = (uz ? (T)0 : P.ua[j]) + alpha * P.pa[j];
      u[oa + hN] = (uz ? (T)0 : P.ub[j]) + alpha * P.pb[j];
    }
  };
  auto stage0 = [&](const Pass& P, int e0) {
#pragma unroll
    for (int j = 0; j < kI; ++j) {
      const int e = e0 + j * NT;
      if (e >= npair) continue;
      const int tau = e >> lks, sidx = e & (KS - 1);
      T a = P.ra[j], b = P.rb[j];
      if (upd && i0 + sidx < g.N) {
        const long oa = base + (long)tau * g.N + i0 + sidx;
        a -= alpha * P.aa[j];
        b -= alpha * P.ab[j];
        in[oa] = a;
        in[oa + hN] = b;
        acc_rr += (double)a * (double)a + (double)b * (double)b;
      }
      const T2 t = P.tw[j];
      Y0[tau * KS + sidx] = T2{t.x * a + t.y * b, t.y * a - t.x * b};
    }
  };
  stage0(P0, threadIdx.x);
  for (int e0 = threadIdx.x + kI * NT; e0 < npair; e0 += kI * NT) {
    Pass P;
    load(P, e0, true, upd, p);
    stage0(P, e0);
    if (upd) update_u(P, e0);
  }
  __syncthreads();
  // Steps 1 and 2 compute their outputs in pairs (k, k + n/2, dft_pair)
  // when the factor is even: half the items, each reading its inputs once.
  const int s1 = H2 << lks;  // Y0 stride between consecutive n1
  if constexpr (H1 % 2 == 0) {
    constexpr int h1 = H1 / 2;
    for (int it = threadIdx.x; it < (KS * H) / 2; it += NT) {
      const int sidx = it & (KS - 1);
      const int rest = it >> lks;  // n2 * h1 + k1, k1 < H1 / 2
      const int n2 = rest / h1, k1 = rest - n2 * h1;
      T2 a, b;
      dft_pair<false, H1 / 2>(Fl + k1 * H1, Y0 + n2 * KS + sidx, s1, H1, a, b);
      const int ia = ((n2 * H1 + k1) << lks) + sidx;
      Y1[ia] = cmul<T2, T>(a, Wl[(n2 * k1) % H]);
      Y1[ia + (h1 << lks)] = cmul<T2, T>(b, Wl[(n2 * (k1 + h1)) % H]);
    }
  } else {
    for (int it = threadIdx.x; it < KS * H; it += NT) {
      const int sidx = it & (KS - 1);
      const int rest = it >> lks;  // n2 * H1 + k1
      const int n2 = rest / H1, k1 = rest - n2 * H1;
      const T2* yp = Y0 + n2 * KS + sidx;
      const T2* fr = Fl + k1 * H1;
      T2 acc = T2{(T)0, (T)0};
#pragma unroll
      for (int n1 = 0; n1 < H1; ++n1) cmac(acc, fr[n1], yp[n1 * s1]);
      Y1[it] = cmul<T2, T>(acc, Wl[(n2 * k1) % H]);
    }
  }
  __syncthreads();
  const int s2 = H1 << lks;  // Y1 stride between consecutive n2
  if (H2 % 2 == 0) {
    const int h2 = H2 / 2;
    for (int it = threadIdx.x; it < (KS * H) / 2; it += NT) {
      const int sidx = it & (KS - 1);
      const int kk = it >> lks;  // k1 + H1 k2, k2 < H2 / 2
      const int k2 = kk / H1, k1 = kk - k2 * H1;
      if (i0 + sidx >= g.N) continue;
      T2 a, b;
      dft_pair<false, 2>(Fl + H1 * H1 + k2 * H2, Y1 + k1 * KS + sidx, s2, H2, a, b);
      T2* zp = Z + ((long)r * H + kk) * g.N + i0 + sidx;
      zp[0] = T2{a.x * scale, a.y * scale};
      zp[(long)H1 * h2 * g.N] = T2{b.x * scale, b.y * scale};  // output kk + H1 H2 / 2
    }
  } else {
    for (int it = threadIdx.x; it < KS * H; it += NT) {
      const int sidx = it & (KS - 1);
      const int kk = it >> lks;  // k1 + H1 k2 = output frequency
      const int k2 = kk / H1, k1 = kk - k2 * H1;
      if (i0 + sidx >= g.N) continue;
      const T2* yp = Y1 + k1 * KS + sidx;
      const T2* fr = Fl + H1 * H1 + k2 * H2;
      T2 x = T2{(T)0, (T)0};
#pragma unroll 4
      for (int n2 = 0; n2 < H2; ++n2) cmac(x, fr[n2], yp[n2 * s2]);
      Z[((long)r * H + kk) * g.N + i0 + sidx] = T2{x.x * scale, x.y * scale};
    }
  }

  if (upd) update_u(P0, threadIdx.x);
  if (io.in != nullptr) {
    double bs = 0.0;
    if (upd) {
      bs = block_sum<NT, true>(acc_rr, red_sh);
      if (threadIdx.x == 0) s_sh.u32z = 0;
    }
    state_end(io, r, &s_sh, upd ? P_RR : P_NONE, bs, tile, ntiles, tile == 0);
  }
}

// Inverse transform: out[r][tau][i] from Zh[r][k][i] (the same two short
// DFTs with conjugated matrices, then the conjugate twist and the real
// split into tau and tau + H).  Stage 0 copies the tile Zh[k][i0..i0+KS)
// to LDS with coalesced loads; the solver state, issued before them, is
// folded after step 1 (it only decides whether the right-hand side is
// skipped).  With dot != 0 also publishes rdot . out as P_RZ partials.  LDS:
// (H1^2 + H2^2 + H + 2 H KS) complex values.  KI input items per thread and
// pass: 4, or 2 where that already covers the tile in one pass (FP32 loads
// every item slot, in range or not).
template <typename T, int H1, int NT, int KI>
__global__ void __launch_bounds__(NT)
k_tinv(Geom g, int H2, const typename Cplx<T>::type* __restrict__ tw,
       const typename Cplx<T>::type* __restrict__ W, const typename Cplx<T>::type* __restrict__ F,
       const typename Cplx<T>::type* __restrict__ Zh, T* __restrict__ out, int dot,
       const T* __restrict__ rdot, int lks, int ntiles, StIO io) {
  using T2 = typename Cplx<T>::type;
  constexpr int kI = KI;
  const int KS = 1 << lks;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int H = H1 * H2;
  const int nF = H1 * H1 + H2 * H2;
  T2* Fl = reinterpret_cast<T2*>(smem_raw);
  T2* Wl = Fl + nF;
  T2* Zt = Wl + H;
  T2* Y = Zt + H * KS;
  __shared__ double red_sh[NT / 64];
  __shared__ RhsState s_sh;
  const int logical = xcd_contiguous(blockIdx.x, gridDim.x);
  const int r = logical % (gridDim.x / ntiles);
  const int tile = logical / (gridDim.x / ntiles);
  const int i0 = tile * KS;
  const long base = (long)r * g.d;
  const int nel = H << lks;

  // The state is needed only to skip a finished right-hand side and to
  // publish r.z, so its loads go first and are folded after the first
  // short DFT, once they have arrived.
  StLoad<0> sl;  // kpm, the kernel before in a solve, publishes no partials
  if (io.in != nullptr) state_issue(io, r, sl);
  // DFT tables: LDS entry k is F[k] for k < nF, else W[k - nF].  The first
  // kTabR NT entries are loaded into registers here, with the inputs, and
  // stored once they have arrived (a load-and-store loop here would wait
  // for every load issued before it).  FP32: one load per entry from a
  // selected address (W's index clamped into range); FP64, where that
  // measured slower: both arrays at clamped indexes, one store of the two.
  constexpr int kTabR = 2;
  constexpr bool kSel = sizeof(T) == 4;
  T2 tabf[kTabR], tabw[kSel ? 1 : kTabR];
#pragma unroll
  for (int j = 0; j < kTabR; ++j) {
    const int k = threadIdx.x + j * NT;
    if constexpr (kSel) {
      tabf[j] = *(k < nF ? F + k : W + min(max(k - nF, 0), H - 1));
    } else {
      tabf[j] = F[min(k, nF - 1)];
      tabw[j] = W[min(max(k - nF, 0), H - 1)];
    }
  }
  // In FP32, out-of-range items load a valid element instead (no branch,
  // so no load waits for the ones before it); their values are never
  // used: only items in range reach LDS, and a ragged site's column is not
  // written out.  (In FP64 that form puts v in private memory; there the
  // loads stay conditional.)
  T2 v[kI];
  auto load = [&](int e0) {
#pragma unroll
    for (int j = 0; j < kI; ++j) {
      const int e = e0 + j * NT;
      if constexpr (sizeof(T) == 4) {
        const int ec = e < nel ? e : 0;
        const int site = min(i0 + (ec & (KS - 1)), g.N - 1);
        v[j] = Zh[((long)r * H + (ec >> lks)) * g.N + site];
      } else {
        const int k = e >> lks, sidx = e & (KS - 1);
        v[j] = (e < nel && i0 + sidx < g.N) ? Zh[((long)r * H + k) * g.N + i0 + sidx]
                                           : T2{(T)0, (T)0};
      }
    }
  };
  load(threadIdx.x);
  // Steps 1 and 2 compute their outputs in pairs (dft_pair) when both
  // factors are even; step 2 then writes slices tau and tau + H1 H2 / 2 of
  // each pair item.  In FP32 the twist and r (for r.z) of the first kPre
  // passes of paired step-2 items are loaded with the inputs, not inside
  // step 2 (in FP64 the registers would cost occupancy).
  constexpr bool kPair1 = H1 % 2 == 0;
  const bool pair = kPair1 && H2 % 2 == 0;
  const int hh = H / 2;  // H1 H2 / 2: tau of the second output of a pair item
  constexpr int kPre = sizeof(T) == 4 ? 2 : 0;
  T2 twp[kPre > 0 ? kPre : 1][2];
  T rdp[kPre > 0 ? kPre : 1][4];
  const long hN = (long)H * g.N;
  if (pair) {
#pragma unroll
    for (int j = 0; j < kPre; ++j) {
      // As above, out-of-range items load valid elements they never use
      // (rdot is a readable buffer even without r.z).
      const int it0 = threadIdx.x + j * NT;
      const int it = it0 < (KS * H) / 2 ? it0 : 0;
      const int pi = it >> lks;  // k1 + H1 k2, k2 < H2 / 2
      const long oa = base + (long)pi * g.N + min(i0 + (it & (KS - 1)), g.N - 1);
      const long oc = oa + (long)hh * g.N;
      twp[j][0] = tw[pi];
      twp[j][1] = tw[pi + hh];
      rdp[j][0] = rdot[oa];
      rdp[j][1] = rdot[oa + hN];
      rdp[j][2] = rdot[oc];
      rdp[j][3] = rdot[oc + hN];
    }
  }
#pragma unroll
  for (int j = 0; j < kTabR; ++j) {
    const int k = threadIdx.x + j * NT;
    // Wl follows Fl.  (Guarded stores: a select between the two register
    // arrays can be compiled as an indexed private array.)
    if constexpr (kSel) {
      if (k < nF + H) Fl[k] = tabf[j];
    } else {
      if (k < nF) Fl[k] = tabf[j];
      else if (k < nF + H) Fl[k] = tabw[j];
    }
  }
  for (int k = threadIdx.x + kTabR * NT; k < nF + H; k += NT) Fl[k] = k < nF ? F[k] : W[k - nF];
  const T scale = (T)(2.0 / sqrt((double)g.Ltau));
  double acc_dot = 0.0;

  for (int e0 = threadIdx.x; e0 < nel; e0 += kI * NT) {
    if (e0 != (int)threadIdx.x) load(e0);
#pragma unroll
    for (int j = 0; j < kI; ++j)
      if (e0 + j * NT < nel) Zt[e0 + j * NT] = v[j];
  }
  __syncthreads();
  const int s1 = H2 << lks;
  if constexpr (kPair1) {
    constexpr int h1 = H1 / 2;
    for (int it = threadIdx.x; it < (KS * H) / 2; it += NT) {
      const int sidx = it & (KS - 1);
      const int rest = it >> lks;  // n2 * h1 + k1, k1 < H1 / 2
      const int n2 = rest / h1, k1 = rest - n2 * h1;
      T2 a, b;
      dft_pair<true, H1 / 2>(Fl + k1 * H1, Zt + n2 * KS + sidx, s1, H1, a, b);
      const int ia = ((n2 * H1 + k1) << lks) + sidx;
      Y[ia] = cmulc<T2, T>(a, Wl[(n2 * k1) % H]);
      Y[ia + (h1 << lks)] = cmulc<T2, T>(b, Wl[(n2 * (k1 + h1)) % H]);
    }
  } else {
    for (int it = threadIdx.x; it < KS * H; it += NT) {
      const int sidx = it & (KS - 1);
      const int rest = it >> lks;  // n2 * H1 + k1
      const int n2 = rest / H1, k1 = rest - n2 * H1;
      const T2* yp = Zt + n2 * KS + sidx;
      const T2* fr = Fl + k1 * H1;
      T2 acc = T2{(T)0, (T)0};
#pragma unroll
      for (int n1 = 0; n1 < H1; ++n1) cmacc(acc, fr[n1], yp[n1 * s1]);
      Y[it] = cmulc<T2, T>(acc, Wl[(n2 * k1) % H]);
    }
  }
  if (io.in != nullptr) {
    state_finish<NT>(io, r, sl, &s_sh);  // its barrier also orders Y
    if (s_sh.done) {
      state_end(io, r, &s_sh, P_NONE, 0.0, tile, ntiles, tile == 0);
      return;
    }
  } else {
    __syncthreads();
  }
  const int s2 = H1 << lks;
  // Output slice tau (and tau + H) of one site from the step-2 sum x.
  auto emit = [&](int tau, int sidx, const T2& x, T2 twt, T ra, T rb, bool pre) {
    const long oa = base + (long)tau * g.N + i0 + sidx;
    const long ob = oa + hN;
    if (!pre) {
      twt = tw[tau];
      if (dot) {
        ra = rdot[oa];
        rb = rdot[ob];
      }
    }
    const T2 sv = cmulc<T2, T>(x, twt);
    const T va = scale * sv.x, vb = -scale * sv.y;
    out[oa] = va;
    out[ob] = vb;
    if (dot) acc_dot += (double)ra * (double)va + (double)rb * (double)vb;
  };
  if (pair) {
    const int h2 = H2 / 2;
    auto step2p = [&](int it, int j, bool pre) {
      const int sidx = it & (KS - 1);
      const int pi = it >> lks;  // k1 + H1 k2, k2 < H2 / 2
      const int k2 = pi / H1, k1 = pi - k2 * H1;
      if (i0 + sidx >= g.N) return;
      T2 a, b;
      dft_pair<true, 2>(Fl + H1 * H1 + k2 * H2, Y + k1 * KS + sidx, s2, H2, a, b);
      const T2 z0 = T2{(T)0, (T)0};
      emit(pi, sidx, a, pre ? twp[j][0] : z0, pre ? rdp[j][0] : (T)0, pre ? rdp[j][1] : (T)0, pre);
      emit(pi + H1 * h2, sidx, b, pre ? twp[j][1] : z0, pre ? rdp[j][2] : (T)0,
           pre ? rdp[j][3] : (T)0, pre);
    };
#pragma unroll
    for (int j = 0; j < kPre; ++j) {
      const int it = threadIdx.x + j * NT;
      if (it < (KS * H) / 2) step2p(it, j, true);
    }
    for (int it = threadIdx.x + kPre * NT; it < (KS * H) / 2; it += NT) step2p(it, 0, false);
  } else {
    for (int it = threadIdx.x; it < KS * H; it += NT) {
      const int sidx = it & (KS - 1);
      const int tau = it >> lks;  // k1 + H1 k2
      const int k2 = tau / H1, k1 = tau - k2 * H1;
      if (i0 + sidx >= g.N) continue;
      const T2* yp = Y + k1 * KS + sidx;
      const T2* fr = Fl + H1 * H1 + k2 * H2;
      T2 x = T2{(T)0, (T)0};
#pragma unroll 4
      for (int n2 = 0; n2 < H2; ++n2) cmacc(x, fr[n2], yp[n2 * s2]);
      emit(tau, sidx, x, T2{(T)0, (T)0}, (T)0, (T)0, false);
    }
  }

  if (io.in != nullptr) {
    double bs = 0.0;
    if (dot) bs = block_sum<NT, true>(acc_dot, red_sh);
    state_end(io, r, &s_sh, dot ? P_RZ : P_NONE, bs, tile, ntiles, tile == 0);
  }
}

// ------------------------------------------------------------ KPM kernel

// Sites around the even plaquette with corner (x0, y0): rows y0-1, y0,
// y0+1, y0+2 and columns x0-1, x0..x0+1, x0+2 (periodic).  The odd
// plaquettes of P_B that cover the plaquette's four sites lie in this
// window (site (dx, dy) of the even plaquette is local site (1-dx, 1-dy)
// of its odd plaquette).  A slice in LDS is stored as two planes, even
// and odd columns: site (x, y) at (x & 1) S L + (x >> 1) + S y, so the
// single-site loads of consecutive plaquettes are consecutive; after the
// 2 S L entries each slice buffer has kWinPad spare entries.  The row
// stride S >= L/2 puts the plaquette rows a wave reads in one pass on
// different banks (kpm_row_stride).  The thread's own four sites are never
// read back: it keeps what it published.  A thread without a plaquette
// points every index at the spare entries, so all threads run the same
// branch-free steps (its values are never stored).
constexpr int kWinPad = 4;

// Plane row stride S for rows of hL plaquettes.  LDS has 64 banks of 4
// bytes; a wave's 8-byte loads are served 32 lanes per pass, covering
// 32 / hL plaquette rows whose starts differ by 2 S elements.  With
// S = hL/2 (mod 16) those starts tile the 32 banks pairs evenly.  Rows of
// 32 or more plaquettes fill a pass alone.  (16-byte elements are served
// 16 lanes per pass, one row for hL >= 16.)
__host__ __device__ inline int kpm_row_stride(int hL) {
  if (hL % 32 == 0) return hL;
  int S = hL;
  while (S % 16 != (hL / 2) % 16) ++S;
  return S;
}

struct Win {
  int row[4];        // global row offsets L y of rows y0-1, y0, y0+1, y0+2
  int x0;
  int qa, qb;        // plaquettes above (y0-2) and below (y0+2), periodic
  int own[4];        // LDS: (x0, y0), (x0+1, y0), (x0, y0+1), (x0+1, y0+1)
  int hm[4], hp[4];  // LDS: rows y0-1 and y0+2 at columns x0-1, x0, x0+1, x0+2
  int cm[2], cp[2];  // LDS: rows y0 and y0+1 at columns x0-1 and x0+2
};

FPH_DEVINL Win make_win(const Geom& g, int q, bool own) {
  Win w;
  const int qq = own ? q : 0;
  const int x0 = 2 * (qq % g.hL), y0 = 2 * (qq / g.hL);
  const int ym = (y0 == 0) ? g.L - 1 : y0 - 1;
  const int yp = (y0 + 2 == g.L) ? 0 : y0 + 2;
  const int xm = (x0 == 0) ? g.L - 1 : x0 - 1;
  const int xp = (x0 + 2 == g.L) ? 0 : x0 + 2;
  w.x0 = x0;
  w.row[0] = g.L * ym;
  w.row[1] = g.L * y0;
  w.row[2] = g.L * (y0 + 1);
  w.row[3] = g.L * yp;
  const int nrow = g.L / 2;  // plaquette rows
  const int qy = qq / g.hL;
  w.qa = qq + g.hL * ((qy == 0) ? nrow - 1 : -1);
  w.qb = qq + g.hL * ((qy == nrow - 1) ? 1 - nrow : 1);
  const int S = kpm_row_stride(g.hL);
  const int P = S * g.L;  // plane size; the spare entries start at 2 P
  auto li = [&](int x, int y) { return own ? (x & 1) * P + (x >> 1) + S * y : 2 * P; };
  w.own[0] = li(x0, y0);
  w.own[1] = li(x0 + 1, y0);
  w.own[2] = li(x0, y0 + 1);
  w.own[3] = li(x0 + 1, y0 + 1);
  const int cols[4] = {xm, x0, x0 + 1, xp};
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    w.hm[c] = li(cols[c], ym);
    w.hp[c] = li(cols[c], yp);
  }
  w.cm[0] = li(xm, y0);
  w.cm[1] = li(xm, y0 + 1);
  w.cp[0] = li(xp, y0);
  w.cp[1] = li(xp, y0 + 1);
  if (!own) {
#pragma unroll
    for (int m = 0; m < 4; ++m) w.own[m] = 2 * P + m;
  }
  return w;
}

// Two consecutive complex values (aligned: the index is even).
FPH_DEVINL void ld2c(const float2* p, float2& a, float2& b) {
  const float4 v = *reinterpret_cast<const float4*>(p);
  a = make_float2(v.x, v.y);
  b = make_float2(v.z, v.w);
}
FPH_DEVINL void ld2c(const double2* p, double2& a, double2& b) {
  a = p[0];
  b = p[1];
}
FPH_DEVINL void st2c(float2* p, float2 a, float2 b) {
  *reinterpret_cast<float4*>(p) = make_float4(a.x, a.y, b.x, b.y);
}
FPH_DEVINL void st2c(double2* p, double2 a, double2 b) {
  p[0] = a;
  p[1] = b;
}

// The Chebyshev kernel applies the checkerboard in the primed form of the
// operator kernels (C = ch^4 P'_A P'_B, C2' = [[1, th], [th, 1]]); here
// ch^4 joins the diagonal dbar, which the recurrence applies anyway.
// Complex values stay interleaved (re, im) in registers, as in LDS.

// P'_A on the four sites of one plaquette, both components.
template <typename T2, typename T>
FPH_DEVINL void plaq_rot_c(T2 (&v)[4], T th) {
  T2 a[4];
  a[0].x = fma(th, v[1].x, v[0].x);
  a[0].y = fma(th, v[1].y, v[0].y);
  a[1].x = fma(th, v[0].x, v[1].x);
  a[1].y = fma(th, v[0].y, v[1].y);
  a[2].x = fma(th, v[3].x, v[2].x);
  a[2].y = fma(th, v[3].y, v[2].y);
  a[3].x = fma(th, v[2].x, v[3].x);
  a[3].y = fma(th, v[2].y, v[3].y);
  v[0].x = fma(th, a[2].x, a[0].x);
  v[0].y = fma(th, a[2].y, a[0].y);
  v[2].x = fma(th, a[0].x, a[2].x);
  v[2].y = fma(th, a[0].y, a[2].y);
  v[1].x = fma(th, a[3].x, a[1].x);
  v[1].y = fma(th, a[3].y, a[1].y);
  v[3].x = fma(th, a[1].x, a[3].x);
  v[3].y = fma(th, a[1].y, a[3].y);
}

// P'_B of a complex slice in LDS at the four sites of the thread's even
// plaquette, whose own published values are c: with C2' = [[1, th],
// [th, 1]] per axis,
//   out(dx, dy) = sum_{a,b} c'(1-dy, b) c'(1-dx, a) W[2dy + b][2dx + a].
template <typename T2, typename T>
FPH_DEVINL void pb_window_cn(const Win& w, const T2* __restrict__ sl, T th, const T2 (&c)[4],
                             T2 (&out)[4]) {
  const T2 a0 = sl[w.hm[0]], a1 = sl[w.hm[1]], a2 = sl[w.hm[2]], a3 = sl[w.hm[3]];
  const T2 m0 = sl[w.cm[0]], m1 = sl[w.cm[1]], p0 = sl[w.cp[0]], p1 = sl[w.cp[1]];
  const T2 b0 = sl[w.hp[0]], b1 = sl[w.hp[1]], b2 = sl[w.hp[2]], b3 = sl[w.hp[3]];
  // x-direction pairs (x0-1, x0) and (x0+1, x0+2) on each row
  T2 h0[4], h1[4];
  h0[0].x = fma(th, a0.x, a1.x);
  h0[0].y = fma(th, a0.y, a1.y);
  h1[0].x = fma(th, a3.x, a2.x);
  h1[0].y = fma(th, a3.y, a2.y);
  h0[1].x = fma(th, m0.x, c[0].x);
  h0[1].y = fma(th, m0.y, c[0].y);
  h1[1].x = fma(th, p0.x, c[1].x);
  h1[1].y = fma(th, p0.y, c[1].y);
  h0[2].x = fma(th, m1.x, c[2].x);
  h0[2].y = fma(th, m1.y, c[2].y);
  h1[2].x = fma(th, p1.x, c[3].x);
  h1[2].y = fma(th, p1.y, c[3].y);
  h0[3].x = fma(th, b0.x, b1.x);
  h0[3].y = fma(th, b0.y, b1.y);
  h1[3].x = fma(th, b3.x, b2.x);
  h1[3].y = fma(th, b3.y, b2.y);
  // y-direction pairs (y0-1, y0) and (y0+1, y0+2)
  out[0].x = fma(th, h0[0].x, h0[1].x);
  out[0].y = fma(th, h0[0].y, h0[1].y);
  out[1].x = fma(th, h1[0].x, h1[1].x);
  out[1].y = fma(th, h1[0].y, h1[1].y);
  out[2].x = fma(th, h0[3].x, h0[2].x);
  out[2].y = fma(th, h0[3].y, h0[2].y);
  out[3].x = fma(th, h1[3].x, h1[2].x);
  out[3].y = fma(th, h1[3].y, h1[2].y);
}

template <int N, typename T2>
FPH_DEVINL T2 row_ror2(T2 v) {
  T2 r;
  r.x = row_ror<N>(v.x);
  r.y = row_ror<N>(v.y);
  return r;
}

// y = C' x (TRANS = false: P'_A (P'_B x)) or C'^T x (TRANS = true:
// P'_B (P'_A x)), C = ch^4 C', for a complex vector held one even
// plaquette per thread, in two halves with one LDS exchange between them.
// Two buffers alternate between applies, so one barrier per apply
// suffices; work placed between the halves overlaps the exchange.  The
// diagonal (dbar ch^4) of Bbar is applied by the caller.
//
// Window form (any L): c_publish writes the thread's four sites (x, or
// P'_A x) into the slice buffer and returns them in c; c_finish waits at
// the barrier and forms P'_B at the thread's sites from the window and c
// (then P'_A for C').
//
// Row form (ROW16: L = 32, one plaquette row per 16-lane row of a wave,
// every lane owning a plaquette): P'_B pairs sites along x within a
// plaquette row, whose neighbours the thread takes from lanes i -/+ 1 of
// its row by DPP rotations (periodic in x as the row is).  c_publish forms
// that x half of P'_B on its own two rows and writes it (two complex values
// per row, rows y0 and y0+1 in separate arrays) and returns it in c;
// c_finish waits and combines it along y with the same values of the
// plaquettes above (their row y0-1) and below (their row y0+2): four loads
// instead of twelve, and each row's x half is formed once.  The arithmetic
// per output is the window form's, so the results are the same.
template <typename T2, typename T, bool TRANS, bool ROW16>
FPH_DEVINL void c_publish(const Win& w, const T2 (&x)[4], T2* buf, T th, T2 (&c)[4], int q,
                          int Q) {
#pragma unroll
  for (int m = 0; m < 4; ++m) c[m] = x[m];
  if (TRANS) plaq_rot_c(c, th);
  if (!ROW16) {
#pragma unroll
    for (int m = 0; m < 4; ++m) buf[w.own[m]] = c[m];
  } else {
    const T2 l1 = row_ror2<1>(c[1]), l3 = row_ror2<1>(c[3]);    // sites (x0-1, y0), (x0-1, y0+1)
    const T2 r0 = row_ror2<15>(c[0]), r2 = row_ror2<15>(c[2]);  // sites (x0+2, y0), (x0+2, y0+1)
    T2 h[4];
    h[0].x = fma(th, l1.x, c[0].x);
    h[0].y = fma(th, l1.y, c[0].y);
    h[1].x = fma(th, r0.x, c[1].x);
    h[1].y = fma(th, r0.y, c[1].y);
    h[2].x = fma(th, l3.x, c[2].x);
    h[2].y = fma(th, l3.y, c[2].y);
    h[3].x = fma(th, r2.x, c[3].x);
    h[3].y = fma(th, r2.y, c[3].y);
    st2c(buf + 2 * q, h[0], h[1]);
    st2c(buf + 2 * (Q + q), h[2], h[3]);
#pragma unroll
    for (int m = 0; m < 4; ++m) c[m] = h[m];
  }
}

template <typename T2, typename T, bool TRANS, bool ROW16>
FPH_DEVINL void c_finish(const Win& w, const T2 (&c)[4], T2 (&y)[4], const T2* buf, T th, int Q) {
  __syncthreads();
  if (!ROW16) {
    pb_window_cn(w, buf, th, c, y);
  } else {
    T2 t0, t1, b0, b1;
    ld2c(buf + 2 * (Q + w.qa), t0, t1);  // row y0-1: the plaquette above's second row
    ld2c(buf + 2 * w.qb, b0, b1);        // row y0+2: the plaquette below's first row
    y[0].x = fma(th, t0.x, c[0].x);
    y[0].y = fma(th, t0.y, c[0].y);
    y[1].x = fma(th, t1.x, c[1].x);
    y[1].y = fma(th, t1.y, c[1].y);
    y[2].x = fma(th, b0.x, c[2].x);
    y[2].y = fma(th, b0.y, c[2].y);
    y[3].x = fma(th, b1.x, c[3].x);
    y[3].y = fma(th, b1.y, c[3].y);
  }
  if (!TRANS) plaq_rot_c(y, th);
}

// acc = sum_{m < NP} c'_m T_m(A') x with A' = A (TRANS false, c' = c) or
// A' = A^T (TRANS true, c' = conj(c)), A = sA D C' - cA, D = diag(dbar ch^4)
// (db holds its entries); three-term recurrence of Eq. alpha_recur,
//   alpha_m = 2 sA D (C' alpha_{m-1}) - 2 cA alpha_{m-1} - alpha_{m-2},
// with D folded into the fused multiply-add that forms alpha_m.  For A^T
// the recurrence runs on beta_m = D alpha_m, which obeys the same
// relation with C'^T in place of C' (D A^T D^{-1} = sA D C'^T - cA):
// beta_0 = D x, and the sum is scaled by D^{-1} at the end.  Each new term
// is published for the next apply before it is added to the sum, and each
// coefficient is read one step ahead, after a barrier, beside the
// neighbours' values: read just before a barrier its latency would add to
// the barrier's wait, and read in its own step its wait would come before
// the sum that overlaps the publishing stores.  So neither sits on the
// path from one exchange to the next.  Exchange j of the series uses LDS buffer
// (j - 1) mod 2, fixed per step of the unrolled loop; a series always
// starts on buffer 0.  The two latest terms alternate between two register
// sets, so no copies are made.
template <typename T, bool TRANS, bool ROW16>
FPH_DEVINL void cheb_series(const Win& w, int NP, const typename Cplx<T>::type* cf, T sA, T cA,
                            const typename Cplx<T>::type (&x)[4], const T (&db)[4],
                            typename Cplx<T>::type* buf0, typename Cplx<T>::type* buf1, T th,
                            typename Cplx<T>::type (&acc)[4], int qid, int Q) {
  using T2 = typename Cplx<T>::type;
  const T cj = TRANS ? (T)-1 : (T)1;
  auto accumulate = [&](const T2 c, const T2 (&v)[4]) {
    const T cy = cj * c.y;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      acc[q].x = fma(-cy, v[q].y, fma(c.x, v[q].x, acc[q].x));
      acc[q].y = fma(cy, v[q].x, fma(c.x, v[q].y, acc[q].y));
    }
  };
  // rec: v = fma(d2, y, -c2 u - v), the next term from C' u (in y), u, v
  auto rec = [&](T2 (&v)[4], const T2 (&u)[4], const T2 (&y)[4], const T (&d2)[4], T c2) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      v[q].x = fma(d2[q], y[q].x, fma(-c2, u[q].x, -v[q].x));
      v[q].y = fma(d2[q], y[q].y, fma(-c2, u[q].y, -v[q].y));
    }
  };
  T2 p[4], q[4], y[4], c_[4];  // p = alpha_{m-2}, q = alpha_{m-1}; c_: last published
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    acc[k].x = acc[k].y = (T)0;
    p[k].x = TRANS ? db[k] * x[k].x : x[k].x;
    p[k].y = TRANS ? db[k] * x[k].y : x[k].y;
  }
  if (NP >= 2) c_publish<T2, T, TRANS, ROW16>(w, p, buf0, th, c_, qid, Q);
  accumulate(cf[0], p);
  if (NP >= 2) {
    T sdb[4], db2[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      sdb[k] = sA * db[k];
      db2[k] = (T)2 * sdb[k];
    }
    T2 c = cf[1];
    c_finish<T2, T, TRANS, ROW16>(w, c_, y, buf0, th, Q);
    T2 cn = cf[min(2, NP - 1)];  // the next step's, read beside this step's values
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      q[k].x = fma(sdb[k], y[k].x, -cA * p[k].x);
      q[k].y = fma(sdb[k], y[k].y, -cA * p[k].y);
    }
    if (NP > 2) c_publish<T2, T, TRANS, ROW16>(w, q, buf1, th, c_, qid, Q);
    accumulate(c, q);
    const T c2 = (T)2 * cA;
    for (int m = 2; m < NP; m += 2) {
      c_finish<T2, T, TRANS, ROW16>(w, c_, y, buf1, th, Q);
      c = cn;
      cn = cf[min(m + 1, NP - 1)];
      rec(p, q, y, db2, c2);
      if (m + 1 < NP) c_publish<T2, T, TRANS, ROW16>(w, p, buf0, th, c_, qid, Q);
      accumulate(c, p);
      if (m + 1 >= NP) break;
      c_finish<T2, T, TRANS, ROW16>(w, c_, y, buf0, th, Q);
      c = cn;
      cn = cf[min(m + 2, NP - 1)];
      rec(q, p, y, db2, c2);
      if (m + 2 < NP) c_publish<T2, T, TRANS, ROW16>(w, q, buf1, th, c_, qid, Q);
      accumulate(c, q);
    }
    // A following series first writes buffer 0; after an odd number of
    // exchanges the last one read buffer 0, so every thread must be past it.
    if ((NP - 1) & 1) __syncthreads();
  }
  if (TRANS) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const T inv = (T)1 / db[k];
      acc[k].x *= inv;
      acc[k].y *= inv;
    }
  }
}

// The window-form series on one real part of the block vector, for the
// 1 024-thread FP64 blocks, whose 128 registers per thread do not hold the
// complex recurrence without spilling.  A = sA D C' - cA is real, so the
// recurrence of cheb_series runs on the real part (part 0) and on the
// imaginary part (part 1) of the input separately; each part adds its
// terms to the complex sum times c_m (conjugated for TRANS) and times 1 or
// i.  sdb holds sA D.  The caller zeroes acc before the first part and,
// for TRANS, scales by D^-1 after the second.  The thread's published
// values are read back from LDS and 2 sA D is applied as two fused
// multiply-adds, both to save registers.
template <typename T, bool TRANS>
FPH_DEVINL void cheb_series_part(const Win& w, int NP, const typename Cplx<T>::type* cf, T sA,
                                 T cA, const T (&x)[4], const T (&sdb)[4], T* buf0, T* buf1, T th,
                                 typename Cplx<T>::type (&acc)[4], int part) {
  using T2 = typename Cplx<T>::type;
  const T cj = TRANS ? (T)-1 : (T)1;
  // The window's sixteen LDS indices from five values and the plane and
  // row strides P, S (uniform): own sites B + {0, P, S, P + S}; columns
  // x0 - 1 and x0 + 2 at row y0 from Cm and Cp; rows y0 - 1 and y0 + 2 are
  // row y0 shifted by Rm and Rp (periodic).
  const int B = w.own[0], Pp = w.own[1] - w.own[0], S = w.own[2] - w.own[0];
  const int Cm = w.cm[0], Cp = w.cp[0];
  const int Rm = w.hm[1] - B, Rp = w.hp[1] - B;
  auto accumulate = [&](const T2 c, const T (&v)[4]) {
    const T cr = c.x, ci = cj * c.y;
    const T ax = part ? -ci : cr, ay = part ? cr : ci;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      acc[q].x = fma(ax, v[q], acc[q].x);
      acc[q].y = fma(ay, v[q], acc[q].y);
    }
  };
  auto publish = [&](const T (&v)[4], T* buf) {
    T c[4] = {v[0], v[1], v[2], v[3]};
    if (TRANS) plaq_rot(c, th);
    buf[B] = c[0];
    buf[B + Pp] = c[1];
    buf[B + S] = c[2];
    buf[B + Pp + S] = c[3];
  };
  // y = C' v (C'^T v) from the published slice: P'_B at the thread's sites
  // from the 4x4 window (own values read back), then P'_A for C'.
  auto finish = [&](T (&y)[4], const T* sl) {
    __syncthreads();
    const T c[4] = {sl[B], sl[B + Pp], sl[B + S], sl[B + Pp + S]};
    const T a0 = sl[Cm + Rm], a1 = sl[B + Rm], a2 = sl[B + Pp + Rm], a3 = sl[Cp + Rm];
    const T m0 = sl[Cm], m1 = sl[Cm + S], p0 = sl[Cp], p1 = sl[Cp + S];
    const T b0 = sl[Cm + Rp], b1 = sl[B + Rp], b2 = sl[B + Pp + Rp], b3 = sl[Cp + Rp];
    const T h00 = fma(th, a0, a1), h10 = fma(th, a3, a2);
    const T h01 = fma(th, m0, c[0]), h11 = fma(th, p0, c[1]);
    const T h02 = fma(th, m1, c[2]), h12 = fma(th, p1, c[3]);
    const T h03 = fma(th, b0, b1), h13 = fma(th, b3, b2);
    y[0] = fma(th, h00, h01);
    y[1] = fma(th, h10, h11);
    y[2] = fma(th, h03, h02);
    y[3] = fma(th, h13, h12);
    if (!TRANS) plaq_rot(y, th);
  };
  const T c2 = (T)2 * cA;
  // v = 2 sA D y - c2 u - v
  auto rec = [&](T (&v)[4], const T (&u)[4], const T (&y)[4]) {
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = fma(sdb[k], y[k], fma(sdb[k], y[k], fma(-c2, u[k], -v[k])));
  };
  T p[4], q[4], y[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) p[k] = TRANS ? (sdb[k] / sA) * x[k] : x[k];
  if (NP >= 2) publish(p, buf0);
  accumulate(cf[0], p);
  if (NP < 2) return;
  T2 c = cf[1];
  finish(y, buf0);
  T2 cn = cf[min(2, NP - 1)];  // one step ahead, as in cheb_series
#pragma unroll
  for (int k = 0; k < 4; ++k) q[k] = fma(sdb[k], y[k], -cA * p[k]);
  if (NP > 2) publish(q, buf1);
  accumulate(c, q);
  for (int m = 2; m < NP; m += 2) {
    finish(y, buf1);
    c = cn;
    cn = cf[min(m + 1, NP - 1)];
    rec(p, q, y);
    if (m + 1 < NP) publish(p, buf0);
    accumulate(c, p);
    if (m + 1 >= NP) break;
    finish(y, buf0);
    c = cn;
    cn = cf[min(m + 2, NP - 1)];
    rec(q, p, y);
    if (m + 2 < NP) publish(q, buf1);
    accumulate(c, q);
  }
  // A following series first writes buffer 0; after an odd number of
  // exchanges the last one read buffer 0, so every thread must be past it.
  if ((NP - 1) & 1) __syncthreads();
}

// Per-block Chebyshev apply.  op 0: F (series in A), 1: F^T (conjugate
// series in A^T), 2: F F^T (conjugate series, then series).  Block b
// serves frequency order b / nrhs (longest series first: k = 0, H-1, 1,
// H-2, ...) and right-hand side b % nrhs; one even plaquette per thread
// (NT >= Q).  LDS: two complex slice buffers (2 S L + kWinPad values each)
// and the block's Chebyshev coefficients.
template <typename T, int NT, bool ROW16>
__global__ void __launch_bounds__(NT)
k_kpm(Geom g, int H, int nrhs, int op, const PcInfo* __restrict__ info,
      const int* __restrict__ np, const typename Cplx<T>::type* __restrict__ coef,
      const T* __restrict__ dbar, T th, T c4, const typename Cplx<T>::type* __restrict__ Z,
      typename Cplx<T>::type* __restrict__ Zo, StIO io) {
  using T2 = typename Cplx<T>::type;
  static_assert(NT <= kNPMax, "one coefficient per thread is loaded ahead");
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ RhsState s_sh;
  const int nbuf = 2 * kpm_row_stride(g.hL) * g.L + kWinPad;
  T2* buf0 = reinterpret_cast<T2*>(smem_raw);
  T2* buf1 = buf0 + nbuf;
  T2* cfs = buf1 + nbuf;  // coefficients of this block's frequency
  const int ko = blockIdx.x / nrhs;
  const int r = blockIdx.x % nrhs;
  const int k = (ko % 2 == 0) ? ko / 2 : H - 1 - ko / 2;
  const int q = threadIdx.x;
  const bool own = q < g.Q;
  const Win w = make_win(g, q, own);
  const int i0 = w.x0 + w.row[1], iL = i0 + g.L;

  // The series depends on no scalar of the CG, so inside a solve only one
  // block per right-hand side reads the solver state: the one with the
  // shortest series (the last of the longest-first order), which folds the
  // pending |r|^2 and writes the state for the next kernel.  The other
  // blocks never wait for the state; for a right-hand side that has
  // finished or paused they compute a transform the next kernel ignores.
  // The reading block issues the state loads first and folds them between
  // the conjugate series and the series of F F^T, where they have long
  // arrived (a right-hand side found finished or paused there skips the
  // second series); only F or F^T alone folds before the series.  (The
  // 1024-thread blocks have no registers to spare: they read the state
  // after the block's input, as one step.)
  constexpr bool kIssueFirst = NT < 1024;
  const bool stt = io.in != nullptr && ko == H - 1;
  StLoad<4> sl;
  if (kIssueFirst && stt) state_issue(io, r, sl);
  const int f = field_of(g, r);
  info += f;
  np += (long)f * g.Ltau;
  coef += (long)f * H * kNPMax;
  dbar += (long)f * g.N;
  const int NP = np[2 * k];
  const T sA = (T)info->s, cA = (T)info->c;
  const T2 c_first = coef[(long)k * kNPMax + threadIdx.x];
  T2 x[4], acc[4];
  T db[4];
  const T2* Zin = Z + ((long)r * H + k) * g.N;
  // Unconditional loads (a thread without a plaquette reads plaquette 0's
  // values, which only its spare LDS entry ever sees, and stores nothing),
  // so that no load waits for the ones before it.
  ld2c(Zin + i0, x[0], x[1]);
  ld2c(Zin + iL, x[2], x[3]);
  db[0] = c4 * dbar[i0]; db[1] = c4 * dbar[i0 + 1];
  db[2] = c4 * dbar[iL]; db[3] = c4 * dbar[iL + 1];
  const bool late = kIssueFirst && stt && op == 2;
  if (stt && !late) {
    if constexpr (kIssueFirst)
      state_finish<NT>(io, r, sl, &s_sh);
    else
      state_begin<NT>(io, r, &s_sh, nullptr);
    if (s_sh.done) {
      state_end(io, r, &s_sh, P_NONE, 0.0, 0, 1, true);
      return;
    }
  }
  if ((int)threadIdx.x < NP) cfs[threadIdx.x] = c_first;
  for (int m = threadIdx.x + NT; m < NP; m += NT) cfs[m] = coef[(long)k * kNPMax + m];
  __syncthreads();
  // FP64 in 1 024-thread blocks: the series one real part at a time.
  constexpr bool kParts = sizeof(T) == 8 && NT >= 1024 && !ROW16;
  T* rb0 = reinterpret_cast<T*>(buf0);
  T* rb1 = reinterpret_cast<T*>(buf1);
  auto series = [&](auto trans_tag) {
    constexpr bool TR = decltype(trans_tag)::value;
    if constexpr (kParts) {
      // The imaginary part waits in the unused upper half of buffer 0
      // (the real-valued exchanges use its first nbuf values) while the
      // real part's series runs; each thread reads back what it wrote.
      T* stash = rb0 + nbuf;
      T xp[4], sdb[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        xp[m] = x[m].x;
        stash[w.own[m]] = x[m].y;
        acc[m].x = acc[m].y = (T)0;
        sdb[m] = sA * db[m];
      }
      cheb_series_part<T, TR>(w, NP, cfs, sA, cA, xp, sdb, rb0, rb1, th, acc, 0);
#pragma unroll
      for (int m = 0; m < 4; ++m) xp[m] = stash[w.own[m]];
      cheb_series_part<T, TR>(w, NP, cfs, sA, cA, xp, sdb, rb0, rb1, th, acc, 1);
      if (TR) {
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          const T inv = sA / sdb[m];  // D^-1
          acc[m].x *= inv;
          acc[m].y *= inv;
        }
      }
    } else {
      cheb_series<T, TR, ROW16>(w, NP, cfs, sA, cA, x, db, buf0, buf1, th, acc, q, g.Q);
    }
  };
  if (op == 0) {
    series(std::false_type{});
  } else {
    series(std::true_type{});
    if (op == 2) {
      if (late) {
        state_finish<NT>(io, r, sl, &s_sh);
        if (s_sh.done) {
          state_end(io, r, &s_sh, P_NONE, 0.0, 0, 1, true);
          return;
        }
      }
#pragma unroll
      for (int m = 0; m < 4; ++m) x[m] = acc[m];
      series(std::false_type{});
    }
  }
  if (own) {
    T2* Zout = Zo + ((long)r * H + k) * g.N;
    st2c(Zout + i0, acc[0], acc[1]);
    st2c(Zout + iL, acc[2], acc[3]);
  }
  if (stt) state_end(io, r, &s_sh, P_NONE, 0.0, 0, 1, true);
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
  const int nF = pc->H1 * pc->H1 + pc->H2 * pc->H2;
  PCALLOC(pc->tw64, H * sizeof(double2));
  PCALLOC(pc->W64, H * sizeof(double2));
  PCALLOC(pc->F64, nF * sizeof(double2));
  PCALLOC(pc->tw32, H * sizeof(float2));
  PCALLOC(pc->W32, H * sizeof(float2));
  PCALLOC(pc->F32, nF * sizeof(float2));
  // one set of series tables per field (up to max_rhs fields)
  PCALLOC(pc->info, (size_t)max_rhs * sizeof(PcInfo));
  PCALLOC(pc->np, (size_t)max_rhs * g.Ltau * sizeof(int));
  PCALLOC(pc->coef64, (size_t)max_rhs * H * kNPMax * sizeof(double2));
  PCALLOC(pc->coef32, (size_t)max_rhs * H * kNPMax * sizeof(float2));
  PCALLOC(pc->Z, (size_t)max_rhs * H * g.N * sizeof(double2));
  PCALLOC(pc->Z2, (size_t)max_rhs * H * g.N * sizeof(double2));
#undef PCALLOC
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_pc_twiddles, dim3((H + nF + 255) / 256), dim3(256), 0, 0, H, pc->H1,
                     pc->H2, g.Ltau, pc->tw64, pc->W64, pc->F64, pc->tw32, pc->W32, pc->F32);
  return hipGetLastError();
}

inline void pc_destroy(PcTables* pc) {
  void* ptrs[] = {pc->tw64, pc->W64, pc->F64, pc->tw32, pc->W32, pc->F32, pc->info, pc->np,
                  pc->coef64, pc->coef32, pc->Z, pc->Z2};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  std::memset(pc, 0, sizeof(*pc));
}

// Series tables of field f from its dbar (dbar64 points at that field's N values).
inline hipError_t pc_set_field(PcTables* pc, const Geom& g, const double* dbar64, double dtau,
                               double t, double a1, double a2, hipStream_t s, int f = 0) {
  PcInfo* info = pc->info + f;
  int* np = pc->np + (long)f * g.Ltau;
  hipLaunchKernelGGL(k_pc_bounds, dim3(1), dim3(256), 0, s, g.N, g.Ltau, dbar64, dtau, t, a1, a2,
                     info, np);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_pc_coef, dim3(pc->H), dim3(256), 0, s, g.Ltau, (const PcInfo*)info,
                     (const int*)np, pc->coef64 + (long)f * pc->H * kNPMax,
                     pc->coef32 + (long)f * pc->H * kNPMax);
  return hipGetLastError();
}

// LDS bytes of a transform workgroup with tile width 2^lks.
template <typename T>
size_t pc_tile_lds(const PcTables* pc, int lks) {
  const size_t nF = (size_t)pc->H1 * pc->H1 + (size_t)pc->H2 * pc->H2;
  return (nF + pc->H + 2 * (size_t)pc->H * ((size_t)1 << lks)) * sizeof(typename Cplx<T>::type);
}

// Tile width (log2) of the transforms, for workgroups of kTNT threads:
// the widest tile up to 8 sites that leaves at least 256 tiles (each slice
// row of a tile is a separate short segment, so narrow tiles cost more
// cache lines per byte; wide ones leave CUs idle), not below 2 sites, and
// at most 64 KB of LDS per workgroup.  (At L = 64 FP64 tiles of 4 sites
// would make 1 024 workgroups, two rounds at the two workgroups of this
// kernel a CU holds; 8 sites make one.)
constexpr int kTNT = 512;

template <typename T>
int pc_tile_log2(const PcTables* pc, const Geom& g, int nrhs) {
  int lks = 3;
  while (lks > 1 && (long)((g.N + (1 << lks) - 1) >> lks) * nrhs < 256) --lks;
  while (lks > 0 && pc_tile_lds<T>(pc, lks) > ((size_t)64 << 10)) --lks;
  return lks;
}

template <typename T, int H1, int NT>
hipError_t pc_launch_fwd(const PcTables* pc, const Geom& g, int nrhs, int lks, T* in,
                         typename Cplx<T>::type* Z, T* u, const T* pa, const T* pb, const T* Ap,
                         StateSeq& sq, bool cgupd, hipStream_t s) {
  const int KS = 1 << lks;
  const int ntiles = (g.N + KS - 1) / KS;
  if (pc->H1 * pc->H1 + pc->H2 * pc->H2 + pc->H > 6 * NT) return hipErrorInvalidValue;
  const StIO io = sq.next();
  const size_t lds = pc_tile_lds<T>(pc, lks);
  using T2 = typename Cplx<T>::type;
  const auto* tw = (const T2*)(sizeof(T) == 8 ? (const void*)pc->tw64 : (const void*)pc->tw32);
  const auto* W = (const T2*)(sizeof(T) == 8 ? (const void*)pc->W64 : (const void*)pc->W32);
  const auto* F = (const T2*)(sizeof(T) == 8 ? (const void*)pc->F64 : (const void*)pc->F32);
  dim3 grid(ntiles * nrhs);
  // FP32: four stage-0 items per thread where two would need a second
  // pass (FP64 keeps two: its registers would cost occupancy).
  const bool wide = sizeof(T) == 4 && (pc->H << lks) > 2 * NT;
  auto kern = cgupd ? k_tfwd<T, H1, NT, true, 2> : k_tfwd<T, H1, NT, false, 2>;
  if constexpr (sizeof(T) == 4) {
    if (wide) kern = cgupd ? k_tfwd<T, H1, NT, true, 4> : k_tfwd<T, H1, NT, false, 4>;
  }
  hipError_t e = allow_lds((const void*)kern, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, grid, dim3(NT), lds, s, g, pc->H2, tw, W, F, in, Z, u, pa, pb, Ap, lks,
                     ntiles, io);
  return hipGetLastError();
}

template <typename T, int H1, int NT>
hipError_t pc_launch_inv(const PcTables* pc, const Geom& g, int nrhs, int lks,
                         const typename Cplx<T>::type* Zh, T* out, int dot, const T* rdot,
                         StateSeq& sq, hipStream_t s) {
  const int KS = 1 << lks;
  const int ntiles = (g.N + KS - 1) / KS;
  const StIO io = sq.next();
  const size_t lds = pc_tile_lds<T>(pc, lks);
  using T2 = typename Cplx<T>::type;
  const auto* tw = (const T2*)(sizeof(T) == 8 ? (const void*)pc->tw64 : (const void*)pc->tw32);
  const auto* W = (const T2*)(sizeof(T) == 8 ? (const void*)pc->W64 : (const void*)pc->W32);
  const auto* F = (const T2*)(sizeof(T) == 8 ? (const void*)pc->F64 : (const void*)pc->F32);
  auto kern = k_tinv<T, H1, NT, 4>;
  if constexpr (sizeof(T) == 4) {
    if ((pc->H << lks) <= 2 * NT) kern = k_tinv<T, H1, NT, 2>;
  }
  hipError_t e = allow_lds((const void*)kern, lds);
  if (e != hipSuccess) return e;
  // Without r.z the kernel still loads (and ignores) rdot: it then reads
  // the input, which holds at least as many values.
  const T* rd = dot ? rdot : reinterpret_cast<const T*>(Zh);
  hipLaunchKernelGGL(kern, dim3(ntiles * nrhs), dim3(NT), lds, s, g, pc->H2, tw, W, F, Zh, out,
                     dot, rd, lks, ntiles, io);
  return hipGetLastError();
}

template <typename T>
hipError_t pc_fwd(const PcTables* pc, const Geom& g, int nrhs, T* in, typename Cplx<T>::type* Z,
                  T* u, const T* pa, const T* pb, const T* Ap, StateSeq& sq, bool cgupd,
                  hipStream_t s) {
  const int lks = pc_tile_log2<T>(pc, g, nrhs);
  switch (pc->H1) {
#define FPH_FWD_CASE(h1) \
  case h1: return pc_launch_fwd<T, h1, kTNT>(pc, g, nrhs, lks, in, Z, u, pa, pb, Ap, sq, cgupd, s);
    FPH_FWD_CASE(1) FPH_FWD_CASE(2) FPH_FWD_CASE(3) FPH_FWD_CASE(4) FPH_FWD_CASE(5)
    FPH_FWD_CASE(8) FPH_FWD_CASE(10) FPH_FWD_CASE(16) FPH_FWD_CASE(20)
#undef FPH_FWD_CASE
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t pc_inv(const PcTables* pc, const Geom& g, int nrhs, const typename Cplx<T>::type* Zh,
                  T* out, int dot, const T* rdot, StateSeq& sq, hipStream_t s) {
  const int lks = pc_tile_log2<T>(pc, g, nrhs);
  switch (pc->H1) {
#define FPH_INV_CASE(h1) \
  case h1: return pc_launch_inv<T, h1, kTNT>(pc, g, nrhs, lks, Zh, out, dot, rdot, sq, s);
    FPH_INV_CASE(1) FPH_INV_CASE(2) FPH_INV_CASE(3) FPH_INV_CASE(4) FPH_INV_CASE(5)
    FPH_INV_CASE(8) FPH_INV_CASE(10) FPH_INV_CASE(16) FPH_INV_CASE(20)
#undef FPH_INV_CASE
    default: return hipErrorInvalidValue;
  }
}

template <typename T, int NT, bool ROW16 = false>
hipError_t pc_launch_kpm(const PcTables* pc, const Geom& g, const T* dbar, int op, int nrhs,
                         const typename Cplx<T>::type* Z, typename Cplx<T>::type* Zo,
                         StateSeq& sq, T th, T c4, hipStream_t s) {
  const StIO io = sq.next();
  const size_t nbuf = 2 * (size_t)kpm_row_stride(g.hL) * g.L + kWinPad;
  const size_t lds = (2 * nbuf + kNPMax) * sizeof(typename Cplx<T>::type);
  auto kern = k_kpm<T, NT, ROW16>;
  hipError_t e = allow_lds((const void*)kern, lds);
  if (e != hipSuccess) return e;
  const auto* cf = (const typename Cplx<T>::type*)(sizeof(T) == 8 ? (const void*)pc->coef64 : (const void*)pc->coef32);
  hipLaunchKernelGGL(kern, dim3(pc->H * nrhs), dim3(NT), lds, s, g, pc->H, nrhs, op, pc->info,
                     pc->np, cf, dbar, th, c4, Z, Zo, io);
  return hipGetLastError();
}

template <typename T>
hipError_t pc_kpm(const PcTables* pc, const Geom& g, const T* dbar, int op, int nrhs,
                  const typename Cplx<T>::type* Z, typename Cplx<T>::type* Zo, StateSeq& sq,
                  T th, T c4, hipStream_t s) {
  // L = 32: each plaquette row is one 16-lane row of a wave (row form).
  if (g.hL == 16 && g.Q == 256)
    return pc_launch_kpm<T, 256, true>(pc, g, dbar, op, nrhs, Z, Zo, sq, th, c4, s);
  if (g.Q <= 64) return pc_launch_kpm<T, 64>(pc, g, dbar, op, nrhs, Z, Zo, sq, th, c4, s);
  if (g.Q <= 256) return pc_launch_kpm<T, 256>(pc, g, dbar, op, nrhs, Z, Zo, sq, th, c4, s);
  if (g.Q <= 512) return pc_launch_kpm<T, 512>(pc, g, dbar, op, nrhs, Z, Zo, sq, th, c4, s);
  return pc_launch_kpm<T, 1024>(pc, g, dbar, op, nrhs, Z, Zo, sq, th, c4, s);
}

// out = op(in) (op: 0 F, 1 F^T, 2 F F^T).  With rdot != nullptr the inverse
// transform also publishes rdot . out as P_RZ partials.
template <typename T>
hipError_t pc_apply(const PcTables* pc, const Geom& g, const T* dbar, int op, int nrhs,
                    const T* in, T* out, const T* rdot, StateSeq& sq, hipStream_t s) {
  using T2 = typename Cplx<T>::type;
  T2* Z = reinterpret_cast<T2*>(pc->Z);
  T2* Z2 = reinterpret_cast<T2*>(pc->Z2);
  hipError_t e = pc_fwd<T>(pc, g, nrhs, const_cast<T*>(in), Z, nullptr, nullptr, nullptr,
                           nullptr, sq, false, s);
  if (e != hipSuccess) return e;
  e = pc_kpm<T>(pc, g, dbar, op, nrhs, Z, Z2, sq, (T)pc->th, (T)pc->c4, s);
  if (e != hipSuccess) return e;
  return pc_inv<T>(pc, g, nrhs, Z2, out, rdot ? 1 : 0, rdot, sq, s);
}

// Preconditioned CG update: u += alpha p, r -= alpha Ap (|r|^2 as P_RR),
// then z = F F^T r (the KPM kernel folds P_RR and skips finished
// right-hand sides) and r.z as P_RZ.  Three launches.
template <typename T>
hipError_t pc_cg_update(const PcTables* pc, const Geom& g, const T* dbar, int nrhs, T* u,
                        const T* pa, const T* pb, T* r, const T* Ap, T* z, StateSeq& sq,
                        hipStream_t s) {
  using T2 = typename Cplx<T>::type;
  T2* Z = reinterpret_cast<T2*>(pc->Z);
  T2* Z2 = reinterpret_cast<T2*>(pc->Z2);
  hipError_t e = pc_fwd<T>(pc, g, nrhs, r, Z, u, pa, pb, Ap, sq, true, s);
  if (e != hipSuccess) return e;
  e = pc_kpm<T>(pc, g, dbar, 2, nrhs, Z, Z2, sq, (T)pc->th, (T)pc->c4, s);
  if (e != hipSuccess) return e;
  return pc_inv<T>(pc, g, nrhs, Z2, z, 1, r, sq, s);
}

}  // namespace fph
