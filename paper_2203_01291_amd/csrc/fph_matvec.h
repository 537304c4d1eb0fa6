// Operator kernels: M, M^T, fused M^T M and the phonon force.
//
// (M v)_tau   = v_tau - E_tau * (C v~_{tau-1}),      v~_{-1} = -v_{Ltau-1}
// (M^T w)_tau = w_tau - C^T (E_{tau+1} * w~_{tau+1}), w~_{Ltau} = -w_0
// (Eq. M_def of the paper; B_tau = diag(E_tau) C, Eq. B_def.)
//
// Fused M^T M over a chunk of consecutive slices [tau0, tau0 + Tc): step j
// (tau = tau0 + j, j = 0..Tc) forms w_tau = (M v)_tau in registers and, for
// j >= 1, emits out_{tau-1} = w_{tau-1} - C^T (E_tau w_tau).  Per step:
//   a) load v~_{tau-1} on odd plaquettes, apply P_B, write LDS  | barrier
//   b) read even plaquettes, apply P_A, w = v_tau - E_tau (.);
//      y = P_A (E_tau w) -> LDS (in place), w -> LDS            | barrier
//   c) read odd plaquettes of y, apply P_B: out = w_{tau-1} - P_B y;
//      keep w_tau on the odd plaquettes for the next step.
// Each thread reads and writes only its own plaquette's sites between
// barriers where no other thread can touch them, so two barriers per step
// suffice and LDS holds two slices per chunk.  Only v, E and out touch
// global memory: 3 vectors per application for one right-hand side.
#pragma once

#include "fph_common.h"

namespace fph {

// ------------------------------------------------------- input functors --

// v read directly.
template <typename T>
struct InPlain {
  const T* __restrict__ v;
  FPH_DEVINL void begin(int, const RhsState*) {}
  FPH_DEVINL T load(long off) const { return v[off]; }
  FPH_DEVINL void store_owned(long, T) const {}
};

// p = z + beta p_old computed on the fly (the CG direction update fused
// into the operator); the chunk owner stores p for its own slices.  The
// two direction buffers alternate with the parity of the right-hand side's
// own iteration count, so a paused right-hand side keeps a consistent pair.
template <typename T>
struct InPUpdate {
  const T* __restrict__ z;
  T* pa;
  T* pb;
  const T* __restrict__ pold;
  T* __restrict__ pnew;
  T beta;
  int fresh;
  FPH_DEVINL void begin(int r, const RhsState* st) {
    fresh = st[r].fresh;
    beta = (T)st[r].beta;
    const bool odd = (st[r].iter & 1) != 0;
    pold = odd ? pb : pa;
    pnew = odd ? pa : pb;
  }
  FPH_DEVINL T load(long off) const { return fresh ? z[off] : z[off] + beta * pold[off]; }
  FPH_DEVINL void store_owned(long off, T val) const { pnew[off] = val; }
};

// ---------------------------------------------------- epilogue functors --

// Plain store of out.
template <typename T>
struct EpiStore {
  T* __restrict__ out;
  FPH_DEVINL void begin(int, const RhsState*) {}
  FPH_DEVINL void put(long off, T o, T /*v*/, double& /*acc*/) const { out[off] = o; }
  FPH_DEVINL void finish(RhsState&, double) const {}
  static constexpr bool kReduce = false;
};

// Store out = A p and accumulate p . A p; the last block sets
// alpha = rz / pAp (CG step length).
template <typename T>
struct EpiDotAlpha {
  T* __restrict__ out;
  FPH_DEVINL void begin(int, const RhsState*) {}
  FPH_DEVINL void put(long off, T o, T v, double& acc) const {
    out[off] = o;
    acc += (double)v * (double)o;
  }
  FPH_DEVINL void finish(RhsState& s, double pAp) const {
    s.pAp = pAp;
    s.matvecs += 1;
    if (!(pAp > 0.0) || !isfinite(pAp)) {
      s.status |= isfinite(pAp) ? 4 : 8;  // BREAKDOWN / NONFINITE
      s.done = 1;
      s.alpha = 0.0;
    } else {
      s.alpha = s.rz / pAp;
    }
  }
  static constexpr bool kReduce = true;
};

// True residual r = b - A u in FP64, stored as TR (float or double);
// accumulates |r|^2 (of the stored values) and |b - Au|^2 in FP64.
template <typename TR>
struct EpiResidual {
  const double* __restrict__ b;
  TR* __restrict__ r;
  FPH_DEVINL void begin(int, const RhsState*) {}
  FPH_DEVINL void put(long off, double o, double /*v*/, double& acc) const {
    const double res = b[off] - o;
    r[off] = (TR)res;
    acc += res * res;
  }
  FPH_DEVINL void finish(RhsState& s, double rr) const {
    s.rr_true = rr;
    s.matvecs += 1;
  }
  static constexpr bool kReduce = true;
};

// ------------------------------------------------------ fused M^T M ------

// Launch: grid (nblk, nrhs).  Block b of right-hand side r serves `S`
// chunks of `Tch` slices each; with Q <= NT plaquettes per slice, S = NT/Q
// chunks run side by side (one plaquette per thread), otherwise S = 1 and a
// thread serves up to MAXSLOT plaquettes.  LDS: 2 * S * N elements of T.
template <typename T, int NT, int MAXSLOT, class In, class Epi>
__global__ void __launch_bounds__(NT)
k_mtm(Geom g, const T* __restrict__ E, T ch, T sh, int Tch, In in, Epi epi,
      RhsState* st, double* partial, unsigned* counter) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red_sh[NT / 64];
  __shared__ int flag_sh;
  const int r = blockIdx.y;
  if (st != nullptr && st[r].done) return;

  const int tid = threadIdx.x;
  int S, sub, lane, nslot;
  if (g.Q <= NT) {
    S = NT / g.Q;
    sub = tid / g.Q;
    lane = tid - sub * g.Q;
    nslot = 1;
  } else {
    S = 1;
    sub = 0;
    lane = tid;
    nslot = (g.Q + NT - 1) / NT;
  }
  const int chunk = blockIdx.x * S + sub;
  const int tau0 = chunk * Tch;
  const bool active = (sub < S) && (tau0 < g.Ltau);
  const int Tc = active ? min(Tch, g.Ltau - tau0) : 0;

  T* buf = reinterpret_cast<T*>(smem_raw) + (long)(sub < S ? sub : 0) * g.N;
  T* wbuf = reinterpret_cast<T*>(smem_raw) + (long)S * g.N + (long)(sub < S ? sub : 0) * g.N;

  in.begin(r, st);
  epi.begin(r, st);
  const long base = (long)r * g.d;
  double acc = 0.0;

  T wprev[MAXSLOT][4];
  T vodd[MAXSLOT][4];

  for (int j = 0; j <= Tch; ++j) {
    const int tau = tau0 + j;
    const bool act = active && (j <= Tc);
    const int tm = (tau >= g.Ltau) ? tau - g.Ltau : tau;
    // (a) v~_{tau-1} on odd plaquettes -> P_B -> LDS
    if (act) {
      int pt = tm - 1;
      T psg = (T)1;
      if (pt < 0) {
        pt = g.Ltau - 1;
        psg = (T)-1;
      }
      const long poff = base + (long)pt * g.N;
#pragma unroll
      for (int k = 0; k < MAXSLOT; ++k) {
        const int q = lane + k * NT;
        if (k < nslot && q < g.Q) {
          int s[4];
          odd_sites(g, q, s);
          T t[4];
#pragma unroll
          for (int m = 0; m < 4; ++m) {
            const T val = in.load(poff + s[m]);
            vodd[k][m] = val;
            if (j >= 1) in.store_owned(poff + s[m], val);
            t[m] = psg * val;
          }
          plaq_rot(t, ch, sh);
#pragma unroll
          for (int m = 0; m < 4; ++m) buf[s[m]] = t[m];
        }
      }
    }
    __syncthreads();
    // (b) even plaquettes: P_A, w = v - E (.), y = P_A(E w)
    if (act) {
      const T sg = (tau >= g.Ltau) ? (T)-1 : (T)1;
      const long toff = base + (long)tm * g.N;
      const T* Et = E + (long)tm * g.N;
#pragma unroll
      for (int k = 0; k < MAXSLOT; ++k) {
        const int q = lane + k * NT;
        if (k < nslot && q < g.Q) {
          int s[4];
          even_sites(g, q, s);
          T t[4], w[4];
#pragma unroll
          for (int m = 0; m < 4; ++m) t[m] = buf[s[m]];
          plaq_rot(t, ch, sh);
#pragma unroll
          for (int m = 0; m < 4; ++m) {
            const T e = Et[s[m]];
            w[m] = sg * (in.load(toff + s[m]) - e * t[m]);
            t[m] = e * w[m];
          }
          plaq_rot(t, ch, sh);
#pragma unroll
          for (int m = 0; m < 4; ++m) {
            buf[s[m]] = t[m];
            wbuf[s[m]] = w[m];
          }
        }
      }
    }
    __syncthreads();
    // (c) odd plaquettes: out_{tau-1} = w_{tau-1} - P_B y; keep w_tau
    if (act) {
      const long ooff = base + (long)(tau - 1) * g.N;
#pragma unroll
      for (int k = 0; k < MAXSLOT; ++k) {
        const int q = lane + k * NT;
        if (k < nslot && q < g.Q) {
          int s[4];
          odd_sites(g, q, s);
          T t[4];
#pragma unroll
          for (int m = 0; m < 4; ++m) t[m] = buf[s[m]];
          plaq_rot(t, ch, sh);
          if (j >= 1) {
#pragma unroll
            for (int m = 0; m < 4; ++m) epi.put(ooff + s[m], wprev[k][m] - t[m], vodd[k][m], acc);
          }
#pragma unroll
          for (int m = 0; m < 4; ++m) wprev[k][m] = wbuf[s[m]];
        }
      }
    }
  }

  if constexpr (Epi::kReduce) {
    const double bs = block_sum<NT>(acc, red_sh);
    if (threadIdx.x == 0) partial[(long)r * gridDim.x + blockIdx.x] = bs;
    if (last_block(counter + r, gridDim.x, &flag_sh)) {
      const double tot = reduce_partials<NT>(partial + (long)r * gridDim.x, gridDim.x, red_sh);
      if (threadIdx.x == 0) {
        epi.finish(st[r], tot);
        __threadfence();
        atomicExch(counter + r, 0u);
      }
    }
  }
}

// ------------------------------------------------------------- M alone --

// out = M v (mode 0), or the force (mode 1):
//   grad_tau += scale * sum_r (-2 dtau alpha) (M u)_tau * y_tau,
//   y_tau = E_tau * (C u~_{tau-1}), (M u)_tau = u_tau - y_tau   (Eq. dSF_dx)
// Launch: grid (ceil(Ltau / S / per), nrhs or 1).  Each (sub-)chunk of the
// block handles `per` slices.  LDS: S * N elements.
template <typename T, int NT, int MAXSLOT, int MODE>
__global__ void __launch_bounds__(NT)
k_apply_M(Geom g, const T* __restrict__ E, T ch, T sh, int per, int nrhs,
          const T* __restrict__ v, T* __restrict__ out, double coef) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int tid = threadIdx.x;
  int S, sub, lane, nslot;
  if (g.Q <= NT) {
    S = NT / g.Q;
    sub = tid / g.Q;
    lane = tid - sub * g.Q;
    nslot = 1;
  } else {
    S = 1;
    sub = 0;
    lane = tid;
    nslot = (g.Q + NT - 1) / NT;
  }
  T* buf = reinterpret_cast<T*>(smem_raw) + (long)(sub < S ? sub : 0) * g.N;
  const int tau_first = (blockIdx.x * S + sub) * per;
  const int rb = (MODE == 0) ? blockIdx.y : 0;
  const int re = (MODE == 0) ? blockIdx.y + 1 : nrhs;

  for (int j = 0; j < per; ++j) {
    const int tau = tau_first + j;
    const bool act = (sub < S) && (tau < g.Ltau);
    double gacc[MAXSLOT][4];
#pragma unroll
    for (int k = 0; k < MAXSLOT; ++k)
#pragma unroll
      for (int m = 0; m < 4; ++m) gacc[k][m] = 0.0;
    for (int r = rb; r < re; ++r) {
      const long base = (long)r * g.d;
      if (act) {
        int pt = tau - 1;
        T psg = (T)1;
        if (pt < 0) {
          pt = g.Ltau - 1;
          psg = (T)-1;
        }
#pragma unroll
        for (int k = 0; k < MAXSLOT; ++k) {
          const int q = lane + k * NT;
          if (k < nslot && q < g.Q) {
            int s[4];
            odd_sites(g, q, s);
            T t[4];
#pragma unroll
            for (int m = 0; m < 4; ++m) t[m] = psg * v[base + (long)pt * g.N + s[m]];
            plaq_rot(t, ch, sh);
#pragma unroll
            for (int m = 0; m < 4; ++m) buf[s[m]] = t[m];
          }
        }
      }
      __syncthreads();
      if (act) {
#pragma unroll
        for (int k = 0; k < MAXSLOT; ++k) {
          const int q = lane + k * NT;
          if (k < nslot && q < g.Q) {
            int s[4];
            even_sites(g, q, s);
            T t[4];
#pragma unroll
            for (int m = 0; m < 4; ++m) t[m] = buf[s[m]];
            plaq_rot(t, ch, sh);
#pragma unroll
            for (int m = 0; m < 4; ++m) {
              const long off = (long)tau * g.N + s[m];
              const T y = E[off] * t[m];
              const T w = v[base + off] - y;
              if (MODE == 0) {
                out[base + off] = w;
              } else {
                gacc[k][m] += (double)w * (double)y;
              }
            }
          }
        }
      }
      __syncthreads();
    }
    if (MODE == 1 && act) {
#pragma unroll
      for (int k = 0; k < MAXSLOT; ++k) {
        const int q = lane + k * NT;
        if (k < nslot && q < g.Q) {
          int s[4];
          even_sites(g, q, s);
#pragma unroll
          for (int m = 0; m < 4; ++m) {
            const long off = (long)tau * g.N + s[m];
            out[off] = (T)((double)out[off] + coef * gacc[k][m]);
          }
        }
      }
    }
  }
}

// ------------------------------------------------------------ M^T alone --

// out = M^T w.  Launch and LDS as k_apply_M (mode 0).
template <typename T, int NT, int MAXSLOT>
__global__ void __launch_bounds__(NT)
k_apply_MT(Geom g, const T* __restrict__ E, T ch, T sh, int per,
           const T* __restrict__ w, T* __restrict__ out) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int tid = threadIdx.x;
  int S, sub, lane, nslot;
  if (g.Q <= NT) {
    S = NT / g.Q;
    sub = tid / g.Q;
    lane = tid - sub * g.Q;
    nslot = 1;
  } else {
    S = 1;
    sub = 0;
    lane = tid;
    nslot = (g.Q + NT - 1) / NT;
  }
  T* buf = reinterpret_cast<T*>(smem_raw) + (long)(sub < S ? sub : 0) * g.N;
  const int tau_first = (blockIdx.x * S + sub) * per;
  const long base = (long)blockIdx.y * g.d;

  for (int j = 0; j < per; ++j) {
    const int tau = tau_first + j;
    const bool act = (sub < S) && (tau < g.Ltau);
    if (act) {
      int nt = tau + 1;
      T sg = (T)1;
      if (nt == g.Ltau) {
        nt = 0;
        sg = (T)-1;
      }
#pragma unroll
      for (int k = 0; k < MAXSLOT; ++k) {
        const int q = lane + k * NT;
        if (k < nslot && q < g.Q) {
          int s[4];
          even_sites(g, q, s);
          T t[4];
#pragma unroll
          for (int m = 0; m < 4; ++m) {
            const long off = (long)nt * g.N + s[m];
            t[m] = sg * E[off] * w[base + off];
          }
          plaq_rot(t, ch, sh);
#pragma unroll
          for (int m = 0; m < 4; ++m) buf[s[m]] = t[m];
        }
      }
    }
    __syncthreads();
    if (act) {
#pragma unroll
      for (int k = 0; k < MAXSLOT; ++k) {
        const int q = lane + k * NT;
        if (k < nslot && q < g.Q) {
          int s[4];
          odd_sites(g, q, s);
          T t[4];
#pragma unroll
          for (int m = 0; m < 4; ++m) t[m] = buf[s[m]];
          plaq_rot(t, ch, sh);
#pragma unroll
          for (int m = 0; m < 4; ++m) {
            const long off = base + (long)tau * g.N + s[m];
            out[off] = w[off] - t[m];
          }
        }
      }
    }
    __syncthreads();
  }
}

}  // namespace fph
