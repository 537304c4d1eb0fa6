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

// Two consecutive elements (the x-pair of an even plaquette row; the
// offset is even, so the pair is naturally aligned).
FPH_DEVINL void ld2(const double* p, double& a, double& b) {
  const double2 v = *reinterpret_cast<const double2*>(p);
  a = v.x;
  b = v.y;
}
FPH_DEVINL void ld2(const float* p, float& a, float& b) {
  const float2 v = *reinterpret_cast<const float2*>(p);
  a = v.x;
  b = v.y;
}

// ------------------------------------------------------- input functors --

// v read directly.
template <typename T>
struct InPlain {
  const T* __restrict__ v;
  static FPH_DEVINL void prepare(RhsState&) {}
  FPH_DEVINL void begin(const RhsState&) {}
  static FPH_DEVINL void on_state(RhsState&) {}
  FPH_DEVINL T load(long off) const { return v[off]; }
  FPH_DEVINL T load_owned(long off) const { return v[off]; }
  FPH_DEVINL void load2(long off, T& a, T& b) const { ld2(v + off, a, b); }
};

// v = one of two buffers chosen by the parity of the iteration count
// (single-reduction CG keeps its residual double-buffered).
template <typename T>
struct InParity {
  const T* buf[2];
  const T* __restrict__ v;
  static FPH_DEVINL void prepare(RhsState&) {}
  FPH_DEVINL void begin(const RhsState& s) { v = buf[s.iter & 1]; }
  static FPH_DEVINL void on_state(RhsState&) {}
  FPH_DEVINL T load(long off) const { return v[off]; }
  FPH_DEVINL T load_owned(long off) const { return v[off]; }
  FPH_DEVINL void load2(long off, T& a, T& b) const { ld2(v + off, a, b); }
};

// p = z + beta p_old computed on the fly (the CG direction update fused
// into the operator), beta = rz_next / rz (Eq. CG_precon in the standard
// PCG form); the chunk owner stores p for its own slices.  The two
// direction buffers alternate with the parity of the right-hand side's own
// iteration count, so a paused right-hand side keeps a consistent pair.
template <typename T>
struct InPUpdate {
  const T* __restrict__ z;
  T* pa;
  T* pb;
  const T* __restrict__ pold;
  T* __restrict__ pnew;
  T beta;
  int fresh;
  FPH_DEVINL void begin(const RhsState& s) {
    fresh = s.fresh;
    beta = fresh ? (T)0 : (T)(s.rz_next / s.rz);
    const bool odd = (s.iter & 1) != 0;
    pold = odd ? pb : pa;
    pnew = odd ? pa : pb;
  }
  // Direction-update bookkeeping, applied once to the shared state.
  static FPH_DEVINL void on_state(RhsState& s) {
    s.beta = s.fresh ? 0.0 : s.rz_next / s.rz;
    s.rz = s.rz_next;
    s.fresh = 0;
  }
  static FPH_DEVINL void prepare(RhsState&) {}
  FPH_DEVINL T load(long off) const { return fresh ? z[off] : z[off] + beta * pold[off]; }
  FPH_DEVINL T load_owned(long off) const {
    const T v = load(off);
    pnew[off] = v;
    return v;
  }
  FPH_DEVINL void load2(long off, T& a, T& b) const {
    ld2(z + off, a, b);
    if (!fresh) {
      T c, d;
      ld2(pold + off, c, d);
      a += beta * c;
      b += beta * d;
    }
  }
};

// Single-reduction CG (Chronopoulos and Gear, 1989): with gamma_i = r_i.r_i,
// delta_i = r_i.A r_i and w_i = A r_i,
//   beta_i = gamma_i / gamma_{i-1},
//   alpha_i = gamma_i / (delta_i - beta_i gamma_i / alpha_{i-1}),
//   p_i = r_i + beta_i p_{i-1},  s_i = w_i + beta_i s_{i-1}  (= A p_i),
//   x += alpha_i p_i,  r_{i+1} = r_i - alpha_i s_i,  w_{i+1} = A r_{i+1}.
// The operator kernel forms r_{i+1} on the fly (also on halo slices), the
// chunk owner stores p_i, s_i, x and r_{i+1}; the operator output is
// w_{i+1} and the epilogue forms both dots of the next step, so one launch
// is one iteration.  r, w, s, p alternate between two buffers by the
// parity of i.
template <typename T>
struct InCGCG {
  T* R[2];
  T* S[2];
  T* P[2];
  const T* W[2];
  T* x;
  const T* __restrict__ ri;
  const T* __restrict__ wi;
  const T* __restrict__ so;
  const T* __restrict__ po;
  T* __restrict__ rn;
  T* __restrict__ sn;
  T* __restrict__ pn;
  T alpha, beta;
  int fresh;
  static FPH_DEVINL void prepare(RhsState& s) {
    if (s.fresh) {
      s.beta = 0.0;
      if (!(s.delta > 0.0)) {
        s.status |= 4;
        s.done = 1;
        return;
      }
      s.alpha = s.gamma / s.delta;
    } else {
      s.beta = s.gamma / s.gamma_prev;
      const double den = s.delta - s.beta * s.gamma / s.alpha_prev;
      if (!(den > 0.0)) {
        s.status |= 4;
        s.done = 1;
        return;
      }
      s.alpha = s.gamma / den;
    }
  }
  FPH_DEVINL void begin(const RhsState& s) {
    const int c = s.iter & 1, n = c ^ 1;
    ri = R[c];
    wi = W[c];
    rn = R[n];
    so = S[n];
    sn = S[c];
    po = P[n];
    pn = P[c];
    alpha = (T)s.alpha;
    beta = (T)s.beta;
    fresh = s.fresh;
  }
  static FPH_DEVINL void on_state(RhsState& s) {
    s.gamma_prev = s.gamma;
    s.alpha_prev = s.alpha;
    s.fresh = 0;
    s.iter += 1;
    s.matvecs += 1;
  }
  FPH_DEVINL T load(long off) const {
    const T sv = fresh ? wi[off] : wi[off] + beta * so[off];
    return ri[off] - alpha * sv;
  }
  FPH_DEVINL T load_owned(long off) const {
    const T r = ri[off], w = wi[off];
    const T sv = fresh ? w : w + beta * so[off];
    const T pv = fresh ? r : r + beta * po[off];
    const T rv = r - alpha * sv;
    sn[off] = sv;
    pn[off] = pv;
    x[off] += alpha * pv;
    rn[off] = rv;
    return rv;
  }
  FPH_DEVINL void load2(long off, T& a, T& b) const {
    T r0, r1, w0, w1;
    ld2(ri + off, r0, r1);
    ld2(wi + off, w0, w1);
    if (!fresh) {
      T s0, s1;
      ld2(so + off, s0, s1);
      w0 += beta * s0;
      w1 += beta * s1;
    }
    a = r0 - alpha * w0;
    b = r1 - alpha * w1;
  }
};

// ---------------------------------------------------- epilogue functors --

// Plain store of out.
template <typename T>
struct EpiStore {
  T* __restrict__ out;
  FPH_DEVINL void begin(const RhsState&) {}
  FPH_DEVINL void put(long off, T o, T /*v*/, double& /*acc*/, double& /*acc2*/) const { out[off] = o; }
  static constexpr int kKind = P_NONE;
};

// Store out = A p and accumulate p . A p (consumed as P_PAP: alpha).
template <typename T>
struct EpiDot {
  T* __restrict__ out;
  FPH_DEVINL void begin(const RhsState&) {}
  FPH_DEVINL void put(long off, T o, T v, double& acc, double& /*acc2*/) const {
    out[off] = o;
    acc += (double)v * (double)o;
  }
  static constexpr int kKind = P_PAP;
};

// Store w = A r into the buffer of parity (iter + shift) and accumulate
// r.r and r.w (consumed as P_GD by single-reduction CG).
template <typename T>
struct EpiGD {
  T* W[2];
  int shift;
  T* __restrict__ out;
  FPH_DEVINL void begin(const RhsState& s) { out = W[(s.iter + shift) & 1]; }
  FPH_DEVINL void put(long off, T o, T v, double& acc, double& acc2) const {
    out[off] = o;
    acc += (double)v * (double)v;
    acc2 += (double)v * (double)o;
  }
  static constexpr int kKind = P_GD;
};

// True residual r = b - A u in FP64, stored as TR (float or double);
// accumulates |b - A u|^2 in FP64 (consumed as P_TRUE).
template <typename TR>
struct EpiResidual {
  const double* __restrict__ b;
  TR* __restrict__ r;
  FPH_DEVINL void begin(const RhsState&) {}
  FPH_DEVINL void put(long off, double o, double /*v*/, double& acc, double& /*acc2*/) const {
    const double res = b[off] - o;
    r[off] = (TR)res;
    acc += res * res;
  }
  static constexpr int kKind = P_TRUE;
};

// ------------------------------------------------------ fused M^T M ------

// Thread layout of the operator kernels: with Q <= NT plaquettes per
// slice, S = NT / Q chunks run side by side (thread -> (sub, lane));
// otherwise one chunk and up to ceil(Q / NT) plaquettes per thread.
template <int NT>
FPH_DEVINL void block_layout(const Geom& g, int tid, int& S, int& sub, int& lane, int& nslot) {
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
}

// The fused M^T M sweep of one chunk of slices [tau0, tau0 + Tc) of one
// right-hand side (offset `base`), see the file comment.  Every thread of
// the block calls it (inactive threads keep the barriers).  `in` supplies
// the input vector, `epi` consumes the output and accumulates dots.
template <typename T, int NT, int MAXSLOT, class In, class Epi>
FPH_DEVINL void mtm_chunks(const Geom& g, const T* __restrict__ E, T ch, T sh, int Tch, int tau0,
                           int Tc, bool active, int lane, int nslot, T* buf, T* wbuf, long base,
                           const In& in, const Epi& epi, double& acc, double& acc2) {
  T wprev[MAXSLOT][4];
  T vodd[MAXSLOT][4];
  // Software pipeline: the global loads of step j + 1 (odd plaquettes of
  // slice tau-1 for (a), even plaquettes of v and E at slice tau for (b))
  // are issued while step j works on LDS.
  T na[MAXSLOT][4];             // next (a): v at odd sites of slice tau-1
  T nv[MAXSLOT][4], ne[MAXSLOT][4];  // next (b): v, E at even sites of slice tau

  auto issue = [&](int jj) {
    const int tau = tau0 + jj;
    const int tm = (tau >= g.Ltau) ? tau - g.Ltau : tau;
    const int pt = (tm == 0) ? g.Ltau - 1 : tm - 1;
    const long poff = base + (long)pt * g.N;
    const long toff = base + (long)tm * g.N;
    const T* Et = E + (long)tm * g.N;
#pragma unroll
    for (int k = 0; k < MAXSLOT; ++k) {
      const int q = lane + k * NT;
      if (k < nslot && q < g.Q) {
        int so[4], se[4];
        odd_sites(g, q, so);
        even_sites(g, q, se);
        if (jj >= 1) {  // slice tau-1 is owned by this chunk: elementwise updates
#pragma unroll
          for (int m = 0; m < 4; ++m) na[k][m] = in.load_owned(poff + so[m]);
        } else {
#pragma unroll
          for (int m = 0; m < 4; ++m) na[k][m] = in.load(poff + so[m]);
        }
        in.load2(toff + se[0], nv[k][0], nv[k][1]);
        in.load2(toff + se[2], nv[k][2], nv[k][3]);
        ld2(Et + se[0], ne[k][0], ne[k][1]);
        ld2(Et + se[2], ne[k][2], ne[k][3]);
      }
    }
  };

  if (active) issue(0);
  for (int j = 0; j <= Tch; ++j) {
    const int tau = tau0 + j;
    const bool act = active && (j <= Tc);
    const int tm = (tau >= g.Ltau) ? tau - g.Ltau : tau;
    // (a) v~_{tau-1} on odd plaquettes -> P_B -> LDS
    if (act) {
      const T psg = (tm == 0) ? (T)-1 : (T)1;
#pragma unroll
      for (int k = 0; k < MAXSLOT; ++k) {
        const int q = lane + k * NT;
        if (k < nslot && q < g.Q) {
          int s[4];
          odd_sites(g, q, s);
          T t[4];
#pragma unroll
          for (int m = 0; m < 4; ++m) {
            const T val = na[k][m];
            vodd[k][m] = val;
            t[m] = psg * val;
          }
          plaq_rot(t, ch, sh);
#pragma unroll
          for (int m = 0; m < 4; ++m) buf[s[m]] = t[m];
        }
      }
    }
    __syncthreads();
    // (b) even plaquettes: P_A, w = v - E (.), y = P_A(E w); then issue the
    // loads of the next step
    T cv[MAXSLOT][4], ce[MAXSLOT][4];
#pragma unroll
    for (int k = 0; k < MAXSLOT; ++k)
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        cv[k][m] = nv[k][m];
        ce[k][m] = ne[k][m];
      }
    if (active && j + 1 <= Tc) issue(j + 1);
    if (act) {
      const T sg = (tau >= g.Ltau) ? (T)-1 : (T)1;
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
            const T e = ce[k][m];
            w[m] = sg * (cv[k][m] - e * t[m]);
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
            for (int m = 0; m < 4; ++m)
              epi.put(ooff + s[m], wprev[k][m] - t[m], vodd[k][m], acc, acc2);
          }
#pragma unroll
          for (int m = 0; m < 4; ++m) wprev[k][m] = wbuf[s[m]];
        }
      }
    }
  }

}

// Launch: grid (nblk, nrhs).  Block b of right-hand side r serves `S`
// chunks of `Tch` slices each; with Q <= NT plaquettes per slice, S = NT/Q
// chunks run side by side (one plaquette per thread), otherwise S = 1 and a
// thread serves up to MAXSLOT plaquettes.  LDS: 2 * S * N elements of T.
// With io.in set, the kernel takes part in the CG state machine: it folds
// pending partials, skips finished right-hand sides and publishes its own
// partials (Epi::kKind).
template <typename T, int NT, int MAXSLOT, class In, class Epi>
__global__ void __launch_bounds__(NT)
k_mtm(Geom g, const T* __restrict__ E, T ch, T sh, int Tch, In in, Epi epi, StIO io) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red_sh[NT / 64];
  __shared__ RhsState s_sh;
  const int r = blockIdx.y;
  if (io.in != nullptr) {
    state_begin<NT>(io, r, &s_sh, red_sh);
    if (threadIdx.x == 0 && !s_sh.done) In::prepare(s_sh);
    __syncthreads();
    if (s_sh.done) {
      state_end(io, r, &s_sh, P_NONE, 0.0, blockIdx.x, gridDim.x, blockIdx.x == 0);
      return;
    }
    in.begin(s_sh);
    epi.begin(s_sh);
    __syncthreads();
    if (threadIdx.x == 0) In::on_state(s_sh);
  }

  const int tid = threadIdx.x;
  int S, sub, lane, nslot;
  block_layout<NT>(g, tid, S, sub, lane, nslot);
  const int chunk = blockIdx.x * S + sub;
  const int tau0 = chunk * Tch;
  const bool active = (sub < S) && (tau0 < g.Ltau);
  const int Tc = active ? min(Tch, g.Ltau - tau0) : 0;
  T* buf = reinterpret_cast<T*>(smem_raw) + (long)(sub < S ? sub : 0) * g.N;
  T* wbuf = reinterpret_cast<T*>(smem_raw) + (long)S * g.N + (long)(sub < S ? sub : 0) * g.N;
  const long base = (long)r * g.d;
  double acc = 0.0, acc2 = 0.0;
  mtm_chunks<T, NT, MAXSLOT>(g, E, ch, sh, Tch, tau0, Tc, active, lane, nslot, buf, wbuf, base,
                             in, epi, acc, acc2);

  if (io.in != nullptr) {
    double bs = 0.0, bs2 = 0.0;
    if constexpr (Epi::kKind != P_NONE) bs = block_sum<NT>(acc, red_sh);
    if constexpr (Epi::kKind == P_GD) bs2 = block_sum<NT>(acc2, red_sh);
    state_end(io, r, &s_sh, Epi::kKind, bs, blockIdx.x, gridDim.x, blockIdx.x == 0, bs2);
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
