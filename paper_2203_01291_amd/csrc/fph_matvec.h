// Operator kernels: M, M^T, fused M^T M and the phonon force.
//
// (M v)_tau   = v_tau - E_tau * (C v~_{tau-1}),      v~_{-1} = -v_{Ltau-1}
// (M^T w)_tau = w_tau - C^T (E_{tau+1} * w~_{tau+1}), w~_{Ltau} = -w_0
// (Eq. M_def of the paper; B_tau = diag(E_tau) C, Eq. B_def, C = P_A P_B
// with P_B acting first; both factors are symmetric, so C^T = P_B P_A.)
//
// Fused M^T M over a chunk of consecutive slices [tau0, tau0 + Tc): step j
// (tau = tau0 + j, j = 0..Tc) forms w_tau = (M v)_tau in registers and, for
// j >= 1, emits out_{tau-1} = w_{tau-1} - C^T (E_tau w_tau).  Each thread
// owns one even plaquette (four sites, two aligned pairs of consecutive
// indices), so every global access is a paired load or store.  P_A acts
// within the thread; P_B couples the four sites to their odd-plaquette
// neighbours, which the thread reads from the slice in LDS (a 4x4 window).
// Only v, E and out touch global memory: 3 vectors per application for one
// right-hand side.
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

FPH_DEVINL void st2(double* p, double a, double b) {
  *reinterpret_cast<double2*>(p) = make_double2(a, b);
}
FPH_DEVINL void st2(float* p, float a, float b) {
  *reinterpret_cast<float2*>(p) = make_float2(a, b);
}

// ------------------------------------------------------- input functors --

// c ? b : a for two pointers, selected by value.  A plain conditional on
// two members of a by-value kernel argument is turned into a load from a
// computed address, which forces the whole argument into scratch memory.
template <typename P>
FPH_DEVINL P pick(bool c, P a, P b) {
  const uintptr_t m = (uintptr_t)0 - (uintptr_t)c;
  return (P)(((uintptr_t)a & ~m) | ((uintptr_t)b & m));
}

// The same for two values (bitwise, so the result is exactly a or b).
FPH_DEVINL float pickv(bool c, float a, float b) {
  const uint32_t m = 0u - (uint32_t)c;
  return __builtin_bit_cast(float, (__builtin_bit_cast(uint32_t, a) & ~m) |
                                       (__builtin_bit_cast(uint32_t, b) & m));
}
FPH_DEVINL double pickv(bool c, double a, double b) {
  const uint64_t m = 0ull - (uint64_t)c;
  return __builtin_bit_cast(double, (__builtin_bit_cast(uint64_t, a) & ~m) |
                                        (__builtin_bit_cast(uint64_t, b) & m));
}

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
  FPH_DEVINL void load2_owned(long off, T& a, T& b) const { ld2(v + off, a, b); }
  // Two-phase access used by the operator sweep (see mtm_sweep): fetch2
  // issues the loads, use2 forms the pair where it is needed.
  static constexpr bool kPrefetch = true;
  struct Raw {
    T a, b;
  };
  FPH_DEVINL void fetch2(long off, Raw& w, bool) const { ld2(v + off, w.a, w.b); }
  FPH_DEVINL void use2(long, const Raw& w, T& a, T& b, bool, bool) const {
    a = w.a;
    b = w.b;
  }
};

// fetch2 / use2 for inputs whose loads depend on the solver state: the
// whole load (and the owner's stores) happens in fetch2, after the state.
#define FPH_FETCH_AFTER_STATE(T)                                              \
  static constexpr bool kPrefetch = false;                                    \
  struct Raw {                                                                \
    T a, b;                                                                   \
  };                                                                          \
  FPH_DEVINL void fetch2(long off, Raw& w, bool owned) const {                \
    if (owned)                                                                \
      load2_owned(off, w.a, w.b);                                             \
    else                                                                      \
      load2(off, w.a, w.b);                                                   \
  }                                                                           \
  FPH_DEVINL void use2(long, const Raw& w, T& a, T& b, bool, bool) const {   \
    a = w.a;                                                                  \
    b = w.b;                                                                  \
  }

// p = z + beta p_old computed on the fly (the CG direction update fused
// into the operator), beta = rz_next / rz (Eq. CG_precon in the standard
// PCG form); the chunk owner stores p for its own slices.  The two
// direction buffers alternate with the parity of the right-hand side's own
// iteration count, so a paused right-hand side keeps a consistent pair.
// PF: the first slices are fetched before the state is known (z and both
// direction buffers; use2 picks the one the parity selects).
template <typename T, bool PF = false>
struct InPUpdate {
  const T* __restrict__ z;
  T* pa;
  T* pb;
  const T* __restrict__ pold;
  T* __restrict__ pnew;
  T beta;
  int fresh;
  int odd;    // parity of the right-hand side's iteration count
  int known;  // begin() has run: the state is known
  FPH_DEVINL void begin(const RhsState& s) {
    fresh = s.fresh;
    beta = fresh ? (T)0 : (T)(s.rz_next / s.rz);
    odd = (s.iter & 1) != 0;
    pold = pick(odd != 0, pa, pb);
    pnew = pick(odd != 0, pb, pa);
    known = 1;
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
  FPH_DEVINL void load2_owned(long off, T& a, T& b) const {
    load2(off, a, b);
    st2(pnew + off, a, b);
  }
  static constexpr bool kPrefetch = PF;
  struct Raw {
    T z0, z1, a0, a1, b0, b1;
  };
  FPH_DEVINL void fetch2(long off, Raw& w, bool) const {
    // (locals, all fields written: keeps Raw in registers)
    T z0, z1, a0 = (T)0, a1 = (T)0, b0 = (T)0, b1 = (T)0;
    ld2(z + off, z0, z1);
    if (!known || !fresh) ld2(pick<const T*>(known != 0, pa, pold) + off, a0, a1);
    if (!known) ld2(pb + off, b0, b1);
    w.z0 = z0;
    w.z1 = z1;
    w.a0 = a0;
    w.a1 = a1;
    w.b0 = b0;
    w.b1 = b1;
  }
  FPH_DEVINL void use2(long off, const Raw& w, T& a, T& b, bool owned, bool prefetched) const {
    a = w.z0;
    b = w.z1;
    if (!fresh) {
      const bool second = prefetched && odd;
      const T c = pickv(second, w.a0, w.b0), d = pickv(second, w.a1, w.b1);
      a += beta * c;
      b += beta * d;
    }
    if (owned) st2(pnew + off, a, b);
  }
};

// ---------------------------------------------------- epilogue functors --

// Plain store of out.
template <typename T>
struct EpiStore {
  T* __restrict__ out;
  FPH_DEVINL void begin(const RhsState&) {}
  FPH_DEVINL void put(long off, T o, T /*v*/, double& /*acc*/, double& /*acc2*/) const { out[off] = o; }
  FPH_DEVINL void put2(long off, T o0, T o1, T, T, double&, double&) const { st2(out + off, o0, o1); }
  static constexpr int kKind = P_NONE;
};

// Plain store that bypasses the caches (nontemporal): for applies whose
// output is far larger than the caches and is not read back soon.
template <typename T>
struct EpiStream {
  T* __restrict__ out;
  FPH_DEVINL void begin(const RhsState&) {}
  FPH_DEVINL void put2(long off, T o0, T o1, T, T, double&, double&) const {
    typedef T V2 __attribute__((ext_vector_type(2)));
    V2 v;
    v.x = o0;
    v.y = o1;
    __builtin_nontemporal_store(v, reinterpret_cast<V2*>(out + off));
  }
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
  FPH_DEVINL void put2(long off, T o0, T o1, T v0, T v1, double& acc, double&) const {
    st2(out + off, o0, o1);
    acc += (double)v0 * (double)o0 + (double)v1 * (double)o1;
  }
  static constexpr int kKind = P_PAP;
};

// True residual r = b - A u in FP64, stored as TR (float or double);
// accumulates |b - A u|^2 and |b|^2 in FP64 (consumed as P_RES).
template <typename TR>
struct EpiResidual {
  const double* __restrict__ b;
  TR* __restrict__ r;
  FPH_DEVINL void begin(const RhsState&) {}
  FPH_DEVINL void put2(long off, double o0, double o1, double, double, double& acc,
                       double& acc2) const {
    double b0, b1;
    ld2(b + off, b0, b1);
    const double r0 = b0 - o0, r1 = b1 - o1;
    st2(r + off, (TR)r0, (TR)r1);
    acc += r0 * r0 + r1 * r1;
    acc2 += b0 * b0 + b1 * b1;
  }
  static constexpr int kKind = P_RES;
};

// The FP64 iterate of an FP32-refined solve with its FP32 correction added
// on the fly: u = u64[upar] + u32 (u32 omitted while it is zero), read on
// every slice the sweep visits (halo slices too); the chunk owner stores u
// into the other FP64 buffer, so the correction is folded into the iterate
// by the residual evaluation itself, with no race between neighbouring
// chunks (nobody writes the buffer being read).
struct InResid {
  const double* u0;   // u_dev
  double* u1;         // workspace buffer
  const float* u32;
  const double* src;
  double* dst;
  int z;              // the correction is zero
  FPH_DEVINL void begin(const RhsState& s) {
    src = pick(s.upar != 0, u0, (const double*)u1);
    dst = pick(s.upar != 0, u1, const_cast<double*>(u0));
    z = s.u32z;
  }
  static constexpr bool kPrefetch = false;
  struct Raw {
    double a, b;
  };
  FPH_DEVINL void fetch2(long off, Raw& w, bool) const {
    double a, b;
    ld2(src + off, a, b);
    if (!z) {
      float c, d;
      ld2(u32 + off, c, d);
      a += (double)c;
      b += (double)d;
    }
    w.a = a;
    w.b = b;
  }
  FPH_DEVINL void use2(long off, const Raw& w, double& a, double& b, bool owned, bool) const {
    a = w.a;
    b = w.b;
    if (owned) st2(dst + off, a, b);
  }
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

// P_B at the four sites of the even plaquette with corner (x0, y0), read
// from the slice in LDS: the odd plaquettes covering those sites span the
// 4x4 window x0-1..x0+2, y0-1..y0+2 (periodic).  Site (dx, dy) of the even
// plaquette is local site (1-dx, 1-dy) of its odd plaquette, so with
// C2' = [[1, th], [th, 1]] along each axis (P'_B, P_B = ch^2 P'_B)
//   out(dx, dy) = sum_{a,b} c'(1-dy, b) c'(1-dx, a) W[2dy + b][2dx + a].
template <typename T>
FPH_DEVINL void pb_window(const Geom& g, const T* __restrict__ sl, int x0, int y0, T th,
                          T out[4]) {
  const int xm = (x0 == 0) ? g.L - 1 : x0 - 1;
  const int xp = (x0 + 2 == g.L) ? 0 : x0 + 2;
  const int ym = (y0 == 0) ? g.L - 1 : y0 - 1;
  const int yp = (y0 + 2 == g.L) ? 0 : y0 + 2;
  const int rows[4] = {ym, y0, y0 + 1, yp};
  T h0[4], h1[4];  // x-combinations for dx = 0 (cols xm, x0) and dx = 1 (cols x0+1, xp)
#pragma unroll
  for (int rr = 0; rr < 4; ++rr) {
    const T* row = sl + g.L * rows[rr];
    T a, b;
    ld2(row + x0, a, b);
    const T wm = row[xm], wp = row[xp];
    h0[rr] = fma(th, wm, a);
    h1[rr] = fma(th, wp, b);
  }
  out[0] = fma(th, h0[0], h0[1]);
  out[1] = fma(th, h1[0], h1[1]);
  out[2] = fma(th, h0[3], h0[2]);
  out[3] = fma(th, h1[3], h1[2]);
}

// The fused M^T M sweep of one chunk of slices [tau0, tau0 + Tc) of one
// right-hand side (offset `base`), see the file comment; every thread of
// the block calls it (inactive threads keep the barrier).  All global
// traffic is in the even-plaquette layout (pairs of consecutive sites).
// Per step tau (one barrier):
//   (i)  t = P_B v~_{tau-1} from LDS buffer A[j&1]; w_tau = v_tau - E_tau
//        P_A t; y = P_A(E_tau w_tau) -> B[j&1]; v~_tau -> A[(j+1)&1]
//   (ii) out_{tau-1} = w_{tau-1} - P_B y (read from B[j&1]).
// LDS: 4 slices (A[2], B[2]) per chunk.
// Loads run DEPTH slices ahead of their use.  `hook` folds the solver
// state and configures `in` / `epi`; it returns false when the right-hand
// side is finished (then the sweep returns false at once).  With
// In::kPrefetch the loads of the first slices are issued before the hook,
// so they overlap the state's memory round trip.
template <typename T, int NT, int MAXSLOT, int DEPTH, class In, class Epi, class Hook>
FPH_DEVINL bool mtm_sweep(const Geom& g, const T* __restrict__ E, T th, int Tch, int tau0,
                          int Tc, bool active, int lane, int nslot, T* lds4, long base,
                          In& in, Epi& epi, double& acc, double& acc2, Hook&& hook) {
  static_assert(DEPTH == 1 || DEPTH == 2, "DEPTH is 1 or 2");
  using Raw = typename In::Raw;
  T* A0 = lds4;
  T* A1 = lds4 + g.N;
  T* B0 = lds4 + 2 * g.N;
  T* B1 = lds4 + 3 * g.N;
  Raw q0[MAXSLOT][2], q1[MAXSLOT][2];   // v of the next slices, as fetched
  T e0[MAXSLOT][4], e1[MAXSLOT][4];     // E of the next slices
  Raw pro[MAXSLOT][2];                  // v of slice tau0 - 1
  T wprev[MAXSLOT][4], vprev[MAXSLOT][4];
  const int pt = (tau0 == 0) ? g.Ltau - 1 : tau0 - 1;
  const long poff = base + (long)pt * g.N;

  auto fetch = [&](int jj, Raw (&dst)[MAXSLOT][2], T (&e)[MAXSLOT][4]) {
    const int tau = tau0 + jj;
    const int tm = (tau >= g.Ltau) ? tau - g.Ltau : tau;
    const long toff = base + (long)tm * g.N;
    const T* Et = E + (long)tm * g.N;
#pragma unroll
    for (int k = 0; k < MAXSLOT; ++k) {
      const int q = lane + k * NT;
      if (k < nslot && q < g.Q) {
        const int i0 = 2 * (q % g.hL) + g.L * 2 * (q / g.hL);
        in.fetch2(toff + i0, dst[k][0], jj < Tc);
        in.fetch2(toff + i0 + g.L, dst[k][1], jj < Tc);
        ld2(Et + i0, e[k][0], e[k][1]);
        ld2(Et + i0 + g.L, e[k][2], e[k][3]);
      }
    }
  };
  auto fetch_first = [&]() {
    if (!active) return;
#pragma unroll
    for (int k = 0; k < MAXSLOT; ++k) {
      const int q = lane + k * NT;
      if (k < nslot && q < g.Q) {
        const int i0 = 2 * (q % g.hL) + g.L * 2 * (q / g.hL);
        in.fetch2(poff + i0, pro[k][0], false);
        in.fetch2(poff + i0 + g.L, pro[k][1], false);
      }
    }
    fetch(0, q0, e0);
    if (DEPTH == 2 && 1 <= Tc) fetch(1, q1, e1);
  };

  if constexpr (In::kPrefetch) {
    fetch_first();
    if (!hook()) return false;
  } else {
    if (!hook()) return false;
    fetch_first();
  }
  constexpr bool kEarly = In::kPrefetch;  // the first DEPTH slices were fetched before the hook

  // Prologue: v~_{tau0 - 1} into A0 (antiperiodic sign at the wrap).
  if (active) {
    const T psg = (tau0 == 0) ? (T)-1 : (T)1;
#pragma unroll
    for (int k = 0; k < MAXSLOT; ++k) {
      const int q = lane + k * NT;
      if (k < nslot && q < g.Q) {
        const int i0 = 2 * (q % g.hL) + g.L * 2 * (q / g.hL);
        T a, b, c, d;
        in.use2(poff + i0, pro[k][0], a, b, false, kEarly);
        in.use2(poff + i0 + g.L, pro[k][1], c, d, false, kEarly);
        st2(A0 + i0, psg * a, psg * b);
        st2(A0 + i0 + g.L, psg * c, psg * d);
      }
    }
  }
  __syncthreads();

  for (int j = 0; j <= Tch; ++j) {
    const int tau = tau0 + j;
    const bool act = active && (j <= Tc);
    const T* Acur = (j & 1) ? A1 : A0;
    T* Anext = (j & 1) ? A0 : A1;
    T* Bcur = (j & 1) ? B1 : B0;
    Raw cr[MAXSLOT][2];
    T ne[MAXSLOT][4];
#pragma unroll
    for (int k = 0; k < MAXSLOT; ++k) {
      cr[k][0] = q0[k][0];
      cr[k][1] = q0[k][1];
#pragma unroll
      for (int m = 0; m < 4; ++m) ne[k][m] = e0[k][m];
    }
    if (DEPTH == 2) {
#pragma unroll
      for (int k = 0; k < MAXSLOT; ++k) {
        q0[k][0] = q1[k][0];
        q0[k][1] = q1[k][1];
#pragma unroll
        for (int m = 0; m < 4; ++m) e0[k][m] = e1[k][m];
      }
      if (active && j + 2 <= Tc) fetch(j + 2, q1, e1);
    } else {
      if (active && j + 1 <= Tc) fetch(j + 1, q0, e0);
    }
    T wcur[MAXSLOT][4], nv[MAXSLOT][4];
    if (act) {
      const T sg = (tau >= g.Ltau) ? (T)-1 : (T)1;          // w_{Ltau} = -w_0
      const T nsg = (tau + 1 == g.Ltau) ? (T)-1 : (T)1;     // v~ for the next step
      const int tm = (tau >= g.Ltau) ? tau - g.Ltau : tau;
      const long toff = base + (long)tm * g.N;
      const bool early = kEarly && j < DEPTH;
#pragma unroll
      for (int k = 0; k < MAXSLOT; ++k) {
        const int q = lane + k * NT;
        if (k < nslot && q < g.Q) {
          const int x0 = 2 * (q % g.hL), y0 = 2 * (q / g.hL);
          const int i0 = x0 + g.L * y0;
          in.use2(toff + i0, cr[k][0], nv[k][0], nv[k][1], j < Tc, early);
          in.use2(toff + i0 + g.L, cr[k][1], nv[k][2], nv[k][3], j < Tc, early);
          T t[4];
          pb_window(g, Acur, x0, y0, th, t);
          plaq_rot(t, th);
#pragma unroll
          for (int m = 0; m < 4; ++m) {
            wcur[k][m] = sg * (nv[k][m] - ne[k][m] * t[m]);
            t[m] = ne[k][m] * wcur[k][m];
          }
          plaq_rot(t, th);
          st2(Bcur + i0, t[0], t[1]);
          st2(Bcur + i0 + g.L, t[2], t[3]);
          st2(Anext + i0, nsg * nv[k][0], nsg * nv[k][1]);
          st2(Anext + i0 + g.L, nsg * nv[k][2], nsg * nv[k][3]);
        }
      }
    }
    __syncthreads();
    if (act) {
      const long ooff = base + (long)(tau - 1) * g.N;
#pragma unroll
      for (int k = 0; k < MAXSLOT; ++k) {
        const int q = lane + k * NT;
        if (k < nslot && q < g.Q) {
          const int x0 = 2 * (q % g.hL), y0 = 2 * (q / g.hL);
          const int i0 = x0 + g.L * y0;
          if (j >= 1) {
            T t[4];
            pb_window(g, Bcur, x0, y0, th, t);
            epi.put2(ooff + i0, wprev[k][0] - t[0], wprev[k][1] - t[1], vprev[k][0],
                     vprev[k][1], acc, acc2);
            epi.put2(ooff + i0 + g.L, wprev[k][2] - t[2], wprev[k][3] - t[3], vprev[k][2],
                     vprev[k][3], acc, acc2);
          }
#pragma unroll
          for (int m = 0; m < 4; ++m) {
            wprev[k][m] = wcur[k][m];
            vprev[k][m] = nv[k][m];
          }
        }
      }
    }
  }
  return true;
}

// Launch: grid (nblk * nrhs) (see xcd_contiguous).  Block b of right-hand side r serves `S`
// chunks of `Tch` slices each; with Q <= NT plaquettes per slice, S = NT/Q
// chunks run side by side (one plaquette per thread), otherwise S = 1 and a
// thread serves up to MAXSLOT plaquettes.  LDS: 4 * S * N elements of T.
// A plain apply (no solver state; the CG iterations use k_slot_mtm).  Plain
// FP32 applies in 1024-thread workgroups are held to 8 waves per SIMD
// (64 VGPRs), so two workgroups share a CU.
template <typename T, int NT>
constexpr int mtm_min_waves() {
  return (NT == 1024 && sizeof(T) == 4) ? 8 : 1;
}

// Workgroups are handed to the 8 XCDs round robin; renumber them so each
// XCD gets a contiguous range of (chunk-major, right-hand side minor) work:
// neighbouring chunks (which share halo slices) and the chunks of all
// right-hand sides at the same slices (which share E) meet in one L2.
FPH_DEVINL void mtm_block(int nblk, int& r, int& bx) {
  const int logical = xcd_contiguous(blockIdx.x, gridDim.x);
  const int nrhs = gridDim.x / nblk;
  r = logical % nrhs;
  bx = logical / nrhs;
}

template <typename T, int NT, int MAXSLOT, class In, class Epi>
__global__ void __launch_bounds__(NT, (mtm_min_waves<T, NT>()))
k_mtm(Geom g, const T* __restrict__ E, T th, int Tch, int nblk, In in, Epi epi) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  int r, bx;
  mtm_block(nblk, r, bx);
  E += field_off(g, r);
  const int tid = threadIdx.x;
  int S, sub, lane, nslot;
  block_layout<NT>(g, tid, S, sub, lane, nslot);
  const int chunk = bx * S + sub;
  const int tau0 = chunk * Tch;
  const bool active = (sub < S) && (tau0 < g.Ltau);
  const int Tc = active ? min(Tch, g.Ltau - tau0) : 0;
  T* lds4 = reinterpret_cast<T*>(smem_raw) + 4L * (sub < S ? sub : 0) * g.N;
  const long base = (long)r * g.d;
  double acc = 0.0, acc2 = 0.0;
  mtm_sweep<T, NT, MAXSLOT, 1>(g, E, th, Tch, tau0, Tc, active, lane, nslot, lds4, base, in, epi,
                               acc, acc2, [] { return true; });
}

// ------------------------------------------------------------- M alone --

// out = M v (mode 0), or the force (mode 1):
//   grad_tau += coef * s * sum_r (M u)_tau * y_tau,  coef = -2 dtau alpha scale,
//   y_tau = E_tau * (C u~_{tau-1}), (M u)_tau = u_tau - y_tau   (Eq. dSF_dx),
//   s = *scale_dev (device value read at run time) or 1 when scale_dev is null.
// Launch: grid (ceil(Ltau / S / per), nrhs in mode 0; in mode 1 the number
// of fields, block y summing the right-hand sides of field y into grad[y]).
// Each (sub-)chunk of the block handles `per` slices.  LDS: S * N elements.
template <typename T, int NT, int MAXSLOT, int MODE>
__global__ void __launch_bounds__(NT)
k_apply_M(Geom g, const T* __restrict__ E, T th, int per, int nrhs,
          const T* __restrict__ v, T* __restrict__ out, double coef,
          const double* __restrict__ scale_dev) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  if (MODE == 1 && scale_dev != nullptr) coef *= *scale_dev;
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
  int rb, re;
  if (MODE == 0) {
    rb = blockIdx.y;
    re = rb + 1;
  } else if (g.fs) {
    rb = blockIdx.y * g.rpf;
    re = min(rb + g.rpf, nrhs);
    out += (long)blockIdx.y * g.d;
  } else {
    rb = 0;
    re = nrhs;
  }
  E += field_off(g, rb);

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
            plaq_rot(t, th);
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
            plaq_rot(t, th);
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
k_apply_MT(Geom g, const T* __restrict__ E, T th, int per,
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
  E += field_off(g, blockIdx.y);

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
          plaq_rot(t, th);
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
          plaq_rot(t, th);
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
