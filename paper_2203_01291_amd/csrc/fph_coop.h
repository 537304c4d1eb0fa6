// One-launch FP32-refined CG for one right-hand side (Eq. CG on M^T M
// with FP64 residual replacement, as in the multi-kernel solver).
//
// A cooperative launch keeps every workgroup resident for the whole solve.
// Workgroup b owns a chunk of consecutive slices (the operator sweep of
// fph_matvec.h, with halo slices read from its neighbours).  Each phase
// ends in a grid-wide exchange of per-workgroup partial sums that doubles
// as the barrier: every workgroup writes its partial into a slot of the
// phase's region, and the first wave of every workgroup polls the region
// until no slot holds the empty marker, then sums the slots in a fixed
// order (all workgroups get bit-identical totals).  Regions rotate over
// kRegions phases; a workgroup re-marks its own slot of the region used two
// phases earlier, which every reader has finished with by then.
//
// Data exchanged between workgroups (r, the directions, u64, the partial
// slots) are written and read with device-coherent 8-byte accesses, so
// the XCDs' separate L2 caches never serve stale copies; data a workgroup
// only uses itself (u32, Ap) take the ordinary cached path.  Every wait is
// bounded: a workgroup that polls too long raises the abort flag, and all
// workgroups leave at their next exchange.
//
// Per CG iteration (two exchanges):
//   A: p = r + beta p_old (fresh: p = r) on the owned slices, also formed
//      on the halo slices from the neighbours' r and p_old; Ap = M^T M p;
//      partial p.Ap.
//   B: alpha = rz / p.Ap; u32 += alpha p; r -= alpha Ap; partial |r|^2.
// Residual replacement (when |r|^2 fell by delta^2 since the last one,
// reached the tolerance, or the iteration cap): u64 += u32, u32 = 0 |
// r = b - M^T M u64 in FP64 (stored as FP32) with |r|^2 and |b|^2.
#pragma once

#include "fph_blas.h"
#include "fph_common.h"
#include "fph_matvec.h"

namespace fph {

constexpr int kRegions = 4;
constexpr int kCoopMaxBlocks = 512;  // slots per region (2 values each)
constexpr uint64_t kEmptySlot = 0x7ff8dead7ff8deadull;  // a NaN no sum produces
constexpr long kPollLimit = 1L << 20;  // about a second of polling

// ----------------------------------------------------- coherent accesses

FPH_DEVINL uint64_t ld_dev(const uint64_t* p) {
  return __hip_atomic_load(const_cast<uint64_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
FPH_DEVINL void st_dev(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
FPH_DEVINL void ld2_dev(const float* p, float& a, float& b) {
  const uint64_t v = ld_dev(reinterpret_cast<const uint64_t*>(p));
  a = __builtin_bit_cast(float, (uint32_t)v);
  b = __builtin_bit_cast(float, (uint32_t)(v >> 32));
}
FPH_DEVINL void st2_dev(float* p, float a, float b) {
  st_dev(reinterpret_cast<uint64_t*>(p),
         (uint64_t)__builtin_bit_cast(uint32_t, a) |
             ((uint64_t)__builtin_bit_cast(uint32_t, b) << 32));
}
FPH_DEVINL void ld2_dev(const double* p, double& a, double& b) {
  a = __builtin_bit_cast(double, ld_dev(reinterpret_cast<const uint64_t*>(p)));
  b = __builtin_bit_cast(double, ld_dev(reinterpret_cast<const uint64_t*>(p) + 1));
}
FPH_DEVINL void st2_dev(double* p, double a, double b) {
  st_dev(reinterpret_cast<uint64_t*>(p), __builtin_bit_cast(uint64_t, a));
  st_dev(reinterpret_cast<uint64_t*>(p) + 1, __builtin_bit_cast(uint64_t, b));
}

// ------------------------------------------------------------ functors

// Phase A input: p = r + beta p_old formed on the fly; the owner stores p.
struct InCoopDir {
  const float* r;
  const float* pold;
  float* pnew;
  float beta;
  int fresh;
  static constexpr bool kPrefetch = true;
  struct Raw {
    float z0, z1, a0, a1;
  };
  FPH_DEVINL void fetch2(long off, Raw& w, bool) const {
    float z0, z1, a0 = 0.f, a1 = 0.f;
    ld2_dev(r + off, z0, z1);
    if (!fresh) ld2_dev(pold + off, a0, a1);
    w.z0 = z0;
    w.z1 = z1;
    w.a0 = a0;
    w.a1 = a1;
  }
  FPH_DEVINL void use2(long off, const Raw& w, float& a, float& b, bool owned, bool) const {
    a = w.z0;
    b = w.z1;
    if (!fresh) {
      a += beta * w.a0;
      b += beta * w.a1;
    }
    if (owned) st2_dev(pnew + off, a, b);
  }
};

// Phase A output: Ap (owner only) and p . Ap.
struct EpiCoopAp {
  float* Ap;
  FPH_DEVINL void put2(long off, float o0, float o1, float v0, float v1, double& acc,
                       double&) const {
    st2(Ap + off, o0, o1);
    acc += (double)v0 * (double)o0 + (double)v1 * (double)o1;
  }
};

// FP64 u read coherently (halo slices come from the neighbours).
struct InCoopU {
  const double* u;
  static constexpr bool kPrefetch = true;
  struct Raw {
    double a, b;
  };
  FPH_DEVINL void fetch2(long off, Raw& w, bool) const {
    double a, b;
    ld2_dev(u + off, a, b);
    w.a = a;
    w.b = b;
  }
  FPH_DEVINL void use2(long, const Raw& w, double& a, double& b, bool, bool) const {
    a = w.a;
    b = w.b;
  }
};

// r = b - A u in FP64, stored as FP32; |r|^2 and |b|^2.
struct EpiCoopResidual {
  const double* b;
  float* r;
  FPH_DEVINL void put2(long off, double o0, double o1, double, double, double& acc,
                       double& acc2) const {
    double b0, b1;
    ld2(b + off, b0, b1);
    const double r0 = b0 - o0, r1 = b1 - o1;
    st2_dev(r + off, (float)r0, (float)r1);
    acc += r0 * r0 + r1 * r1;
    acc2 += b0 * b0 + b1 * b1;
  }
};

// ---------------------------------------------------------- exchange

struct CoopExchange {
  uint64_t* slots;   // [kRegions][kCoopMaxBlocks][2]
  uint64_t* abort;   // nonzero: leave
  int nblk;
};

// Publish (v0, v1) for this workgroup in the region of `phase` and wait for
// all workgroups; totals in tot[0..1] for every thread.  Returns false when
// the solve is aborted (a wait ran over its limit somewhere).  Call from
// every thread after this thread's global stores of the phase.
template <int NT>
FPH_DEVINL bool coop_exchange(const CoopExchange& x, int phase, int blk, double v0, double v1,
                              double* red_sh, double* tot_sh, int* ok_sh, double tot[2]) {
  // This thread's stores have been performed before the workgroup arrives.
  __builtin_amdgcn_s_waitcnt(0);
  const double s0 = block_sum<NT>(v0, red_sh);
  const double s1 = block_sum<NT>(v1, red_sh);
  uint64_t* region = x.slots + (long)(phase % kRegions) * kCoopMaxBlocks * 2;
  uint64_t* old = x.slots + (long)((phase + kRegions - 2) % kRegions) * kCoopMaxBlocks * 2;
  if (threadIdx.x == 0) {
    st_dev(old + 2 * blk, kEmptySlot);
    st_dev(old + 2 * blk + 1, kEmptySlot);
    st_dev(region + 2 * blk, __builtin_bit_cast(uint64_t, s0));
    st_dev(region + 2 * blk + 1, __builtin_bit_cast(uint64_t, s1));
  }
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    double a = 0.0, b = 0.0;
    int good = 1;
    for (int k0 = 0; k0 < x.nblk; k0 += 64) {
      const int k = k0 + lane;
      uint64_t w0 = 0, w1 = 0;
      long polls = 0;
      while (true) {
        bool ready = true;
        if (k < x.nblk) {
          w0 = ld_dev(region + 2 * k);
          w1 = ld_dev(region + 2 * k + 1);
          ready = (w0 != kEmptySlot) && (w1 != kEmptySlot);
        }
        // the wave leaves the loop together
        const bool all = __all(ready);
        if (all) break;
        if (++polls > kPollLimit || ld_dev(x.abort) != 0) {
          good = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
      if (!good) break;
      if (k < x.nblk) {
        a += __builtin_bit_cast(double, w0);
        b += __builtin_bit_cast(double, w1);
      }
    }
    if (!good && lane == 0) st_dev(x.abort, 1);
    for (int off = 32; off > 0; off >>= 1) {
      a += __shfl_xor(a, off, 64);
      b += __shfl_xor(b, off, 64);
    }
    if (lane == 0) {
      tot_sh[0] = a;
      tot_sh[1] = b;
      *ok_sh = good;
    }
  }
  __syncthreads();
  tot[0] = tot_sh[0];
  tot[1] = tot_sh[1];
  const bool ok = *ok_sh != 0;
  __syncthreads();
  return ok;
}

// --------------------------------------------------------------- kernel

// Result of a cooperative solve (written by workgroup 0, thread 0).
struct CoopStats {
  int status, iters, outer, matvecs;
  double rr_true, bb;
};

struct CoopArgs {
  Geom g;
  float th32;   // tanh(dtau t) (the E buffers hold ch^4 E)
  double th;
  const float* E32;
  const double* E64;
  const double* b;
  double* u;
  float* r;
  float* pa;
  float* pb;
  float* Ap;
  float* u32;
  CoopExchange x;
  CoopStats* out;   // final statistics (written by workgroup 0)
  int Tch;          // slices per chunk
  double tol;
  int maxiter;
  double delta;     // residual-replacement factor (adapted as in pcg_solve)
  int zero_guess;
};

// Owned element pairs of a workgroup: slices [s0, s1) of the (single)
// right-hand side, N/2 pairs each.
template <int NT, class F>
FPH_DEVINL void for_owned_pairs(const Geom& g, int s0, int s1, F&& f) {
  const long p0 = (long)s0 * g.N / 2, p1 = (long)s1 * g.N / 2;
  for (long p = p0 + threadIdx.x; p < p1; p += NT) f(2 * p);
}

// Launch: cooperative, grid = ceil(ceil(Ltau / Tch) / S) workgroups of NT
// threads (S = NT / Q chunks side by side), at most kCoopMaxBlocks.
// Dynamic LDS: 4 * S * N doubles.
template <int NT>
__global__ void __launch_bounds__(NT) k_cg_coop(CoopArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red_sh[NT / 64];
  __shared__ double tot_sh[2];
  __shared__ int ok_sh;
  const Geom& g = a.g;
  const int blk = blockIdx.x;
  int S, sub, lane, nslot;
  block_layout<NT>(g, threadIdx.x, S, sub, lane, nslot);
  const int chunk = blk * S + sub;
  const int tau0 = chunk * a.Tch;
  const bool active = (sub < S) && (tau0 < g.Ltau);
  const int Tc = active ? min(a.Tch, g.Ltau - tau0) : 0;
  const int own0 = min(g.Ltau, blk * S * a.Tch);
  const int own1 = min(g.Ltau, (blk + 1) * S * a.Tch);
  void* lds = smem_raw + (size_t)(sub < S ? sub : 0) * 4 * g.N * sizeof(double);
  auto no_hook = [] { return true; };
  int phase = 0;
  double tot[2];

  // FP64 residual of the current u64 into r (FP32); returns |r|^2, |b|^2.
  auto residual = [&](double& rr, double& bb) -> bool {
    double acc = 0.0, acc2 = 0.0;
    InCoopU in{a.u};
    EpiCoopResidual epi{a.b, a.r};
    mtm_sweep<double, NT, 1, 2>(g, a.E64, a.th, a.Tch, tau0, Tc, active, lane, nslot,
                                reinterpret_cast<double*>(lds), 0, in, epi, acc, acc2, no_hook);
    const bool ok = coop_exchange<NT>(a.x, phase++, blk, acc, acc2, red_sh, tot_sh, &ok_sh, tot);
    rr = tot[0];
    bb = tot[1];
    return ok;
  };

  // Start: u64 = 0 for a zero guess, u32 = 0; wait for every u64, then
  // r = b - A u64.
  for_owned_pairs<NT>(g, own0, own1, [&](long o) {
    if (a.zero_guess) st2_dev(a.u + o, 0.0, 0.0);
    st2(a.u32 + o, 0.f, 0.f);
  });
  bool ok = coop_exchange<NT>(a.x, phase++, blk, 0.0, 0.0, red_sh, tot_sh, &ok_sh, tot);
  double rr = 0.0, bb = 0.0;
  if (ok) ok = residual(rr, bb);
  const double tol2 = a.tol * a.tol * bb;
  double rr_true = rr;
  int matvecs = 1;
  int status = 0;
  if (!(bb >= 0.0) || !isfinite(bb) || !isfinite(rr)) status = 8;
  if (status == 0 && rr <= tol2) status = 1;
  double rz = rr, delta = a.delta, ru_thresh = delta * delta * rr, beta = 0.0;
  int fresh = 1, iter = 0, outer = 0;

  while (ok && status == 0) {
    const bool odd = (iter & 1) != 0;
    float* pold = odd ? a.pb : a.pa;
    float* pnew = odd ? a.pa : a.pb;
    // A: direction, operator, p.Ap
    {
      double acc = 0.0, acc2 = 0.0;
      InCoopDir in{a.r, pold, pnew, (float)beta, fresh};
      EpiCoopAp epi{a.Ap};
      mtm_sweep<float, NT, 1, 2>(g, a.E32, a.th32, a.Tch, tau0, Tc, active, lane, nslot,
                                 reinterpret_cast<float*>(lds), 0, in, epi, acc, acc2, no_hook);
      ok = coop_exchange<NT>(a.x, phase++, blk, acc, 0.0, red_sh, tot_sh, &ok_sh, tot);
      if (!ok) break;
    }
    matvecs += 1;
    const double pAp = tot[0];
    if (!(pAp > 0.0) || !isfinite(pAp)) {
      status = isfinite(pAp) ? 4 : 8;
      break;
    }
    // B: update
    {
      const float alpha = (float)(rz / pAp);
      double acc = 0.0;
      for_owned_pairs<NT>(g, own0, own1, [&](long o) {
        float p0, p1, q0, q1, r0, r1, x0, x1;
        ld2_dev(pnew + o, p0, p1);
        ld2(a.Ap + o, q0, q1);
        ld2_dev(a.r + o, r0, r1);
        ld2(a.u32 + o, x0, x1);
        r0 -= alpha * q0;
        r1 -= alpha * q1;
        st2(a.u32 + o, x0 + alpha * p0, x1 + alpha * p1);
        st2_dev(a.r + o, r0, r1);
        acc += (double)r0 * (double)r0 + (double)r1 * (double)r1;
      });
      ok = coop_exchange<NT>(a.x, phase++, blk, acc, 0.0, red_sh, tot_sh, &ok_sh, tot);
      if (!ok) break;
    }
    const double rr_it = tot[0];
    iter += 1;
    if (!isfinite(rr_it)) {
      status = 8;
      break;
    }
    if (!(rr_it <= tol2 || rr_it < ru_thresh || iter >= a.maxiter)) {
      beta = rr_it / rz;
      rz = rr_it;
      fresh = 0;
      continue;
    }
    // FP64 residual replacement.
    for_owned_pairs<NT>(g, own0, own1, [&](long o) {
      double u0, u1;
      float x0, x1;
      ld2_dev(a.u + o, u0, u1);
      ld2(a.u32 + o, x0, x1);
      st2_dev(a.u + o, u0 + (double)x0, u1 + (double)x1);
      st2(a.u32 + o, 0.f, 0.f);
    });
    ok = coop_exchange<NT>(a.x, phase++, blk, 0.0, 0.0, red_sh, tot_sh, &ok_sh, tot);
    if (!ok) break;
    double rt = 0.0, bdummy = 0.0;
    ok = residual(rt, bdummy);
    if (!ok) break;
    matvecs += 1;
    rr_true = rt;
    outer += 1;
    if (!isfinite(rt)) {
      status = 8;
      break;
    }
    if (rt <= tol2) {
      status = 1;
      break;
    }
    if (iter >= a.maxiter) {
      status = 2;
      break;
    }
    if (rt > 100.0 * rr_it) fresh = 1;
    if (rt > 4.0 * rr_it) delta = fmin(0.5, sqrt(delta));
    ru_thresh = delta * delta * rt;
    beta = fresh ? 0.0 : rt / rz;
    rz = rt;
  }
  if (blk == 0 && threadIdx.x == 0) {
    CoopStats r;
    r.status = ok ? status : (status | 16);
    r.iters = iter;
    r.outer = outer;
    r.matvecs = matvecs;
    r.rr_true = rr_true;
    r.bb = bb;
    *a.out = r;
  }
}

// Fill n 8-byte words with v (the exchange regions before a launch).
__global__ void k_fill_u64(uint64_t* p, long n, uint64_t v) {
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x)
    p[k] = v;
}

}  // namespace fph
