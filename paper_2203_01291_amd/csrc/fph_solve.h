// Device-controlled (P)CG solve (Eqs. CG, CG_precon on M^T M).
//
// A solve is a fixed sequence of launches that the host enqueues without
// reading anything back: a start kernel, then "slots", then two final
// kernels.  Every slot has the same launches, and the per right-hand-side
// state (fph_common.h) decides what each one does:
//
//   operator kernel (k_slot_mtm), one of
//     - a CG iteration's direction update and operator: p = z + beta p_old,
//       Ap = M^T M p, partials p.Ap;
//     - an FP64 residual evaluation r = b - M^T M u with the FP64 field
//       (at the start, when the iterated residual reached the tolerance or
//       fell by the replacement factor, or at the iteration cap), partials
//       |r|^2 and |b|^2;
//     - nothing (finished, or paused);
//   then, without the preconditioner, k_cg_update (u += alpha p,
//   r -= alpha Ap, |r|^2; or, after a residual evaluation, only the decision
//   that folds it); with it, the forward transform with the same update,
//   the Chebyshev series F F^T and the inverse transform with r.z.
//
// A slot performs one CG iteration or one residual evaluation, so a solve
// that may run `maxiter` iterations and `max_outer` evaluations after the
// first fits in 1 + maxiter + max_outer slots; slots after convergence
// return at once.  The decisions are taken in the kernels that fold the
// partial sums (state_begin), identically in every workgroup.
//
// FP32-refined (reliable updates of the residual, Sleijpen and van der
// Vorst 1996; the mixed-precision form of Clark et al. 2010): the iteration
// runs in FP32 on a correction u32; the FP64 iterate lives in u_dev and a
// workspace buffer alternately: each residual evaluation reads
// u64 + u32 (on the fly, halo slices included) and its chunk owners write
// the sum to the other buffer, which becomes the iterate; the correction
// restarts from zero.  The final kernel moves the iterate into u_dev.
#pragma once

#include "fph_blas.h"
#include "fph_common.h"
#include "fph_matvec.h"

namespace fph {

// Statistics written to device memory (same layout as fph_pcg_stats_t).
struct PcgStatsDev {
  int status, iters, outer_iters, matvecs;
  double rel_resid, action;
};

// Arguments of the operator kernel of a slot, TI the iteration precision.
template <typename TI>
struct SlotArgs {
  const TI* E;         // field of the iteration (ch^4 E, rounded for FP32)
  const double* E64;   // FP64 field of the residual evaluations
  TI th;
  double th64;
  const TI* z;         // z = F F^T r (preconditioned) or r
  TI* pa;
  TI* pb;
  TI* Ap;
  const double* b;
  TI* r;               // receives an evaluated residual (rounded for FP32)
  double* u;           // u_dev: the FP64 iterate (FP64 solves update it in place)
  double* u64b;        // FP32-refined: the second FP64 buffer
  const float* u32;    // FP32-refined: the FP32 correction
};

// Launch: as k_mtm, grid nblk * nrhs, LDS 4 * S * N doubles (the residual
// path runs in FP64).  Takes part in the state sequence (io).  PF: prefetch
// ahead of the state (see below).
template <typename TI, int NT, int MS, bool PF>
__global__ void __launch_bounds__(NT)
k_slot_mtm(Geom g, int Tch, int nblk, SlotArgs<TI> a, StIO io) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red_sh[NT / 64];
  __shared__ RhsState s_sh;
  int r, bx;
  mtm_block(nblk, r, bx);
  // The state loads go first and the state is folded in the sweep's hook.
  // With PF (small systems, where the kernel is latency bound) the first
  // slices of a CG iteration (z and both direction buffers, as the parity
  // is not known yet) are loaded while the state is in flight; a slot that
  // turns out to evaluate the residual, or to have nothing to do, drops
  // those loads.
  StLoad<(PF ? 8 : 16)> sl;
  state_issue(io, r, sl);
  const long fo = field_off(g, r);
  int S, sub, lane, nslot;
  block_layout<NT>(g, threadIdx.x, S, sub, lane, nslot);
  const int chunk = bx * S + sub;
  const int tau0 = chunk * Tch;
  const bool active = (sub < S) && (tau0 < g.Ltau);
  const int Tc = active ? min(Tch, g.Ltau - tau0) : 0;
  const long base = (long)r * g.d;
  const long lo = 4L * (sub < S ? sub : 0) * g.N;
  double acc = 0.0, acc2 = 0.0;
  int path = 0;
  {
    InPUpdate<TI, PF> in{a.z, a.pa, a.pb, nullptr, nullptr, (TI)0, 0};
    EpiDot<TI> epi{a.Ap};
    auto hook = [&]() {
      state_finish<NT>(io, r, sl, &s_sh);
      path = s_sh.final_ ? 0 : (s_sh.replace ? 2 : (s_sh.done ? 0 : 1));
      if (path != 1) return false;
      in.begin(s_sh);
      return true;
    };
    if (mtm_sweep<TI, NT, MS, 1>(g, a.E + fo, a.th, Tch, tau0, Tc, active, lane, nslot,
                                 reinterpret_cast<TI*>(smem_raw) + lo, base, in, epi, acc, acc2,
                                 hook)) {
      const double bs = block_sum<NT, true>(acc, red_sh);
      // The direction update enters the state only now: every thread read
      // the state (in.begin) before the block sum's barrier.
      if (threadIdx.x == 0) InPUpdate<TI, PF>::on_state(s_sh);
      state_end(io, r, &s_sh, P_PAP, bs, bx, nblk, bx == 0);
      return;
    }
  }
  if (path == 0) {
    state_end(io, r, &s_sh, P_NONE, 0.0, bx, nblk, bx == 0);
    return;
  }
  auto no_hook = [] { return true; };
  EpiResidual<TI> epi{a.b, a.r};
  double* lds4 = reinterpret_cast<double*>(smem_raw) + lo;
  if constexpr (sizeof(TI) == 4) {
    InResid in{a.u, a.u64b, a.u32, nullptr, nullptr, 0};
    in.begin(s_sh);
    mtm_sweep<double, NT, MS, 1>(g, a.E64 + fo, a.th64, Tch, tau0, Tc, active, lane, nslot,
                                 lds4, base, in, epi, acc, acc2, no_hook);
  } else {
    InPlain<double> in{a.u};
    mtm_sweep<double, NT, MS, 1>(g, a.E64 + fo, a.th64, Tch, tau0, Tc, active, lane, nslot,
                                 lds4, base, in, epi, acc, acc2, no_hook);
  }
  const double bs = block_sum<NT>(acc, red_sh);
  const double bs2 = block_sum<NT, true>(acc2, red_sh);
  state_end(io, r, &s_sh, P_RES, bs, bx, nblk, bx == 0, bs2);
}

// Initial state of a solve: the first slot evaluates the residual of the
// initial guess (and |b|^2).  Writes the state copy the first slot reads.
struct SolveInit {
  double tol;
  double rdelta;   // FP32-refined replacement factor
  int maxiter;
  int max_outer;
  int refined;
  int pad;
};

__global__ void k_solve_init(int nrhs, SolveInit p, RhsState* st) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrhs) return;
  RhsState s;
  memset(&s, 0, sizeof(s));
  s.tol = p.tol;
  s.rdelta = p.rdelta;
  s.maxiter = p.maxiter;
  s.max_outer = p.max_outer;
  s.refined = p.refined;
  s.fresh = 1;
  s.done = 1;
  s.replace = 1;
  s.u32z = 1;
  s.pend = P_NONE;
  st[r] = s;
}

// v[0..n) = 0 (a fill kernel rather than a memset, so that a captured
// solve holds kernel nodes only).
__global__ void k_fill_zero(long n, double* __restrict__ v) {
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n;
       k += (long)gridDim.x * blockDim.x)
    v[k] = 0.0;
}

// The solution in u_dev and the partials of S_F = b . u (FP64).
// FP32-refined: u_dev = u64[upar] + u32 (the correction only if non-zero),
// so a right-hand side that stopped between evaluations (breakdown) still
// returns its latest iterate.  b = 0: u = 0 exactly.  Launch: grid
// (nb, nrhs), 256 threads; reads the latest state copy.
__global__ void __launch_bounds__(256)
k_solve_final(long d, const RhsState* __restrict__ st, const double* __restrict__ b, double* u,
              const double* u64b, const float* __restrict__ u32, double* __restrict__ part) {
  __shared__ double red_sh[4];
  const int r = blockIdx.y;
  const RhsState& s = st[r];
  const bool zero = s.started && s.bb == 0.0;
  const bool from_ws = s.refined && s.upar == 1;
  const bool add32 = s.refined && !s.u32z;
  const bool write = zero || from_ws || add32;
  const long off = (long)r * d;
  double acc = 0.0;
  for (long k = 4 * (blockIdx.x * 256L + threadIdx.x); k < d; k += 4L * gridDim.x * 256) {
    auto uu = Vec4<double>::ld((from_ws ? u64b : u) + off + k);
    if (add32) {
      const float4 c = Vec4<float>::ld(u32 + off + k);
      uu.x += (double)c.x; uu.y += (double)c.y; uu.z += (double)c.z; uu.w += (double)c.w;
    }
    if (zero) uu = Vec4<double>::V{0.0, 0.0, 0.0, 0.0};
    if (write) Vec4<double>::st(u + off + k, uu);
    const auto bv = Vec4<double>::ld(b + off + k);
    acc += bv.x * uu.x + bv.y * uu.y + bv.z * uu.z + bv.w * uu.w;
  }
  const double bs = block_sum<256>(acc, red_sh);
  if (threadIdx.x == 0) part[(long)r * kPStride + blockIdx.x] = bs;
}

// Statistics of every right-hand side (one block each): a right-hand side
// that did not finish within the enqueued slots reports MAXITER.
__global__ void __launch_bounds__(256)
k_solve_stats(int nb, const RhsState* __restrict__ st, const double* __restrict__ part,
              PcgStatsDev* __restrict__ out) {
  __shared__ double red_sh[4];
  const int r = blockIdx.x;
  const double act = reduce_partials<256>(part + (long)r * kPStride, nb, red_sh);
  if (threadIdx.x == 0) {
    const RhsState s = st[r];
    PcgStatsDev o;
    o.status = s.final_ ? s.status : (s.status | 2);
    o.iters = s.iter;
    o.outer_iters = s.outer;
    o.matvecs = s.matvecs;
    o.rel_resid = s.bb > 0.0 ? sqrt(s.rr_true / s.bb) : 0.0;
    o.action = act;
    out[r] = o;
  }
}

// Number of right-hand sides not finished (one wave), stored to pinned host
// memory (a system-scope vector store): read by the blocking driver, which
// stops enqueueing once a solve is done.
__global__ void __launch_bounds__(64)
k_solve_open(int nrhs, const RhsState* __restrict__ st, int* __restrict__ open) {
  int n = 0;
  for (int r = threadIdx.x; r < nrhs; r += 64) n += st[r].final_ ? 0 : 1;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) n += __shfl_xor(n, off, 64);
  if (threadIdx.x == 0) __hip_atomic_store(open, n, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

}  // namespace fph
