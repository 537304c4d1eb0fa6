// Batched solves of many independent systems in one persistent launch.
//
// A work item is one (system, right-hand side) pair.  Each workgroup takes
// items from a queue (one atomic add per item, items sorted by size,
// largest first) and runs the whole solve of its item: FP32 (preconditioned)
// conjugate gradients on M^T M (the operator sweep of fph_matvec.h over all
// slices of the item, chunks side by side in the block; with the
// preconditioner, z = F F^T r by fph_batch_pc.h in the same workgroup), and,
// whenever the FP32 residual has fallen by `delta` or below the tolerance,
// an FP64 residual replacement: u64 += u32, r = b - M^T M u64 evaluated in
// FP64 with the FP64 field, iteration continues with the replaced residual.
// All reductions are workgroup-local, so no workgroup ever waits for
// another; every workgroup leaves when the queue is empty.
#pragma once

#include "fph_batch_pc.h"
#include "fph_blas.h"
#include "fph_common.h"
#include "fph_matvec.h"

namespace fph {

struct BatchItem {
  Geom g;
  double th;              // tanh(dtau t); E64/E32 hold ch^4 E
  const double* E64;      // [Ltau][N] of the item's system
  const float* E32;
  const double* b;        // right-hand side [Ltau][N]
  double* u;              // solution (FP64)
  float* r;               // FP32 workspace, d values each
  float* pa;
  float* pb;
  float* Ap;
  float* u32;
  float* z;               // preconditioned direction input z = F F^T r
  float2* Zw;             // transform workspace, [H][N] complex (d floats)
  BatchPc pc;             // the system's preconditioner tables
  int out;                // index into the statistics array
  int pad;
};

struct BatchStat {
  int status, iters, outer, matvecs;
  double rel_resid, action;
};

// Sum over the block, returned to every thread.
template <int NT>
FPH_DEVINL double block_allsum(double v, double* sh, double* bcast) {
  const double s = block_sum<NT>(v, sh);
  if (threadIdx.x == 0) *bcast = s;
  __syncthreads();
  const double out = *bcast;
  __syncthreads();
  return out;
}

// z = F F^T r for one item (fph_batch_pc.h); returns r . z in every thread.
template <int NT>
FPH_DEVINL double bpc_apply(const BatchItem& it, const float* r, float* z, unsigned char* lds,
                            double* red_sh, double* bcast) {
  float2* l = reinterpret_cast<float2*>(lds);
  bpc_forward<NT>(it.g, it.pc, r, it.Zw, l);
  bpc_series<NT>(it.g, it.pc, (float)it.th, it.Zw, l);
  const double part = bpc_inverse<NT>(it.g, it.pc, it.Zw, r, z, l);
  return block_allsum<NT>(part, red_sh, bcast);
}

// Input: p = z + beta p_old on the fly (fresh: p = z); owner stores p.
template <typename T>
struct InDir {
  const T* __restrict__ z;
  const T* __restrict__ pold;
  T* __restrict__ pnew;
  T beta;
  int fresh;
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
  // loads issued ahead, p formed (and stored by the owner) where used
  static constexpr bool kPrefetch = true;
  struct Raw {
    T z0, z1, a0, a1;
  };
  FPH_DEVINL void fetch2(long off, Raw& w, bool) const {
    T z0, z1, a0 = (T)0, a1 = (T)0;
    ld2(z + off, z0, z1);
    if (!fresh) ld2(pold + off, a0, a1);
    w.z0 = z0;
    w.z1 = z1;
    w.a0 = a0;
    w.a1 = a1;
  }
  FPH_DEVINL void use2(long off, const Raw& w, T& a, T& b, bool owned, bool) const {
    a = w.z0;
    b = w.z1;
    if (!fresh) {
      a += beta * w.a0;
      b += beta * w.a1;
    }
    if (owned) st2(pnew + off, a, b);
  }
};

template <int NT, int MS>
FPH_DEVINL void batch_solve_item(const BatchItem& it, double tol, int maxiter, double delta,
                                 int pre, unsigned char* lds, double* red_sh, double* bcast,
                                 BatchStat* stats) {
  const Geom& g = it.g;
  const long d = g.d;
  int S, sub, lane, nslot;
  block_layout<NT>(g, threadIdx.x, S, sub, lane, nslot);
  const int Tch = (g.Ltau + S - 1) / S;
  const int tau0 = sub * Tch;
  const bool active = (sub < S) && (tau0 < g.Ltau);
  const int Tc = active ? min(Tch, g.Ltau - tau0) : 0;
  const int so = (sub < S) ? sub : 0;
  // The direction update reads z = F F^T r with the preconditioner, r without.
  const float* zdir = pre ? it.z : it.r;

  // Initial state: u = 0, r = b.
  double bb = 0.0, rr = 0.0;
  for (long k = threadIdx.x; k < d; k += NT) {
    const double bv = it.b[k];
    const float rv = (float)bv;
    it.u[k] = 0.0;
    it.u32[k] = 0.0f;
    it.r[k] = rv;
    bb += bv * bv;
    rr += (double)rv * (double)rv;
  }
  bb = block_allsum<NT>(bb, red_sh, bcast);
  rr = block_allsum<NT>(rr, red_sh, bcast);
  const double tol2 = tol * tol * bb;
  double rz = rr, rr_ref = rr, rr_true = bb, beta = 0.0;
  int fresh = 1, iter = 0, outer = 0, matvecs = 0, status = 0;
  float* pold = it.pa;
  float* pnew = it.pb;
  if (bb == 0.0) status = 1;
  if (!isfinite(bb)) status = 8;
  if (status == 0 && pre) {
    rz = bpc_apply<NT>(it, it.r, it.z, lds, red_sh, bcast);
    if (!(rz > 0.0) || !isfinite(rz)) status = isfinite(rz) ? 4 : 8;
  }

  while (status == 0) {
    // Direction update fused into the operator: Ap = A (z + beta p).
    {
      float* lds4 = reinterpret_cast<float*>(lds) + 4L * so * g.N;
      InDir<float> in{zdir, pold, pnew, (float)beta, fresh};
      EpiDot<float> epi{it.Ap};
      double acc = 0.0, acc2 = 0.0;
      mtm_sweep<float, NT, MS, 1>(g, it.E32, (float)it.th, Tch, tau0, Tc, active,
                                  lane, nslot, lds4, 0, in, epi, acc, acc2, [] { return true; });
      const double pAp = block_allsum<NT>(acc, red_sh, bcast);
      matvecs += 1;
      if (!(pAp > 0.0) || !isfinite(pAp)) {
        status = isfinite(pAp) ? 4 : 8;
        break;
      }
      const float alpha = (float)(rz / pAp);
      double acc_rr = 0.0;
      for (long k = threadIdx.x; k < d; k += NT) {
        const float rv = it.r[k] - alpha * it.Ap[k];
        it.u32[k] += alpha * pnew[k];
        it.r[k] = rv;
        acc_rr += (double)rv * (double)rv;
      }
      rr = block_allsum<NT>(acc_rr, red_sh, bcast);
    }
    iter += 1;
    fresh = 0;
    float* t = pold;
    pold = pnew;
    pnew = t;
    if (!isfinite(rr)) {
      status = 8;
      break;
    }
    if (!(rr <= tol2 || rr < delta * delta * rr_ref || iter >= maxiter)) {
      const double rz_new = pre ? bpc_apply<NT>(it, it.r, it.z, lds, red_sh, bcast) : rr;
      if (!(rz_new > 0.0) || !isfinite(rz_new)) {
        status = isfinite(rz_new) ? 4 : 8;
        break;
      }
      beta = rz_new / rz;
      rz = rz_new;
      continue;
    }

    // FP64 residual replacement.
    const double rr_iter = rr;
    for (long k = threadIdx.x; k < d; k += NT) {
      it.u[k] += (double)it.u32[k];
      it.u32[k] = 0.0f;
    }
    __syncthreads();
    {
      double* lds4 = reinterpret_cast<double*>(lds) + 4L * so * g.N;
      InPlain<double> in{it.u};
      EpiResidual<float> epi{it.b, it.r};
      double acc = 0.0, acc2 = 0.0;
      mtm_sweep<double, NT, MS, 1>(g, it.E64, it.th, Tch, tau0, Tc, active, lane, nslot,
                                   lds4, 0, in, epi, acc, acc2, [] { return true; });
      rr_true = block_allsum<NT>(acc, red_sh, bcast);
    }
    matvecs += 1;
    outer += 1;
    if (rr_true <= tol2) {
      status = 1;
      break;
    }
    if (iter >= maxiter) {
      status = 2;
      break;
    }
    double acc_rr = 0.0;
    for (long k = threadIdx.x; k < d; k += NT) {
      const double rv = it.r[k];
      acc_rr += rv * rv;
    }
    rr = block_allsum<NT>(acc_rr, red_sh, bcast);
    if (rr > 100.0 * rr_iter) fresh = 1;  // replaced residual far from the iterated one
    const double rz_new = pre ? bpc_apply<NT>(it, it.r, it.z, lds, red_sh, bcast) : rr;
    if (!(rz_new > 0.0) || !isfinite(rz_new)) {
      status = isfinite(rz_new) ? 4 : 8;
      break;
    }
    beta = rz_new / rz;
    rz = rz_new;
    rr_ref = rr;
  }

  // S_F = b . u in FP64.
  double act = 0.0;
  for (long k = threadIdx.x; k < d; k += NT) act += it.b[k] * it.u[k];
  act = block_allsum<NT>(act, red_sh, bcast);
  if (threadIdx.x == 0) {
    BatchStat st;
    st.status = status;
    st.iters = iter;
    st.outer = outer;
    st.matvecs = matvecs;
    st.rel_resid = bb > 0.0 ? sqrt(rr_true / bb) : 0.0;
    st.action = act;
    stats[it.out] = st;
  }
  __syncthreads();
}

// Persistent batched solve.  Launch: any number of blocks of NT threads;
// LDS: the larger of 4 * S * Nmax doubles (S = NT / Qmax chunks) and, with
// the preconditioner (pre != 0, NT >= Qmax), the transforms' and the
// series' needs (bpc_lds_tf, bpc_lds_series).  `queue` must be 0.
template <int NT, int MS>
__global__ void __launch_bounds__(NT)
k_batch_solve(const BatchItem* __restrict__ items, int nitems, unsigned* queue, double tol,
              int maxiter, double delta, int pre, BatchStat* stats) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red_sh[NT / 64];
  __shared__ double bcast;
  __shared__ int item_sh;
  while (true) {
    if (threadIdx.x == 0) item_sh = (int)atomicAdd(queue, 1u);
    __syncthreads();
    const int k = item_sh;
    __syncthreads();
    if (k >= nitems) break;
    batch_solve_item<NT, MS>(items[k], tol, maxiter, delta, pre, smem_raw, red_sh, &bcast, stats);
  }
}

__global__ void k_zero_u32(unsigned* p) { *p = 0u; }

}  // namespace fph
