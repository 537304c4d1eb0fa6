// Shared device-side definitions of the gfx950 fermion solver.
//
// Layout (everything site-fastest): a right-hand side is [Ltau][N] with
// site i = x + L*y; several right-hand sides follow each other.  The field
// enters only through E[tau][i] = exp(-dtau*(alpha*x - mu)).
//
// Checkerboard: C = P_A P_B (P_B acts first).  P_A mixes the four sites of
// each plaquette with even corner (x0, y0); P_B those with odd corner,
// wrapping periodically.  Each plaquette factor is kron(C2, C2) with
// C2 = [[ch, sh], [sh, ch]], ch = cosh(dtau t), sh = sinh(dtau t)
// (Sec. II D of the paper; the split itself is the reading documented with
// the C header).  Both factors are symmetric, so C^T = P_B P_A.
//
// Thread mapping used by every operator kernel: a thread owns one or more
// plaquettes of the even grid ("even layout": sites (x0,y0), (x0+1,y0),
// (x0,y0+1), (x0+1,y0+1), x0, y0 even) and, for P_B, the odd plaquette whose
// corner is (x0+1, y0+1) ("odd layout").  P_A works in registers on the
// even layout, P_B on the odd layout; switching layouts goes through LDS.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define FPH_DEVINL __device__ __forceinline__

namespace fph {

// ----------------------------------------------------------------- geometry

struct Geom {
  int L;      // lattice side
  int hL;     // L / 2
  int N;      // L * L
  int Q;      // N / 4 plaquettes per slice (per group)
  int Ltau;   // time slices
  long d;     // N * Ltau elements per right-hand side
};

// Site indices of even plaquette q: (corner, +x, +y, +x+y).
FPH_DEVINL void even_sites(const Geom& g, int q, int s[4]) {
  const int x0 = 2 * (q % g.hL), y0 = 2 * (q / g.hL);
  const int i0 = x0 + g.L * y0;
  s[0] = i0;
  s[1] = i0 + 1;
  s[2] = i0 + g.L;
  s[3] = i0 + g.L + 1;
}

// Site indices of the odd plaquette with corner (x0+1, y0+1) (wrapping).
FPH_DEVINL void odd_sites(const Geom& g, int q, int s[4]) {
  const int x0 = 2 * (q % g.hL), y0 = 2 * (q / g.hL);
  const int xa = x0 + 1, ya = y0 + 1;
  const int xb = (x0 + 2 == g.L) ? 0 : x0 + 2;
  const int yb = (y0 + 2 == g.L) ? 0 : y0 + 2;
  s[0] = xa + g.L * ya;
  s[1] = xb + g.L * ya;
  s[2] = xa + g.L * yb;
  s[3] = xb + g.L * yb;
}

// kron(C2, C2) on one plaquette, local order index = dx + 2*dy.
template <typename T>
FPH_DEVINL void plaq_rot(T v[4], T ch, T sh) {
  T a0 = ch * v[0] + sh * v[1];
  T a1 = sh * v[0] + ch * v[1];
  T a2 = ch * v[2] + sh * v[3];
  T a3 = sh * v[2] + ch * v[3];
  v[0] = ch * a0 + sh * a2;
  v[2] = sh * a0 + ch * a2;
  v[1] = ch * a1 + sh * a3;
  v[3] = sh * a1 + ch * a3;
}

// ------------------------------------------------------------ solver state

// Per right-hand-side scalars of a CG solve, resident in device memory.
// Written only by the last workgroup of a reduction (see last_block()).
struct RhsState {
  double bb;        // |b|^2
  double rr;        // |r|^2 (current residual, iterated)
  double rz;        // r . z
  double rz_prev;   // r . z of the previous iteration
  double pAp;       // p . A p
  double alpha;     // rz / pAp
  double beta;      // rz / rz_prev
  double rr_ref;    // |r|^2 at the last FP64 residual recomputation
  double rr_true;   // |b - A u|^2 from the last FP64 recomputation
  double tol2;      // tol^2 * bb
  double ru_thresh; // >0: pause (done = 1) once rr < ru_thresh, so the host
                    // can replace the FP32 residual by the FP64 one
  int iter;         // CG iterations done
  int done;         // nonzero: kernels skip this right-hand side
  int status;       // FPH_ST_* bits
  int fresh;        // 1: next direction update starts p = z
  int matvecs;
  int maxiter;
};

// Device constants of the preconditioner for the current field.
struct PcInfo {
  double bmin, bmax;
  double s, c;          // A = s * Bbar - c
  int maxnp;
  int pad;
};

// ------------------------------------------------------------- reductions

// Sum of one double over the workgroup; result valid in thread 0.
template <int NT>
FPH_DEVINL double block_sum(double v, double* sh) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) s += sh[w];
  }
  __syncthreads();
  return s;
}

// Arrival at a per-right-hand-side counter after this block published its
// partial sums (thread 0 wrote them).  Returns true in every thread of the
// last arriving block; that block then reduces the partials in a fixed
// order (deterministic) and resets the counter.
FPH_DEVINL bool last_block(unsigned* counter, unsigned nblocks, int* flag_sh) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    const unsigned prev = atomicAdd(counter, 1u);
    *flag_sh = (prev == nblocks - 1) ? 1 : 0;
  }
  __syncthreads();
  const bool last = *flag_sh != 0;
  if (last) __threadfence();
  return last;
}

// Deterministic sum of n partials by the whole block; result in thread 0.
template <int NT>
FPH_DEVINL double reduce_partials(const double* part, int n, double* sh) {
  double v = 0.0;
  for (int k = threadIdx.x; k < n; k += NT) v += part[k];
  return block_sum<NT>(v, sh);
}

}  // namespace fph
