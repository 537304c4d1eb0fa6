// Shared device-side definitions of the gfx950 fermion solver.
//
// Layout (everything site-fastest): a right-hand side is [Ltau][N] with
// site i = x + L*y; several right-hand sides follow each other.  The field
// enters only through E[tau][i] = exp(-dtau*(alpha*x - mu)), which the
// operator kernels read pre-multiplied by ch^4 (see below).
//
// Checkerboard: C = P_A P_B (P_B acts first).  P_A mixes the four sites of
// each plaquette with even corner (x0, y0); P_B those with odd corner,
// wrapping periodically.  Each plaquette factor is kron(C2, C2) with
// C2 = [[ch, sh], [sh, ch]], ch = cosh(dtau t), sh = sinh(dtau t)
// (Sec. II D of the paper; the split itself is the reading documented with
// the C header).  Both factors are symmetric, so C^T = P_B P_A.
//
// The kernels apply C2 = ch C2' with C2' = [[1, th], [th, 1]],
// th = tanh(dtau t): then P_A P_B = ch^4 P'_A P'_B, each output of a primed
// factor costs one fused multiply-add instead of a multiply and a
// multiply-add, and ch^4 is folded into the stored E (M's off-diagonal
// blocks are E C = (ch^4 E) C').  So every E buffer the operator kernels
// read holds ch^4 exp(-dtau (alpha x - mu)).
//
// Thread mapping used by every operator kernel: a thread owns one or more
// plaquettes of the even grid ("even layout": sites (x0,y0), (x0+1,y0),
// (x0,y0+1), (x0+1,y0+1), x0, y0 even) and, for P_B, the odd plaquette whose
// corner is (x0+1, y0+1) ("odd layout").  P_A works in registers on the
// even layout, P_B on the odd layout; switching layouts goes through LDS.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <map>
#include <mutex>
#include <utility>

#define FPH_DEVINL __device__ __forceinline__

namespace fph {

// Dynamic LDS above 48 KB needs a per-kernel opt-in.  The limit set for
// each (device, kernel) is remembered, so the launch path makes the runtime
// call only when a launch needs more than any earlier one.
inline hipError_t allow_lds(const void* kern, size_t bytes) {
  if (bytes <= 48 * 1024) return hipSuccess;
  static std::mutex mu;
  static std::map<std::pair<int, const void*>, size_t> granted;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(mu);
  size_t& have = granted[{dev, kern}];
  if (have >= bytes) return hipSuccess;
  e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e == hipSuccess) have = bytes;
  return e;
}

// ----------------------------------------------------------------- geometry

struct Geom {
  int L;        // lattice side
  int hL;       // L / 2
  int N;        // L * L
  int Q;        // N / 4 plaquettes per slice (per group)
  int Ltau;     // time slices
  long d;       // N * Ltau elements per right-hand side
  long fs = 0;  // field stride: 0 when every right-hand side shares field 0,
                // d when right-hand side r uses field r / rpf
  int rpf = 1;  // right-hand sides per field
};

// Field of right-hand side r, and the offset of its E in the field buffers.
FPH_DEVINL int field_of(const Geom& g, int r) { return g.fs ? r / g.rpf : 0; }
FPH_DEVINL long field_off(const Geom& g, int r) { return (long)field_of(g, r) * g.fs; }

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

// kron(C2', C2') on one plaquette, local order index = dx + 2*dy.
template <typename T>
FPH_DEVINL void plaq_rot(T v[4], T th) {
  const T a0 = fma(th, v[1], v[0]);
  const T a1 = fma(th, v[0], v[1]);
  const T a2 = fma(th, v[3], v[2]);
  const T a3 = fma(th, v[2], v[3]);
  v[0] = fma(th, a2, a0);
  v[2] = fma(th, a0, a2);
  v[1] = fma(th, a3, a1);
  v[3] = fma(th, a1, a3);
}

// ------------------------------------------------------------ solver state

// Workgroup i of a 1-D launch of n runs on XCD i % 8 (round-robin
// dispatch).  Returns a renumbering that is a bijection of [0, n) and gives
// each XCD a contiguous range, XCDs with one workgroup more first.
FPH_DEVINL int xcd_contiguous(int i, int n) {
  constexpr int kXcd = 8;
  const int q = n / kXcd, rem = n % kXcd;
  const int x = i % kXcd, slot = i / kXcd;
  return (x < rem) ? x * (q + 1) + slot : rem * (q + 1) + (x - rem) * q + slot;
}

// Kinds of pending partial sums: a kernel that reduces something writes one
// partial per block; the next state-aware kernel in stream order sums them
// (every block in the same order, so all blocks agree bit for bit) and
// folds the total into the state.  No kernel waits for another block.
enum Pend : int {
  P_NONE = 0,
  P_RR = 2,    // |r|^2 after a CG update (an iteration completed)
  P_PAP = 3,   // p . A p
  P_RZ = 4,    // r . z after preconditioning
  P_RES = 5    // (|b - A u|^2, |b|^2) of an FP64 residual evaluation
};

constexpr int kPStride = 4096;  // partial slots per right-hand side
constexpr int kPHalf = 2048;    // second value of two-value partials (P_RES)

// Per right-hand-side scalars of a CG solve.  Two copies alternate: a
// kernel reads copy `in` and its first block writes copy `out`.  The whole
// control of a solve lives here: the kernels of every iteration fold the
// partial sums of the previous kernel and take the same decisions in every
// block, so the host only enqueues.
struct RhsState {
  double tol;       // relative residual target
  double bb;        // |b|^2
  double tol2;      // tol^2 |b|^2
  double rr;        // |r|^2 of the iterated residual
  double rz;        // r . z of the residual that built the current direction
  double rz_next;   // r . z of the newest residual (becomes rz at the next
                    // direction update)
  double pAp;       // p . A p
  double alpha;     // rz / pAp
  double beta;      // rz_next / rz
  double rr_true;   // |b - A u|^2 from the last FP64 evaluation
  double ru_thresh; // > 0: pause once rr < ru_thresh (FP32 residual replacement)
  double rdelta;    // FP32-refined: replacement factor, lengthened when needed
  double rr_pause;  // iterated |r|^2 when the right-hand side paused
  int iter;         // CG iterations completed
  int done;         // nonzero: the CG-iteration kernels skip this right-hand side
  int status;       // FPH_ST_* bits
  int fresh;        // 1: the next direction update starts p = z
  int matvecs;
  int maxiter;
  int pend;         // Pend kind of the partials waiting in `pin`
  int npart;        // number of waiting partials
  int final_;       // 1: finished; every kernel skips it
  int replace;      // 1: the next operator kernel evaluates the FP64 residual
  int started;      // the first residual (and |b|^2) has been evaluated
  int outer;        // FP64 residual replacements after the first residual
  int max_outer;    // cap on `outer`
  int refined;      // FP32 iteration on an FP64 iterate (FP32-refined solve)
  int upar;         // refined: the FP64 iterate is in u_dev (0) or the workspace (1)
  int u32z;         // refined: the FP32 correction is zero (not written since the
                    // last replacement)
  int own;          // the pause came from the iterated residual reaching tol
  int folded;       // Pend kind the last state_begin folded (P_NONE: none)
};

struct StIO {
  const RhsState* in;  // nullptr: no solver state (plain operator call)
  RhsState* out;
  const double* pin;   // pending partials, [rhs][kPStride]
  double* pout;        // partials written by this kernel
  int precond;         // preconditioned CG (z != r)
};

// Ping-pong bookkeeping of the CG state for a sequence of launches: each
// state-aware kernel reads copy `cur`, writes copy `cur ^ 1` (and its
// partial sums, at most kPStride per right-hand side, to the partial
// buffer of the same parity).  The sequence depends only on the launches,
// never on values, so the host can enqueue a whole solve without reading
// anything back.
struct StateSeq {
  RhsState* st[2];
  double* part[2];
  int cur;
  int precond;
  bool active;  // false: plain operator calls without solver state
  StIO next() {
    if (!active) return StIO{nullptr, nullptr, nullptr, nullptr, precond};
    StIO io{st[cur], st[cur ^ 1], part[cur], part[cur ^ 1], precond};
    cur ^= 1;
    return io;
  }
  RhsState* latest() const { return st[cur]; }
};

// Device constants of the preconditioner for the current field.
struct PcInfo {
  double bmin, bmax;
  double s, c;          // A = s * Bbar - c
  int maxnp;
  int pad;
};

// ------------------------------------------------------------- reductions

// One 32-bit lane value from lane (i - n) mod 16 of the same 16-lane row
// (DPP row rotation right by n).
template <int N>
FPH_DEVINL float row_ror(float v) {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x120 + N, 0xf, 0xf, true));
}
template <int N>
FPH_DEVINL double row_ror(double v) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)(u & 0xffffffffull), 0x120 + N, 0xf, 0xf,
                                          true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(u >> 32), 0x120 + N, 0xf, 0xf, true);
  return __builtin_bit_cast(double,
                            ((unsigned long long)(unsigned)hi << 32) | (unsigned long long)(unsigned)lo);
}
// The double held by lane `lane` (uniform result).
FPH_DEVINL double readlane_d(double v, int lane) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u & 0xffffffffull), lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), lane);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | (unsigned long long)lo);
}

// Sum of v over the 64 lanes of a wave, valid in every lane: each 16-lane
// row adds its rotations by 8, 4, 2 and 1 (DPP), then the totals held by
// lanes 0, 16, 32 and 48 are added in that order.  The order of operations
// is fixed, so every wave given the same values gets the same bits.
FPH_DEVINL double wave_sum_fixed(double v) {
  v += row_ror<8>(v);
  v += row_ror<4>(v);
  v += row_ror<2>(v);
  v += row_ror<1>(v);
  return ((readlane_d(v, 0) + readlane_d(v, 16)) + readlane_d(v, 32)) + readlane_d(v, 48);
}

// Sum of one double over the workgroup; result valid in thread 0.  LAST:
// the kernel's last use of sh, so no barrier is needed after thread 0 has
// read it (the kernel ends without waiting for it at its tail).
template <int NT, bool LAST = false>
FPH_DEVINL double block_sum(double v, double* sh) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  v = wave_sum_fixed(v);
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) s += sh[w];
  }
  if (!LAST) __syncthreads();
  return s;
}

// Deterministic sum of n partials by the whole block; result in thread 0.
template <int NT>
FPH_DEVINL double reduce_partials(const double* part, int n, double* sh) {
  double v = 0.0;
  for (int k = threadIdx.x; k < n; k += NT) v += part[k];
  return block_sum<NT>(v, sh);
}

// A right-hand side stops for good with status bits `bits`.
FPH_DEVINL void rhs_finish(RhsState& s, int bits) {
  s.status |= bits;
  s.done = 1;
  s.final_ = 1;
  s.replace = 0;
}

// The iterated residual asks for an FP64 residual evaluation: the CG
// kernels skip the right-hand side until the next operator kernel has
// evaluated it.
FPH_DEVINL void rhs_pause(RhsState& s, int own) {
  s.done = 1;
  s.replace = 1;
  s.own = own;
  s.rr_pause = s.rr;
}

// Decision after an FP64 residual evaluation r = b - A u (rr = |r|^2,
// bb = |b|^2 at the first one).  FP32-refined: the evaluation also moved
// the FP64 iterate to the other buffer with the FP32 correction added, so
// the correction restarts from zero.  Continuing right-hand sides keep
// their directions (reliable update) unless the evaluated residual is far
// from the iterated one, or, in FP64, the iterated residual had claimed
// convergence; FP32-refined shortens the replacement interval (delta ->
// sqrt delta, at most 0.5) when the evaluated residual exceeds the
// iterated one more than twice.
FPH_DEVINL void rhs_after_residual(RhsState& s, double rr, double bb, int precond) {
  s.matvecs += 1;
  s.replace = 0;
  if (s.refined) {
    s.upar ^= 1;
    s.u32z = 1;
  }
  const bool first = !s.started;
  if (first) {
    s.started = 1;
    s.bb = bb;
    s.tol2 = s.tol * s.tol * bb;
    if (!isfinite(bb)) {
      s.rr_true = rr;
      rhs_finish(s, 8);
      return;
    }
    if (bb == 0.0) {  // b = 0: u = 0 exactly (the final kernel writes it)
      s.rr_true = 0.0;
      rhs_finish(s, 1);
      return;
    }
  } else {
    s.outer += 1;
  }
  s.rr_true = rr;
  s.rr = rr;
  if (!precond) s.rz_next = rr;
  if (!isfinite(rr)) {
    rhs_finish(s, 8);
    return;
  }
  if (rr <= s.tol2) {
    rhs_finish(s, 1);
    return;
  }
  if (s.iter >= s.maxiter || s.outer >= s.max_outer) {
    rhs_finish(s, 2);
    return;
  }
  if (first) {
    s.fresh = 1;
  } else if (s.refined) {
    if (rr > 100.0 * s.rr_pause) s.fresh = 1;
    if (rr > 4.0 * s.rr_pause) s.rdelta = fmin(0.5, sqrt(s.rdelta));
  } else if (s.own) {
    s.fresh = 1;  // FP64: the iterated residual said converged, the true one did not
  }
  s.ru_thresh = s.refined ? s.rdelta * s.rdelta * rr : 0.0;
  s.own = 0;
  s.done = 0;
}

// Fold a completed reduction into the state (thread 0 only).  tot2 is the
// second value of two-value partials.
FPH_DEVINL void apply_pending(RhsState& s, int kind, double tot, double tot2, int precond) {
  switch (kind) {
    case P_RR:
      s.rr = tot;
      s.iter += 1;
      if (!precond) s.rz_next = tot;
      if (!isfinite(tot)) {
        rhs_finish(s, 8);
      } else if (tot <= s.tol2) {
        rhs_pause(s, 1);
      } else if (s.iter >= s.maxiter || tot < s.ru_thresh) {
        rhs_pause(s, 0);
      }
      break;
    case P_PAP:
      s.pAp = tot;
      s.matvecs += 1;
      if (!(tot > 0.0) || !isfinite(tot)) {
        rhs_finish(s, isfinite(tot) ? 4 : 8);
        s.alpha = 0.0;
      } else {
        s.alpha = s.rz / tot;
      }
      break;
    case P_RZ:
      s.rz_next = tot;
      if (!(tot > 0.0) || !isfinite(tot)) rhs_finish(s, isfinite(tot) ? 4 : 8);
      break;
    case P_RES:
      rhs_after_residual(s, tot, tot2, precond);
      break;
    default:
      break;
  }
  s.folded = kind;
  s.pend = P_NONE;
}

// Reading the state of right-hand side r is split in two so that a kernel
// can issue the loads first and fold them where it needs the result:
// state_issue (first wave only) loads the first 64 NS partial slots and
// the state itself, one 32-bit word per lane.  These are
// vector loads: a barrier waits only for LDS and scalar loads, so they stay
// in flight across the kernel's own LDS exchanges.  state_finish writes the
// words into s_sh, sums the partials (lane l adds partials l, l + 64, ...
// in order, then wave_sum_fixed: the same order in every block), folds
// them (thread 0) and ends with a workgroup barrier.
constexpr int kStWords = (int)(sizeof(RhsState) / 4);
static_assert(sizeof(RhsState) % 4 == 0 && kStWords <= 64, "one state word per lane of a wave");

// NS: partials per lane loaded ahead (lane l: l, l + 64, ...); a kernel
// that holds the loads for long takes few, and more pending partials than
// 64 NS are loaded when folded.
template <int NS>
struct StLoad {
  double pre[NS > 0 ? NS : 1];
  uint32_t w;  // state word `lane`
};

// The loads are unconditional (no branch per load, so none waits for the
// ones before it): slots past the announced partials are read but never
// added (state_finish adds only the first npart), and lanes past the
// state's last word read that word again.
template <int NS>
FPH_DEVINL void state_issue(const StIO& io, int r, StLoad<NS>& L) {
  static_assert(64 * NS <= kPStride, "preloaded partial slots stay inside the right-hand side's");
  if (threadIdx.x < 64) {
    const double* part = io.pin + (long)r * kPStride;
#pragma unroll
    for (int j = 0; j < NS; ++j) L.pre[j] = part[threadIdx.x + 64 * j];
    const uint32_t* sw = reinterpret_cast<const uint32_t*>(io.in + r);
    L.w = sw[min((int)threadIdx.x, kStWords - 1)];
  }
}

template <int NT, int NS>
FPH_DEVINL void state_finish(const StIO& io, int r, const StLoad<NS>& L, RhsState* s_sh) {
  if (threadIdx.x < 64) {
    const int pend = __builtin_amdgcn_readlane((int)L.w, (int)(offsetof(RhsState, pend) / 4));
    const int npart = __builtin_amdgcn_readlane((int)L.w, (int)(offsetof(RhsState, npart) / 4));
    if ((int)threadIdx.x < kStWords) reinterpret_cast<uint32_t*>(s_sh)[threadIdx.x] = L.w;
    if (pend != P_NONE) {
      const double* part = io.pin + (long)r * kPStride;
      // The sums start from -0, the exact identity of addition, so the
      // first partial is not added to anything: a lane's first add would
      // otherwise be computed as soon as its load arrives, stalling the
      // wave right behind the state loads.
      double v = -0.0, v2 = -0.0;
      if (npart <= 64 * NS) {  // all of them were loaded ahead
#pragma unroll
        for (int j = 0; j < NS; ++j) {
          if (64 * j >= npart) break;  // uniform
          if ((int)threadIdx.x + 64 * j < npart) v += L.pre[j];
        }
      } else {
        for (int k = threadIdx.x; k < npart; k += 64) v += part[k];
      }
      if (pend == P_RES)
        for (int k = threadIdx.x; k < npart; k += 64) v2 += part[kPHalf + k];
      v = wave_sum_fixed(v);
      if (pend == P_RES) v2 = wave_sum_fixed(v2);
      if (threadIdx.x == 0) {
        // The fold reads and writes the fields it needs in place.  The
        // wave's own LDS writes above reach LDS first (one wave's LDS
        // operations complete in order); the compiler barrier keeps the
        // compiler from moving these accesses above the word writes.
        asm volatile("" ::: "memory");
        apply_pending(*s_sh, pend, v, v2, io.precond);
      }
    } else if (threadIdx.x == 0) {
      s_sh->folded = P_NONE;
    }
  }
  __syncthreads();
}

// Load the state of right-hand side r into LDS and fold in any pending
// partial sums.  Call from every thread; s_sh is valid afterwards.
template <int NT>
FPH_DEVINL void state_begin(const StIO& io, int r, RhsState* s_sh, double* red_sh) {
  (void)red_sh;
  StLoad<16> L;
  state_issue(io, r, L);
  state_finish<NT>(io, r, L, s_sh);
}

// Publish this block's partial (thread 0 passes its block sum) and, from
// the designated block, the state.  `kind` P_NONE: no partials produced.
FPH_DEVINL void state_end(const StIO& io, int r, RhsState* s_sh, int kind, double blocksum,
                          int block, int nblocks, bool writer, double blocksum2 = 0.0) {
  if (threadIdx.x == 0) {
    if (kind != P_NONE) {
      io.pout[(long)r * kPStride + block] = blocksum;
      if (kind == P_RES) io.pout[(long)r * kPStride + kPHalf + block] = blocksum2;
      s_sh->pend = kind;
      s_sh->npart = nblocks;
    }
    if (writer) io.out[r] = *s_sh;
  }
}

}  // namespace fph
