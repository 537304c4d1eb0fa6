// SSH-type coupling: the phonon field enters the hopping of every bond,
// t_b(x_tau) = t - g (x_{j,tau} - x_{i,tau}) for b = (i, j = i + x^ or i + y^),
// inside the checkerboard factors of exp(-dtau K_tau) (Sec. II C, closing
// remark), so B_tau = diag(E_tau) F_xe F_ye F_xo F_yo with each family factor
// a direct sum of two-site blocks [[cosh, sinh], [sinh, cosh]](dtau t_b).  The
// matrix M keeps the block structure of Eq. M_def; the force goes by the
// product rule through the four factors (Sec. III A).
//
// Kernels work one time slice per workgroup: the slice (N values) sits in
// LDS and the four family factors are applied in place, one barrier apart;
// every thread owns the same BPT bonds of each family.  Setting the field
// forms per-slice tables of the bond coefficients (cosh, sinh) and of E (one
// expm1 per bond), which the operator kernels load into registers; the force
// kernel forms them from x_tau in LDS.  The operator and CG kernels take the
// vector type as a parameter: FP64, or FP32 with the tables rounded to FP32
// for the iterations of the FP32-refined solve (partial sums in FP64).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <utility>
#include <vector>

#include "../../include/holstein_hmc.h"
#include "fph_internal.h"

namespace {

constexpr int kNT = 256;        // threads of a slice workgroup
constexpr int kRedBlocks = 256;  // partial sums per right-hand side of the dot-product kernel
constexpr int kXrBlocks = 512;   // |r|^2 partials per right-hand side of the CG update
constexpr int kMaxChunk = 4096;

struct SshGeom {
  int L, N, Ltau;
  long d;
  double dtau, t, mu, alpha, g;
};

// Sites (i, j) of bond k of family f (0 x-even, 1 y-even, 2 x-odd, 3 y-odd).
__device__ __forceinline__ void bond_sites(int L, int f, int k, int& i, int& j) {
  const int hL = L >> 1;
  const int par = f >> 1;
  if ((f & 1) == 0) {  // x-bonds: row y, start column 2c + par
    const int y = k / hL, x = 2 * (k - y * hL) + par;
    i = x + L * y;
    j = (x + 1 == L ? 0 : x + 1) + L * y;
  } else {  // y-bonds: column x, start row 2r + par
    const int x = k % L, y = 2 * (k / L) + par;
    i = x + L * y;
    j = x + L * (y + 1 == L ? 0 : y + 1);
  }
}

// cosh and sinh of a = dtau t_b without cancellation: with m = expm1(a),
// sinh a = m (1 + e^-a) / 2 and cosh a = 1 + m^2 e^-a / 2.
__device__ __forceinline__ void bond_cs(const SshGeom& G, const double* xs, int i, int j, double& ch,
                                        double& sh) {
  const double a = G.dtau * (G.t - G.g * (xs[j] - xs[i]));
  const double m = expm1(a);
  const double ei = 1.0 / (1.0 + m);
  sh = 0.5 * m * (1.0 + ei);
  ch = 1.0 + 0.5 * m * m * ei;
}

// w <- F_f w in LDS for the workgroup's bonds of family f.
template <int BPT>
__device__ __forceinline__ void apply_family(const SshGeom& G, const double* xs, double* w, int f) {
  const int nb = G.N >> 1;
#pragma unroll
  for (int q = 0; q < BPT; ++q) {
    const int k = threadIdx.x + q * kNT;
    if (k < nb) {
      int i, j;
      bond_sites(G.L, f, k, i, j);
      double ch, sh;
      bond_cs(G, xs, i, j, ch, sh);
      const double wi = w[i], wj = w[j];
      w[i] = ch * wi + sh * wj;
      w[j] = sh * wi + ch * wj;
    }
  }
}

// Per right-hand side CG state: rr = |r|^2, rz = r.z, bb = |b|^2, alpha, beta, iters, status.
// FP32-refined solves also stop (pause) the iteration once |r|^2 <= delta2 rr_ref,
// rr_ref the FP64 |r|^2 of the last evaluation (delta2 = 0 otherwise).
struct CgState {
  double rr, rz, bb, alpha, beta, tol2, rr_ref, delta2;
  int iters, status, done, maxiter;
};

// Sum of acc over a 256-thread workgroup, returned to every thread: a
// shuffle tree inside each wave, then the four wave sums in a fixed order
// (deterministic; one barrier pair).
__device__ double block_sum(double acc) {
  __shared__ double sh[4];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  const double v = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  __syncthreads();  // sh may be reused by the next call
  return v;
}

__device__ double sum_parts(const double* part, int nb) {
  double acc = 0.0;
  for (int b = threadIdx.x; b < nb; b += 256) acc += part[b];
  return block_sum(acc);
}

// One CG step's scalars from |r|^2 = v and r.z = vz (in place): iteration
// count, non-finite and breakdown tests, convergence and cap, beta = rz'/rz.
__device__ void cg_step2(CgState& S, double v, double vz) {
  if (S.done) {
    S.alpha = S.beta = 0.0;
    return;
  }
  S.iters += 1;
  if (!isfinite(v) || !isfinite(vz)) {
    S.status |= FPH_ST_NONFINITE;
    S.done = 1;
    S.beta = 0.0;
    return;
  }
  S.rr = v;
  if (v <= S.tol2 * S.bb || v <= S.delta2 * S.rr_ref || S.iters >= S.maxiter) {
    S.done = 1;  // rz keeps the last step's r.z
    return;
  }
  if (!(vz > 0.0)) {
    S.status |= FPH_ST_BREAKDOWN;
    S.done = 1;
    return;
  }
  S.beta = vz / S.rz;
  S.rz = vz;
}

__device__ __forceinline__ double e_site(const SshGeom& G, double x) {
  return exp(-G.dtau * (G.alpha * x - G.mu));
}

// out = M v (OP 0) or M^T v (OP 1) for right-hand side blockIdx.y, slice blockIdx.x.
//   (M v)_tau   = v_tau - s_tau E_tau C(x_tau) v_{tau-1}
//   (M^T v)_tau = v_tau - s_tau' C(x_tau')^T (E_tau' v_tau'),  tau' = tau + 1 (mod Ltau)
// with s = +1, except s_0 = -1 (the +B_0 corner block).
// Per-slice tables of the field, formed once per field (one workgroup per
// slice): hop[tau][f][k] = (cosh, sinh)(dtau t_b) for bond k of family f,
// Et[tau][i] = E_{tau,i}.  The operator kernels then start their slice with
// plain loads instead of a chain of expm1 between the LDS passes.  hop32
// and Et32 receive the same tables rounded to FP32.
__global__ void __launch_bounds__(kNT) k_ssh_tables(SshGeom G, const double* __restrict__ x,
                                                    double2* __restrict__ hop, double* __restrict__ Et,
                                                    float2* __restrict__ hop32, float* __restrict__ Et32) {
  extern __shared__ double sm[];
  double* xs = sm;
  const int tau = blockIdx.x;
  const double* xt = x + (long)tau * G.N;
  for (int i = threadIdx.x; i < G.N; i += kNT) {
    const double xv = xt[i];
    xs[i] = xv;
    const double e = e_site(G, xv);
    Et[(long)tau * G.N + i] = e;
    Et32[(long)tau * G.N + i] = (float)e;
  }
  __syncthreads();
  const int nb = G.N >> 1;
  double2* ht = hop + (long)tau * 2 * G.N;
  float2* ht32 = hop32 + (long)tau * 2 * G.N;
  for (int f = 0; f < 4; ++f)
    for (int k = threadIdx.x; k < nb; k += kNT) {
      int i, j;
      bond_sites(G.L, f, k, i, j);
      double ch, sh;
      bond_cs(G, xs, i, j, ch, sh);
      ht[f * nb + k] = make_double2(ch, sh);
      ht32[f * nb + k] = make_float2((float)ch, (float)sh);
    }
}

// (cosh, sinh) pairs of the bond tables in the vector type T.
template <typename T> struct Pair;
template <> struct Pair<double> { using type = double2; };
template <> struct Pair<float> { using type = float2; };

// w <- F_f w with the thread's bond coefficients hc[q] = (cosh, sinh) of bond
// threadIdx.x + q kNT of family f.
template <typename T, int BPT>
__device__ __forceinline__ void apply_family_t(const SshGeom& G, T* w, int f,
                                               const typename Pair<T>::type (&hc)[BPT]) {
  const int nb = G.N >> 1;
#pragma unroll
  for (int q = 0; q < BPT; ++q) {
    const int k = threadIdx.x + q * kNT;
    if (k < nb) {
      int i, j;
      bond_sites(G.L, f, k, i, j);
      const T wi = w[i], wj = w[j];
      w[i] = hc[q].x * wi + hc[q].y * wj;
      w[j] = hc[q].y * wi + hc[q].x * wj;
    }
  }
}

// out = M v (OP 0) or M^T v (OP 1) for right-hand side blockIdx.y, slice blockIdx.x:
//   (M v)_tau   = v_tau - s_tau E_tau C(x_tau) v_{tau-1}
//   (M^T v)_tau = v_tau - s_tau' C(x_tau')^T (E_tau' v_tau'),  tau' = tau + 1 (mod Ltau)
// with s = +1, except s_0 = -1 (the +B_0 corner block); bond coefficients and
// E from the field's tables.
// With dotv != nullptr the workgroup also writes part[r * Ltau + tau] =
// dotv_{r,tau} . out_{r,tau} (the p . M^T M p partials of CG).  PUPD (M
// only): the operand is the CG direction p = z + beta_r in, formed on the fly
// from zv and the previous direction `in`; the workgroup stores its own slice
// of p in pnew (a buffer other than `in`, so no workgroup reads a slice that
// another one is rewriting); a right-hand side whose state says done is
// skipped (its direction stays where it was last written).
template <typename T, int OP, int BPT, bool PUPD>
__global__ void __launch_bounds__(kNT) k_ssh_apply(SshGeom G, const typename Pair<T>::type* __restrict__ hop,
                                                   const T* __restrict__ Et,
                                                   const T* __restrict__ in,
                                                   T* __restrict__ out,
                                                   const T* __restrict__ dotv,
                                                   double* __restrict__ part,
                                                   const T* __restrict__ zv,
                                                   const CgState* __restrict__ st,
                                                   T* __restrict__ pnew) {
  using V2 = typename Pair<T>::type;
  extern __shared__ double sm[];
  T* w = reinterpret_cast<T*>(sm);
  // a stopped right-hand side keeps its direction (as in k_ssh_mtm)
  if (PUPD && st[blockIdx.y].done) return;
  const int tau = blockIdx.x;
  const long ro = (long)blockIdx.y * G.d;
  const int ts = OP == 0 ? tau : (tau + 1 == G.Ltau ? 0 : tau + 1);  // slice of the field used
  const int tv = OP == 0 ? (tau == 0 ? G.Ltau - 1 : tau - 1) : ts;   // slice of v transported
  const int nb = G.N >> 1;
  const V2* ht = hop + (long)ts * 2 * G.N;
  const T* Es = Et + (long)ts * G.N;
  V2 hc[4][BPT];
#pragma unroll
  for (int f = 0; f < 4; ++f)
#pragma unroll
    for (int q = 0; q < BPT; ++q) {
      const int k = threadIdx.x + q * kNT;
      hc[f][q] = k < nb ? ht[f * nb + k] : V2{(T)0, (T)0};
    }
  const T* vt = in + ro + (long)tv * G.N;
  const T beta = PUPD ? (T)st[blockIdx.y].beta : (T)0;
  const T* zt = PUPD ? zv + ro + (long)tv * G.N : nullptr;
  for (int i = threadIdx.x; i < G.N; i += kNT) {
    if (PUPD)
      w[i] = zt[i] + beta * vt[i];
    else
      w[i] = OP == 0 ? vt[i] : Es[i] * vt[i];
  }
  __syncthreads();
  if (OP == 0) {
#pragma unroll
    for (int f = 3; f >= 0; --f) {
      apply_family_t<T, BPT>(G, w, f, hc[f]);
      __syncthreads();
    }
  } else {
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      apply_family_t<T, BPT>(G, w, f, hc[f]);
      __syncthreads();
    }
  }
  const T s = (OP == 0 ? tau : ts) == 0 ? (T)-1 : (T)1;
  const T* vi = in + ro + (long)tau * G.N;
  T* vo = out + ro + (long)tau * G.N;
  double acc = 0.0;
  const T* zi = PUPD ? zv + ro + (long)tau * G.N : nullptr;
  T* pn = PUPD ? pnew + ro + (long)tau * G.N : nullptr;
  for (int i = threadIdx.x; i < G.N; i += kNT) {
    const T bw = OP == 0 ? Es[i] * w[i] : w[i];
    T v = vi[i];
    if (PUPD) {
      v = zi[i] + beta * v;
      pn[i] = v;
    }
    const T o = v - s * bw;
    vo[i] = o;
    if (dotv != nullptr) acc += (double)dotv[ro + (long)tau * G.N + i] * (double)o;
  }
  if (dotv != nullptr) {
    const double v = block_sum(acc);
    if (threadIdx.x == 0) part[(long)blockIdx.y * G.Ltau + tau] = v;
  }
}

// q = M^T M p in one launch (N <= 2048, BPT <= 4), slice blockIdx.x of
// right-hand side blockIdx.y: with a = tau - 1, c = tau + 1 (mod Ltau),
//   y_tau = p_tau - s_tau E_tau C_tau p_a,   y_c = p_c - s_c E_c C_c p_tau,
//   q_tau = y_tau - s_c C_c^T (E_c y_c),
// the two forward products sharing the four family passes (two LDS
// buffers), then the transposed product: y_c is formed twice, by this
// workgroup and by the next one, instead of a launch and a round trip of M p
// through memory.  dotv, part, PUPD, zv, st and pnew as for k_ssh_apply
// (the dot is p . q with p the direction used).
// In CG (PUPD) the kernel also finishes the previous step's scalars: every
// workgroup of right-hand side r forms beta and the convergence decision
// from |r|^2 and r.z partials (part_rr: kXrBlocks, part_rz: nbz each) and the
// state st_old[r], all the same way; workgroup 0 stores the new state in
// st_new[r] (a second buffer: no workgroup reads what another one writes).
// With from_state the state is taken as it is (first step of a chunk).  A
// finished right-hand side is skipped.
template <typename T, int BPT, bool PUPD>
__global__ void __launch_bounds__(kNT) k_ssh_mtm(SshGeom G, const typename Pair<T>::type* __restrict__ hop,
                                                 const T* __restrict__ Et,
                                                 const T* __restrict__ in,
                                                 T* __restrict__ out, bool dot,
                                                 double* __restrict__ part,
                                                 const T* __restrict__ zv,
                                                 const CgState* __restrict__ st_old,
                                                 CgState* __restrict__ st_new,
                                                 const double* __restrict__ part_rr,
                                                 const double* __restrict__ part_rz, int nbz,
                                                 int from_state,
                                                 T* __restrict__ pnew) {
  using V2 = typename Pair<T>::type;
  constexpr int kOwn = 2 * BPT;  // sites per thread: N <= 2 * BPT * kNT
  extern __shared__ double sm[];
  T* wA = reinterpret_cast<T*>(sm);
  T* wB = wA + G.N;
  const int tau = blockIdx.x;
  const long ro = (long)blockIdx.y * G.d;
  const int ta = tau == 0 ? G.Ltau - 1 : tau - 1;
  const int tc = tau + 1 == G.Ltau ? 0 : tau + 1;
  const T sb = tau == 0 ? (T)-1 : (T)1;
  const T sc = tc == 0 ? (T)-1 : (T)1;
  const int nb = G.N >> 1;
  const V2* hb = hop + (long)tau * 2 * G.N;
  const V2* hcp = hop + (long)tc * 2 * G.N;
  V2 cB[4][BPT], cC[4][BPT];
#pragma unroll
  for (int f = 0; f < 4; ++f)
#pragma unroll
    for (int q = 0; q < BPT; ++q) {
      const int k = threadIdx.x + q * kNT;
      cB[f][q] = k < nb ? hb[f * nb + k] : V2{(T)0, (T)0};
      cC[f][q] = k < nb ? hcp[f * nb + k] : V2{(T)0, (T)0};
    }
  const T* Eb = Et + (long)tau * G.N;
  const T* Ec = Et + (long)tc * G.N;
  T beta = (T)0;
  if (PUPD) {
    const int r = blockIdx.y;
    CgState S = st_old[r];
    if (!from_state) {
      const double v = sum_parts(part_rr + (long)r * kXrBlocks, kXrBlocks);
      const double vz = part_rz == part_rr ? v : sum_parts(part_rz + (long)r * nbz, nbz);
      cg_step2(S, v, vz);  // the same inputs and steps in every thread: a uniform result
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) st_new[r] = S;
    if (S.done) return;
    beta = (T)S.beta;
  }
  auto dir = [&](int t, int i) -> T {  // the direction p at slice t, site i
    const long o = ro + (long)t * G.N + i;
    return PUPD ? zv[o] + beta * in[o] : in[o];
  };
  T pb[kOwn], pc[kOwn], yb[kOwn];
#pragma unroll
  for (int m = 0; m < kOwn; ++m) {
    const int i = threadIdx.x + m * kNT;
    pb[m] = pc[m] = (T)0;
    if (i < G.N) {
      wA[i] = dir(ta, i);
      pb[m] = dir(tau, i);
      pc[m] = dir(tc, i);
      wB[i] = pb[m];
      if (PUPD) pnew[ro + (long)tau * G.N + i] = pb[m];
    }
  }
  __syncthreads();
#pragma unroll
  for (int f = 3; f >= 0; --f) {
    apply_family_t<T, BPT>(G, wA, f, cB[f]);
    apply_family_t<T, BPT>(G, wB, f, cC[f]);
    __syncthreads();
  }
#pragma unroll
  for (int m = 0; m < kOwn; ++m) {
    const int i = threadIdx.x + m * kNT;
    yb[m] = (T)0;
    if (i < G.N) {
      yb[m] = pb[m] - sb * Eb[i] * wA[i];
      const T e = Ec[i];
      wB[i] = e * (pc[m] - sc * e * wB[i]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    apply_family_t<T, BPT>(G, wB, f, cC[f]);
    __syncthreads();
  }
  double acc = 0.0;
  T* vo = out + ro + (long)tau * G.N;
#pragma unroll
  for (int m = 0; m < kOwn; ++m) {
    const int i = threadIdx.x + m * kNT;
    if (i < G.N) {
      const T q = yb[m] - sc * wB[i];
      vo[i] = q;
      acc += (double)pb[m] * (double)q;
    }
  }
  if (dot) {
    const double v = block_sum(acc);
    if (threadIdx.x == 0) part[(long)blockIdx.y * G.Ltau + tau] = v;
  }
}

// grad_tau += scale * s * sum_r dS_F/dx_tau with S_F = Phi . (M^T M)^{-1} Phi
// (s = *scale_dev read at run time, 1 when scale_dev is null):
//   dS_F/dx_{i,tau} = 2 s_tau sum_r y_{r,tau} . (dB_tau/dx_{i,tau}) u_{r,tau-1},  y = M u.
// dB = d(diag E) C + diag(E) sum_f F_xe .. dF_f .. F_yo: the vector entering
// F_f from the right (a_f) is kept per thread in registers while C u is
// formed; the row vector (E y) is then carried through the factors from the
// left, and each bond adds dtau [c_i c_j] [[sh, ch], [ch, sh]] [a_i a_j]^T
// times dt_b/dx = +g (site i), -g (site j).
template <int BPT>
__global__ void __launch_bounds__(kNT) k_ssh_force(SshGeom G, int nrhs, const double* __restrict__ x,
                                                   const double* __restrict__ u,
                                                   const double* __restrict__ y, double scale,
                                                   const double* __restrict__ scale_dev,
                                                   double* __restrict__ grad) {
  extern __shared__ double sm[];
  double* xs = sm;
  double* w = sm + G.N;
  double* cv = sm + 2 * G.N;
  double* ga = sm + 3 * G.N;
  const int tau = blockIdx.x;
  const int tp = tau == 0 ? G.Ltau - 1 : tau - 1;
  const double s = tau == 0 ? -1.0 : 1.0;
  const double* xt = x + (long)tau * G.N;
  const int nb = G.N >> 1;
  for (int i = threadIdx.x; i < G.N; i += kNT) {
    xs[i] = xt[i];
    ga[i] = 0.0;
  }
  for (int r = 0; r < nrhs; ++r) {
    const double* ur = u + (long)r * G.d + (long)tp * G.N;
    const double* yr = y + (long)r * G.d + (long)tau * G.N;
    __syncthreads();  // xs/ga ready; the previous right-hand side is done with w, cv
    for (int i = threadIdx.x; i < G.N; i += kNT) {
      w[i] = ur[i];
      cv[i] = e_site(G, xs[i]) * yr[i];
    }
    __syncthreads();
    double A[4][BPT][2];
#pragma unroll
    for (int f = 3; f >= 0; --f) {
#pragma unroll
      for (int q = 0; q < BPT; ++q) {
        const int k = threadIdx.x + q * kNT;
        if (k < nb) {
          int i, j;
          bond_sites(G.L, f, k, i, j);
          A[f][q][0] = w[i];
          A[f][q][1] = w[j];
        }
      }
      apply_family<BPT>(G, xs, w, f);
      __syncthreads();
    }
    // on-site term: dE_i/dx_i (C u)_i y_i = -dtau alpha (E y)_i (C u)_i
    for (int i = threadIdx.x; i < G.N; i += kNT) ga[i] -= G.dtau * G.alpha * cv[i] * w[i];
    __syncthreads();
#pragma unroll
    for (int f = 0; f < 4; ++f) {
#pragma unroll
      for (int q = 0; q < BPT; ++q) {
        const int k = threadIdx.x + q * kNT;
        if (k < nb) {
          int i, j;
          bond_sites(G.L, f, k, i, j);
          double ch, sh;
          bond_cs(G, xs, i, j, ch, sh);
          const double ci = cv[i], cj = cv[j];
          const double ai = A[f][q][0], aj = A[f][q][1];
          const double gb = G.g * G.dtau * (sh * (ci * ai + cj * aj) + ch * (ci * aj + cj * ai));
          ga[i] += gb;
          ga[j] -= gb;
          cv[i] = ch * ci + sh * cj;  // c_{f+1} = F_f c_f
          cv[j] = sh * ci + ch * cj;
        }
      }
      __syncthreads();
    }
  }
  double* gt = grad + (long)tau * G.N;
  const double c = 2.0 * s * scale * (scale_dev != nullptr ? *scale_dev : 1.0);
  for (int i = threadIdx.x; i < G.N; i += kNT) gt[i] += c * ga[i];
}

// ------------------------------------------------------------ CG on M^T M

// part[r][b] = sum over block b's share of a_r . c_r (FP64 sums)
template <typename T>
__global__ void __launch_bounds__(256) k_dot_parts(long d, const T* __restrict__ a,
                                                   const T* __restrict__ c,
                                                   double* __restrict__ part) {
  const int r = blockIdx.y;
  a += (long)r * d;
  c += (long)r * d;
  double acc = 0.0;
  for (long k = blockIdx.x * 256L + threadIdx.x; k < d; k += (long)gridDim.x * 256)
    acc += (double)a[k] * (double)c[k];
  const double v = block_sum(acc);
  if (threadIdx.x == 0) part[(long)r * gridDim.x + blockIdx.x] = v;
}


// stage 0: rr = |r|^2, rz = r.z at the start; stage 2: rr' = |r|^2
// (convergence and cap tests), rz' = r.z, beta = rz'/rz.  (alpha is formed
// by k_cg_xr.)
// part2 holds the r.z partials (part2 == part without a preconditioner, z = r).
__global__ void __launch_bounds__(256) k_cg_scalar(int stage, int nb, int nb2, const double* __restrict__ part,
                                                   const double* __restrict__ part2,
                                                   CgState* __restrict__ st) {
  const int r = blockIdx.x;
  const double v = sum_parts(part + (long)r * nb, nb);
  const double vz = part2 == part ? v : sum_parts(part2 + (long)r * nb2, nb2);
  if (threadIdx.x != 0) return;
  CgState& S = st[r];
  if (stage == 0) {
    S.rr = v;
    S.rz = vz;
    S.alpha = S.beta = 0.0;
    S.iters = 0;
    S.status = 0;
    S.done = !(v > S.tol2 * S.bb) ? 1 : 0;
    if (!S.done && !(vz > 0.0)) {
      S.status |= isfinite(vz) ? FPH_ST_BREAKDOWN : FPH_ST_NONFINITE;
      S.done = 1;
    }
    if (!isfinite(v)) {
      S.status |= FPH_ST_NONFINITE;
      S.done = 1;
    }
    return;
  }
  cg_step2(S, v, vz);
}

// alpha = rz / p.q from the operator's per-slice partials (every block sums
// them in the same order, so all blocks take the same decision; block 0
// records it), then u += alpha p, r -= alpha q, and part[k][block] = the
// block's share of |r|^2 (grid: kXrBlocks x nrhs).  A finished right-hand
// side is left alone; its partials are then stale and its scalars ignore them.
template <typename T>
__global__ void __launch_bounds__(256) k_cg_xr(long d, CgState* __restrict__ st, int npq,
                                               const double* __restrict__ part_pq,
                                               const T* __restrict__ p, const T* __restrict__ q,
                                               T* __restrict__ u, T* __restrict__ r,
                                               double* __restrict__ part) {
  const int k = blockIdx.y;
  // block 0 may set done below: read it once per block so the exit is uniform
  __shared__ int done_sh;
  if (threadIdx.x == 0) done_sh = st[k].done;
  __syncthreads();
  if (done_sh) return;
  const double pq = sum_parts(part_pq + (long)k * npq, npq);
  const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
  if (!(pq > 0.0) || !isfinite(pq)) {
    if (lead) {
      st[k].status |= isfinite(pq) ? FPH_ST_BREAKDOWN : FPH_ST_NONFINITE;
      st[k].alpha = 0.0;
      st[k].done = 1;
    }
    return;
  }
  const double a = st[k].rz / pq;
  if (lead) st[k].alpha = a;
  const T at = (T)a;
  const long o = (long)k * d;
  double acc = 0.0;
  for (long i = blockIdx.x * 256L + threadIdx.x; i < d; i += (long)gridDim.x * 256) {
    u[o + i] += at * p[o + i];
    const T rv = r[o + i] - at * q[o + i];
    r[o + i] = rv;
    acc += (double)rv * (double)rv;
  }
  const double v = block_sum(acc);
  if (threadIdx.x == 0) part[(long)k * gridDim.x + blockIdx.x] = v;
}

// out[r] = sum of the kRedBlocks partials of right-hand side r, in block order
__global__ void __launch_bounds__(256) k_sum_rhs(int nb, const double* __restrict__ part,
                                                 double* __restrict__ out) {
  const double v = sum_parts(part + (long)blockIdx.x * nb, nb);
  if (threadIdx.x == 0) out[blockIdx.x] = v;
}

// r = b - r (r holds M^T M u on entry)
__global__ void __launch_bounds__(256) k_sub_from(long n, const double* __restrict__ b, double* __restrict__ r) {
  for (long i = blockIdx.x * 256L + threadIdx.x; i < n; i += (long)gridDim.x * 256) r[i] = b[i] - r[i];
}

// dst = (float) src
__global__ void __launch_bounds__(256) k_to_f32(long n, const double* __restrict__ src, float* __restrict__ dst) {
  for (long i = blockIdx.x * 256L + threadIdx.x; i < n; i += (long)gridDim.x * 256) dst[i] = (float)src[i];
}

// u += (double) e, e = 0: the FP32 correction moved into the FP64 iterate
__global__ void __launch_bounds__(256) k_fold_f32(long n, double* __restrict__ u, float* __restrict__ e) {
  for (long i = blockIdx.x * 256L + threadIdx.x; i < n; i += (long)gridDim.x * 256) {
    u[i] += (double)e[i];
    e[i] = 0.0f;
  }
}

int grid_for(long n) {
  const long b = (n + 255) / 256;
  return (int)(b < 2048 ? (b < 1 ? 1 : b) : 2048);
}

}  // namespace

struct fph_ssh_s {
  SshGeom G;
  int max_rhs;
  int bpt;
  bool have_field;
  double* x;     // the field [Ltau][N]
  double2* hop;  // bond (cosh, sinh) per slice and family [Ltau][4][N/2]
  double* Et;    // E of the field [Ltau][N]
  double* tmp;   // [max_rhs][d]
  double* r;     // CG residual
  double* p;     // CG direction
  double* p2;    // the next direction (formed inside the operator launch)
  double* q;     // M^T M p
  double* z;     // preconditioned residual
  double* part;  // [max_rhs][kRedBlocks]
  double* part2; // r.z partials
  CgState* st;   // [2][max_rhs]: the fused CG alternates between the two
  double* part3; // p.q partials of the fused CG
  CgState* st_host;
  // FP32-refined solves: the tables rounded to FP32 and the FP32 vectors
  float2* hop32;  // [Ltau][4][N/2]
  float* Et32;    // [Ltau][N]
  float* r32;     // FP32 residual
  float* z32;     // preconditioned residual
  float* pa32;    // directions (two buffers, as p / p2)
  float* pb32;
  float* q32;     // M^T M p
  float* tmp32;   // M p (unfused operator)
  float* u32;     // the correction since the last residual replacement
  fph_handle_t pc;  // Holstein handle whose preconditioner serves the solves (or NULL)
  int pc_max_rhs;
  double pc_a1, pc_a2;  // its Chebyshev-order constants (fph_set_field)
};

namespace {

#define SSH_CHECK(call)                                      \
  do {                                                       \
    hipError_t e_ = (call);                                  \
    if (e_ != hipSuccess) return fph::record_hip_error(e_);  \
  } while (0)

size_t apply_lds(const fph_ssh_s* c) { return (size_t)c->G.N * sizeof(double); }
size_t force_lds(const fph_ssh_s* c) { return 4 * (size_t)c->G.N * sizeof(double); }

// Dynamic LDS above the default 64 KiB (L = 64: the force kernel takes 128 KiB).
template <typename K>
hipError_t allow_lds(K kern, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// The field's tables and the operator workspace in the vector type T.
template <typename T> struct Tabs;
template <> struct Tabs<double> {
  static const double2* hop(const fph_ssh_s* c) { return c->hop; }
  static const double* Et(const fph_ssh_s* c) { return c->Et; }
  static double* tmp(const fph_ssh_s* c) { return c->tmp; }
};
template <> struct Tabs<float> {
  static const float2* hop(const fph_ssh_s* c) { return c->hop32; }
  static const float* Et(const fph_ssh_s* c) { return c->Et32; }
  static float* tmp(const fph_ssh_s* c) { return c->tmp32; }
};

// PUPD launches (OP 0 only) take zv, the state and pnew as described at the kernel.
template <typename T, int OP, bool PUPD = false>
hipError_t launch_apply_op(const fph_ssh_s* c, int nrhs, const T* in, T* out, hipStream_t s,
                           const T* dotv = nullptr, const T* zv = nullptr,
                           T* pnew = nullptr, double* pt = nullptr) {
  const dim3 grid(c->G.Ltau, nrhs);
  const size_t lds = apply_lds(c);
  const CgState* st = c->st;
  if (c->bpt == 8) {
    hipError_t e = allow_lds(k_ssh_apply<T, OP, 8, PUPD>, lds);
    if (e != hipSuccess) return e;
  }
#define SSH_APPLY_CASE(b)                                                                      \
  hipLaunchKernelGGL((k_ssh_apply<T, OP, b, PUPD>), grid, dim3(kNT), lds, s, c->G,               \
                     Tabs<T>::hop(c), Tabs<T>::Et(c), in, out, dotv, pt, zv, st, pnew)
  switch (c->bpt) {
    case 1: SSH_APPLY_CASE(1); break;
    case 2: SSH_APPLY_CASE(2); break;
    case 4: SSH_APPLY_CASE(4); break;
    default: SSH_APPLY_CASE(8); break;
  }
#undef SSH_APPLY_CASE
  return hipGetLastError();
}

// q = M^T M p in one launch when the lattice allows it (BPT <= 4); returns
// false (nothing launched) otherwise.  With dot, part[r * Ltau + tau] = p . q.
bool mtm_fusable(const fph_ssh_s* c) { return c->bpt <= 4; }

// CG arguments of a fused launch (see k_ssh_mtm).
template <typename T>
struct MtmCg {
  const T* zv = nullptr;
  T* pnew = nullptr;
  const CgState* st_old = nullptr;
  CgState* st_new = nullptr;
  const double* part_rr = nullptr;
  const double* part_rz = nullptr;
  int nbz = kRedBlocks;  // r.z partials per right-hand side (kXrBlocks when part_rz == part_rr)
  int from_state = 1;
};

// q = M^T M p in one launch (only where mtm_fusable).  With dot,
// pt[r * Ltau + tau] = p . q.
template <typename T, bool PUPD>
hipError_t launch_mtm_fused(const fph_ssh_s* c, int nrhs, const T* in, T* out, hipStream_t s,
                            bool dot, double* pt, const MtmCg<T>& a) {
  const dim3 grid(c->G.Ltau, nrhs);
  const size_t lds = 2 * (size_t)c->G.N * sizeof(T);
  const auto* hop = Tabs<T>::hop(c);
  const T* Et = Tabs<T>::Et(c);
#define SSH_MTM_CASE(b)                                                                                    \
  hipLaunchKernelGGL((k_ssh_mtm<T, b, PUPD>), grid, dim3(kNT), lds, s, c->G, hop, Et, in, out, dot, pt, a.zv, \
                     a.st_old, a.st_new, a.part_rr, a.part_rz, a.nbz, a.from_state, a.pnew)
  switch (c->bpt) {
    case 1: SSH_MTM_CASE(1); break;
    case 2: SSH_MTM_CASE(2); break;
    default: SSH_MTM_CASE(4); break;
  }
#undef SSH_MTM_CASE
  return hipGetLastError();
}

// out = op(in); MTM goes through the workspace of type T (so in/out must not
// be it).  With dotv (MTM only), c->part[r * Ltau + tau] receive the slices
// of dotv . out.
template <typename T>
hipError_t launch_apply(const fph_ssh_s* c, int op, int nrhs, const T* in, T* out, hipStream_t s,
                        const T* dotv = nullptr) {
  if (op == FPH_OP_M) return launch_apply_op<T, 0>(c, nrhs, in, out, s);
  if (op == FPH_OP_MT) return launch_apply_op<T, 1>(c, nrhs, in, out, s);
  if (dotv == nullptr && mtm_fusable(c))
    return launch_mtm_fused<T, false>(c, nrhs, in, out, s, false, nullptr, MtmCg<T>{});
  hipError_t e = launch_apply_op<T, 0>(c, nrhs, in, Tabs<T>::tmp(c), s);
  if (e != hipSuccess) return e;
  return launch_apply_op<T, 1>(c, nrhs, Tabs<T>::tmp(c), out, s, dotv);
}

hipError_t launch_force(const fph_ssh_s* c, int nrhs, const double* u, const double* y, double scale,
                        const double* scale_dev, double* grad, hipStream_t s) {
  const dim3 grid(c->G.Ltau);
  const size_t lds = force_lds(c);
  if (c->bpt == 8) {
    hipError_t e = allow_lds(k_ssh_force<8>, lds);
    if (e != hipSuccess) return e;
  }
  switch (c->bpt) {
    case 1: hipLaunchKernelGGL((k_ssh_force<1>), grid, dim3(kNT), lds, s, c->G, nrhs, c->x, u, y, scale, scale_dev, grad); break;
    case 2: hipLaunchKernelGGL((k_ssh_force<2>), grid, dim3(kNT), lds, s, c->G, nrhs, c->x, u, y, scale, scale_dev, grad); break;
    case 4: hipLaunchKernelGGL((k_ssh_force<4>), grid, dim3(kNT), lds, s, c->G, nrhs, c->x, u, y, scale, scale_dev, grad); break;
    default: hipLaunchKernelGGL((k_ssh_force<8>), grid, dim3(kNT), lds, s, c->G, nrhs, c->x, u, y, scale, scale_dev, grad); break;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t dots(const fph_ssh_s* c, int nrhs, const T* a, const T* b, hipStream_t s,
                double* part = nullptr) {
  hipLaunchKernelGGL(k_dot_parts<T>, dim3(kRedBlocks, nrhs), dim3(256), 0, s, c->G.d, a, b,
                     part ? part : c->part);
  return hipGetLastError();
}

// FP32-refined (P)CG on M^T M (reliable updates of the residual, as the
// Holstein solver's FP32-refined mode): FP32 CG on a correction u32 with the
// FP32 tables.  The iteration of a right-hand side stops on the device
// when its FP32 residual has fallen by delta since the last FP64 evaluation,
// reaches the tolerance, hits the cap or breaks down; every `chunk`
// iterations the host reads the state, and if any has stopped, the
// corrections are moved into the FP64 iterate, the FP64 residual
// r = b - M^T M u is evaluated with the FP64 tables, and the FP32 iteration
// continues from it: r32 = r, z = F F^T r, |r|^2 and r.z replaced, and the
// directions kept with beta = r.z (replaced) / r.z (previous step), unless
// the evaluated residual is 100x the iterated one (then beta = 0).  A
// right-hand side finishes when its FP64 residual reaches the tolerance, or
// at the caps.
int solve_refined(fph_ssh_s* c, int nrhs, const double* b_dev, double* u_dev, const fph_pcg_opts_t* opts,
                  fph_pcg_stats_t* stats_host, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  const long d = c->G.d;
  const long n = (long)nrhs * d;
  const bool pre = opts->use_precond != 0;
  const int chunk = opts->chunk > 0 ? (opts->chunk < kMaxChunk ? opts->chunk : kMaxChunk) : 64;
  double delta = opts->ru_delta > 0.0 ? std::min(opts->ru_delta, 0.5) : (pre ? 0.1 : 0.3);
  const int max_outer = opts->max_outer > 0 ? opts->max_outer : 32;
  const double tol2 = opts->tol * opts->tol;
  float* z = pre ? c->z32 : c->r32;
  const double* p2 = pre ? c->part2 : c->part;
  auto sum_host = [&](const double* part_dev, std::vector<double>& out) -> int {
    std::vector<double> part((size_t)nrhs * kRedBlocks);
    SSH_CHECK(hipStreamSynchronize(s));
    SSH_CHECK(hipMemcpy(part.data(), part_dev, part.size() * sizeof(double), hipMemcpyDeviceToHost));
    out.assign(nrhs, 0.0);
    for (int r = 0; r < nrhs; ++r)
      for (int k = 0; k < kRedBlocks; ++k) out[r] += part[(size_t)r * kRedBlocks + k];
    return FPH_OK;
  };
  // FP64 residual of the iterate into c->r and its |r|^2 on the host
  auto residual64 = [&](std::vector<double>& rr) -> int {
    SSH_CHECK(launch_apply<double>(c, FPH_OP_MTM, nrhs, u_dev, c->r, s));
    hipLaunchKernelGGL(k_sub_from, dim3(grid_for(n)), dim3(256), 0, s, n, b_dev, c->r);
    SSH_CHECK(hipGetLastError());
    SSH_CHECK(dots<double>(c, nrhs, c->r, c->r, s));
    return sum_host(c->part, rr);
  };
  // r32 = (float) r64, z = F F^T r32 (or r32), and |r32|^2, r32 . z
  auto start32 = [&](std::vector<double>& rr32, std::vector<double>& rz32) -> int {
    hipLaunchKernelGGL(k_to_f32, dim3(grid_for(n)), dim3(256), 0, s, n, (const double*)c->r, c->r32);
    SSH_CHECK(hipGetLastError());
    if (pre) {
      const int rc = fph_precond_apply(c->pc, FPH_PC_FFT, FPH_F32, nrhs, c->r32, c->z32, stream);
      if (rc != FPH_OK) return rc;
    }
    SSH_CHECK(dots<float>(c, nrhs, c->r32, c->r32, s));
    int rc = sum_host(c->part, rr32);
    if (rc != FPH_OK) return rc;
    if (!pre) {
      rz32 = rr32;
      return FPH_OK;
    }
    SSH_CHECK(dots<float>(c, nrhs, c->r32, c->z32, s, c->part2));
    return sum_host(c->part2, rz32);
  };

  std::vector<double> bb, rr64, rr32, rz32, act;
  SSH_CHECK(dots<double>(c, nrhs, b_dev, b_dev, s));
  int rc = sum_host(c->part, bb);
  if (rc != FPH_OK) return rc;
  if (opts->zero_guess) SSH_CHECK(hipMemsetAsync(u_dev, 0, n * sizeof(double), s));
  for (int r = 0; r < nrhs; ++r)  // b = 0: u = 0 exactly
    if (bb[r] == 0.0) SSH_CHECK(hipMemsetAsync(u_dev + (long)r * d, 0, d * sizeof(double), s));
  SSH_CHECK(hipMemsetAsync(c->u32, 0, n * sizeof(float), s));
  rc = residual64(rr64);
  if (rc != FPH_OK) return rc;
  rc = start32(rr32, rz32);
  if (rc != FPH_OK) return rc;
  std::vector<int> fin(nrhs, 0), conv(nrhs, 0);
  std::vector<double> rr_ref(rr64);
  for (int r = 0; r < nrhs; ++r) {
    CgState& S = c->st_host[r];
    std::memset(&S, 0, sizeof(S));
    S.tol2 = tol2;
    S.maxiter = opts->maxiter;
    S.bb = bb[r];
    S.rr = rr32[r];
    S.rz = rz32[r];
    S.rr_ref = rr64[r];
    S.delta2 = delta * delta;
    if (!std::isfinite(rr64[r]) || !std::isfinite(rz32[r])) {
      S.status |= FPH_ST_NONFINITE;
      fin[r] = 1;
    } else if (!(rr64[r] > tol2 * bb[r])) {
      fin[r] = conv[r] = 1;
    } else if (!(rz32[r] > 0.0)) {
      S.status |= FPH_ST_BREAKDOWN;
      fin[r] = 1;
    }
    S.done = fin[r];
  }
  SSH_CHECK(hipMemcpyAsync(c->st, c->st_host, nrhs * sizeof(CgState), hipMemcpyHostToDevice, s));
  SSH_CHECK(hipMemcpyAsync(c->pa32, z, n * sizeof(float), hipMemcpyDeviceToDevice, s));
  float* pc = c->pa32;  // the current direction
  float* pn = c->pb32;  // receives the next one
  const bool fused = mtm_fusable(c);
  CgState* sa = c->st;
  CgState* sb = c->st + c->max_rhs;
  int outer = 0;
  const int matvecs0 = opts->zero_guess ? 0 : 1;
  std::vector<int> iters0(nrhs, 0);
  for (;;) {
    bool all = true;
    for (int r = 0; r < nrhs; ++r) all = all && fin[r];
    if (all) break;
    for (int r = 0; r < nrhs; ++r) iters0[r] = c->st_host[r].iters;
    for (int k = 0; k < chunk; ++k) {
      const double* pq = c->part2;
      if (fused) {
        MtmCg<float> a;
        a.zv = z;
        a.pnew = pn;
        a.st_old = sa;
        a.st_new = sb;
        a.part_rr = c->part;
        a.part_rz = p2;
        a.nbz = pre ? kRedBlocks : kXrBlocks;
        a.from_state = k == 0;
        SSH_CHECK((launch_mtm_fused<float, true>(c, nrhs, pc, c->q32, s, true, c->part3, a)));
        std::swap(sa, sb);
        pq = c->part3;
      } else {
        SSH_CHECK((launch_apply_op<float, 0, true>(c, nrhs, pc, c->tmp32, s, nullptr, z, pn)));
        SSH_CHECK((launch_apply_op<float, 1>(c, nrhs, c->tmp32, c->q32, s, pn, nullptr, nullptr, c->part2)));
      }
      hipLaunchKernelGGL(k_cg_xr<float>, dim3(kXrBlocks, nrhs), dim3(256), 0, s, d, sa, c->G.Ltau, pq,
                         (const float*)pn, (const float*)c->q32, c->u32, c->r32, c->part);
      SSH_CHECK(hipGetLastError());
      if (pre) {
        rc = fph_precond_apply(c->pc, FPH_PC_FFT, FPH_F32, nrhs, c->r32, c->z32, stream);
        if (rc != FPH_OK) return rc;
        SSH_CHECK(dots<float>(c, nrhs, c->r32, c->z32, s, c->part2));
      }
      if (!fused || k + 1 == chunk) {
        hipLaunchKernelGGL(k_cg_scalar, dim3(nrhs), dim3(256), 0, s, 2, kXrBlocks, pre ? kRedBlocks : kXrBlocks,
                           (const double*)c->part, p2, sa);
        SSH_CHECK(hipGetLastError());
      }
      std::swap(pc, pn);
    }
    SSH_CHECK(hipMemcpyAsync(c->st_host, sa, nrhs * sizeof(CgState), hipMemcpyDeviceToHost, s));
    SSH_CHECK(hipStreamSynchronize(s));
    bool due = false;
    for (int r = 0; r < nrhs; ++r) {
      const CgState& S = c->st_host[r];
      if (!fin[r] && (S.done || S.rr <= delta * delta * rr_ref[r])) due = true;
    }
    if (!due) continue;
    // move the corrections into the FP64 iterate and evaluate its residual
    hipLaunchKernelGGL(k_fold_f32, dim3(grid_for(n)), dim3(256), 0, s, n, u_dev, c->u32);
    SSH_CHECK(hipGetLastError());
    rc = residual64(rr64);
    if (rc != FPH_OK) return rc;
    ++outer;
    std::vector<int> restart(nrhs, 0), paused(nrhs, 0);
    for (int r = 0; r < nrhs; ++r) {
      if (fin[r]) continue;
      CgState& S = c->st_host[r];
      paused[r] = S.done;
      // The launch of chunk step k writes the next direction into the buffer
      // that is current after the step; a right-hand side that stopped after
      // j = iters - iters0 iterations (its j-th scalars folded in step j)
      // last wrote it in step j - 1, so after the chunk its direction is in
      // the current buffer when chunk - j is even, else in the other one.
      const int j = S.iters - iters0[r];
      if (S.done && j >= 1 && ((chunk - j) & 1))
        SSH_CHECK(hipMemcpyAsync(pc + (long)r * d, pn + (long)r * d, d * sizeof(float),
                                 hipMemcpyDeviceToDevice, s));
      if (!std::isfinite(rr64[r])) {
        S.status |= FPH_ST_NONFINITE;
        fin[r] = 1;
      } else if (!(rr64[r] > tol2 * bb[r])) {
        fin[r] = conv[r] = 1;
      } else if (S.status & (FPH_ST_BREAKDOWN | FPH_ST_NONFINITE)) {
        fin[r] = 1;
      } else if (S.iters >= S.maxiter || outer >= max_outer) {
        fin[r] = 1;
      } else {
        if (rr64[r] > 4.0 * S.rr) delta = std::sqrt(delta);  // FP32 recursion drifted: replace sooner
        restart[r] = rr64[r] > 1e4 * S.rr;
        rr_ref[r] = rr64[r];
      }
    }
    rc = start32(rr32, rz32);
    if (rc != FPH_OK) return rc;
    for (int r = 0; r < nrhs; ++r) {
      CgState& S = c->st_host[r];
      S.done = fin[r];
      if (fin[r]) continue;
      // beta with the replaced r.z: a stopped iteration kept the previous
      // step's r.z; a running one has already formed beta from its own
      const double rz_prev = paused[r] ? S.rz : S.rz / S.beta;
      S.beta = restart[r] || !(rz_prev > 0.0) ? 0.0 : rz32[r] / rz_prev;
      S.rr = rr32[r];
      S.rz = rz32[r];
      S.rr_ref = rr64[r];
      S.delta2 = delta * delta;
      if (!(rz32[r] > 0.0)) {
        S.status |= std::isfinite(rz32[r]) ? FPH_ST_BREAKDOWN : FPH_ST_NONFINITE;
        S.done = fin[r] = 1;
      }
    }
    SSH_CHECK(hipMemcpyAsync(sa, c->st_host, nrhs * sizeof(CgState), hipMemcpyHostToDevice, s));
  }
  SSH_CHECK(dots<double>(c, nrhs, b_dev, u_dev, s));
  rc = sum_host(c->part, act);
  if (rc != FPH_OK) return rc;
  if (stats_host) {
    for (int r = 0; r < nrhs; ++r) {
      const CgState& S = c->st_host[r];
      fph_pcg_stats_t& o = stats_host[r];
      std::memset(&o, 0, sizeof(o));
      o.iters = S.iters;
      o.outer_iters = outer;
      o.matvecs = matvecs0 + S.iters + outer;
      o.rel_resid = bb[r] > 0.0 ? std::sqrt(rr64[r] / bb[r]) : 0.0;
      o.action = act[r];
      o.status = S.status & (FPH_ST_BREAKDOWN | FPH_ST_NONFINITE);
      if (conv[r]) o.status |= FPH_ST_CONVERGED;
      else if (!o.status) o.status |= FPH_ST_MAXITER;
    }
  }
  return FPH_OK;
}

}  // namespace

extern "C" {

int fph_ssh_create(fph_ssh_t* out, const fph_lattice_t* lat, double g, int32_t max_rhs) {
  if (out == nullptr || lat == nullptr) return FPH_E_NULL;
  *out = nullptr;
  if (lat->L < 4 || lat->L % 2 || lat->L > 64 || lat->Ltau < 2 || lat->Ltau % 2 || lat->Ltau > 65535 ||
      !std::isfinite(lat->dtau) || !std::isfinite(lat->t) || !std::isfinite(lat->mu) ||
      !std::isfinite(lat->alpha) || lat->dtau <= 0.0)
    return FPH_E_LATTICE;
  if (!std::isfinite(g)) return FPH_E_ARG;
  if (max_rhs < 1 || max_rhs > 65535) return FPH_E_NRHS;
  fph_ssh_s* c = new fph_ssh_s();
  std::memset(c, 0, sizeof(*c));
  c->G.L = lat->L;
  c->G.N = lat->L * lat->L;
  c->G.Ltau = lat->Ltau;
  c->G.d = (long)c->G.N * lat->Ltau;
  c->G.dtau = lat->dtau;
  c->G.t = lat->t;
  c->G.mu = lat->mu;
  c->G.alpha = lat->alpha;
  c->G.g = g;
  c->max_rhs = max_rhs;
  const int nb = c->G.N / 2;
  c->bpt = nb <= kNT ? 1 : nb <= 2 * kNT ? 2 : nb <= 4 * kNT ? 4 : 8;
  const long d = c->G.d;
  hipError_t e = hipSuccess;
#define SSH_ALLOC(ptr, bytes) \
  if (e == hipSuccess) e = hipMalloc((void**)&(ptr), (bytes));
  SSH_ALLOC(c->x, d * sizeof(double));
  SSH_ALLOC(c->hop, 2 * d * sizeof(double2));
  SSH_ALLOC(c->Et, d * sizeof(double));
  SSH_ALLOC(c->tmp, (size_t)max_rhs * d * sizeof(double));
  SSH_ALLOC(c->r, (size_t)max_rhs * d * sizeof(double));
  SSH_ALLOC(c->p, (size_t)max_rhs * d * sizeof(double));
  SSH_ALLOC(c->p2, (size_t)max_rhs * d * sizeof(double));
  SSH_ALLOC(c->q, (size_t)max_rhs * d * sizeof(double));
  SSH_ALLOC(c->z, (size_t)max_rhs * d * sizeof(double));
  // partials: kRedBlocks per right-hand side from the vector kernels, Ltau from the operator
  SSH_ALLOC(c->part, (size_t)max_rhs * (lat->Ltau > kXrBlocks ? lat->Ltau : kXrBlocks) * sizeof(double));
  SSH_ALLOC(c->part2, (size_t)max_rhs * (lat->Ltau > kRedBlocks ? lat->Ltau : kRedBlocks) * sizeof(double));
  SSH_ALLOC(c->part3, (size_t)max_rhs * (lat->Ltau > kRedBlocks ? lat->Ltau : kRedBlocks) * sizeof(double));
  SSH_ALLOC(c->st, 2 * (size_t)max_rhs * sizeof(CgState));
  SSH_ALLOC(c->hop32, 2 * d * sizeof(float2));
  SSH_ALLOC(c->Et32, d * sizeof(float));
  SSH_ALLOC(c->r32, (size_t)max_rhs * d * sizeof(float));
  SSH_ALLOC(c->z32, (size_t)max_rhs * d * sizeof(float));
  SSH_ALLOC(c->pa32, (size_t)max_rhs * d * sizeof(float));
  SSH_ALLOC(c->pb32, (size_t)max_rhs * d * sizeof(float));
  SSH_ALLOC(c->q32, (size_t)max_rhs * d * sizeof(float));
  SSH_ALLOC(c->tmp32, (size_t)max_rhs * d * sizeof(float));
  SSH_ALLOC(c->u32, (size_t)max_rhs * d * sizeof(float));
#undef SSH_ALLOC
  if (e == hipSuccess)
    e = hipHostMalloc((void**)&c->st_host, (size_t)max_rhs * sizeof(CgState), hipHostMallocDefault);
  if (e != hipSuccess) {
    fph_ssh_destroy(c);
    return fph::record_hip_error(e);
  }
  *out = c;
  return FPH_OK;
}

int fph_ssh_destroy(fph_ssh_t c) {
  if (c == nullptr) return FPH_E_NULL;
  (void)hipDeviceSynchronize();
  void* ptrs[] = {c->x,   c->hop,   c->Et,  c->tmp,  c->r,    c->p,    c->p2,   c->q,   c->z,
                  c->part, c->part2, c->part3, c->st, c->hop32, c->Et32, c->r32, c->z32, c->pa32,
                  c->pb32, c->q32, c->tmp32, c->u32};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (c->st_host) (void)hipHostFree(c->st_host);
  delete c;
  return FPH_OK;
}

int ssh_set_field(fph_ssh_t c, const double* x_dev, void* stream) {
  if (c == nullptr || x_dev == nullptr) return FPH_E_NULL;
  hipStream_t s = (hipStream_t)stream;
  SSH_CHECK(hipMemcpyAsync(c->x, x_dev, c->G.d * sizeof(double), hipMemcpyDeviceToDevice, s));
  hipLaunchKernelGGL(k_ssh_tables, dim3(c->G.Ltau), dim3(kNT), c->G.N * sizeof(double), s, c->G,
                     (const double*)c->x, c->hop, c->Et, c->hop32, c->Et32);
  SSH_CHECK(hipGetLastError());
  c->have_field = true;
  if (c->pc != nullptr) return fph_set_field(c->pc, x_dev, c->pc_a1, c->pc_a2, stream);
  return FPH_OK;
}

int ssh_matvec(fph_ssh_t c, int32_t op, int32_t nrhs, const double* in_dev, double* out_dev,
               void* stream) {
  if (c == nullptr || in_dev == nullptr || out_dev == nullptr) return FPH_E_NULL;
  if (!c->have_field) return FPH_E_NOFIELD;
  if (op < FPH_OP_M || op > FPH_OP_MTM) return FPH_E_PREC;
  if (nrhs < 1 || nrhs > c->max_rhs) return FPH_E_NRHS;
  const long bytes = (long)nrhs * c->G.d * 8;
  const char *a = (const char*)in_dev, *b = (const char*)out_dev;
  if (a < b + bytes && b < a + bytes) return FPH_E_ARG;
  SSH_CHECK(launch_apply(c, op, nrhs, in_dev, out_dev, (hipStream_t)stream));
  return FPH_OK;
}

int ssh_force(fph_ssh_t c, int32_t nrhs, const double* u_dev, double* grad_dev, double scale,
              const double* scale_dev, void* stream) {
  if (c == nullptr || u_dev == nullptr || grad_dev == nullptr) return FPH_E_NULL;
  if (!c->have_field) return FPH_E_NOFIELD;
  if (nrhs < 1 || nrhs > c->max_rhs) return FPH_E_NRHS;
  if (!std::isfinite(scale)) return FPH_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  SSH_CHECK((launch_apply_op<double, 0>(c, nrhs, u_dev, c->tmp, s)));  // y = M u
  SSH_CHECK(launch_force(c, nrhs, u_dev, c->tmp, scale, scale_dev, grad_dev, s));
  return FPH_OK;
}

int ssh_action(fph_ssh_t c, int32_t nrhs, const double* b_dev, const double* u_dev, double* out_dev,
               void* stream) {
  if (c == nullptr || b_dev == nullptr || u_dev == nullptr || out_dev == nullptr) return FPH_E_NULL;
  if (nrhs < 1 || nrhs > c->max_rhs) return FPH_E_NRHS;
  hipStream_t s = (hipStream_t)stream;
  SSH_CHECK(dots(c, nrhs, b_dev, u_dev, s));
  hipLaunchKernelGGL(k_sum_rhs, dim3(nrhs), dim3(256), 0, s, kRedBlocks, (const double*)c->part, out_dev);
  SSH_CHECK(hipGetLastError());
  return FPH_OK;
}

int ssh_set_preconditioner(fph_ssh_t c, fph_handle_t h, double a1, double a2) {
  if (c == nullptr) return FPH_E_NULL;
  if (h == nullptr) {
    c->pc = nullptr;
    return FPH_OK;
  }
  fph_lattice_t lat;
  int32_t mr = 0;
  const int rc = fph_get_lattice(h, &lat, &mr);
  if (rc != FPH_OK) return rc;
  if (lat.L != c->G.L || lat.Ltau != c->G.Ltau || lat.dtau != c->G.dtau || lat.t != c->G.t ||
      lat.mu != c->G.mu || lat.alpha != c->G.alpha)
    return FPH_E_LATTICE;
  if (!std::isfinite(a1) || !std::isfinite(a2)) return FPH_E_ARG;
  c->pc = h;
  c->pc_max_rhs = mr;
  c->pc_a1 = a1;
  c->pc_a2 = a2;
  return FPH_OK;
}

int ssh_solve(fph_ssh_t c, int32_t nrhs, const double* b_dev, double* u_dev, const fph_pcg_opts_t* opts,
              fph_pcg_stats_t* stats_host, void* stream) {
  if (c == nullptr || b_dev == nullptr || u_dev == nullptr || opts == nullptr) return FPH_E_NULL;
  if (!c->have_field) return FPH_E_NOFIELD;
  if (nrhs < 1 || nrhs > c->max_rhs) return FPH_E_NRHS;
  if ((opts->prec != FPH_F64 && opts->prec != FPH_F32_REFINED) || opts->use_precond < 0 ||
      opts->use_precond > 1)
    return FPH_E_PREC;
  const bool pre = opts->use_precond != 0;
  if (pre && c->pc == nullptr) return FPH_E_ARG;
  if (pre && nrhs > c->pc_max_rhs) return FPH_E_NRHS;
  if (!(opts->tol > 0.0) || !std::isfinite(opts->tol) || opts->maxiter < 1 || opts->chunk < 0)
    return FPH_E_ARG;
  if (opts->prec == FPH_F32_REFINED) {
    if (opts->max_outer < 0 || !(opts->ru_delta >= 0.0)) return FPH_E_ARG;
    return solve_refined(c, nrhs, b_dev, u_dev, opts, stats_host, stream);
  }
  hipStream_t s = (hipStream_t)stream;
  const long d = c->G.d;
  const long n = (long)nrhs * d;
  const int chunk = opts->chunk > 0 ? (opts->chunk < kMaxChunk ? opts->chunk : kMaxChunk) : 64;
  double* z = pre ? c->z : c->r;  // z = F F^T r, or r itself
  const double* p2 = pre ? c->part2 : c->part;
  auto precondition = [&]() -> int {
    return pre ? fph_precond_apply(c->pc, FPH_PC_FFT, FPH_F64, nrhs, c->r, c->z, stream) : FPH_OK;
  };
  auto sum_host = [&](std::vector<double>& out) -> int {
    std::vector<double> part((size_t)nrhs * kRedBlocks);
    SSH_CHECK(hipStreamSynchronize(s));
    SSH_CHECK(hipMemcpy(part.data(), c->part, part.size() * sizeof(double), hipMemcpyDeviceToHost));
    out.assign(nrhs, 0.0);
    for (int r = 0; r < nrhs; ++r)
      for (int k = 0; k < kRedBlocks; ++k) out[r] += part[(size_t)r * kRedBlocks + k];
    return FPH_OK;
  };
  std::vector<double> bb, rr, act;
  SSH_CHECK(dots(c, nrhs, b_dev, b_dev, s));
  int rc = sum_host(bb);
  if (rc != FPH_OK) return rc;
  for (int r = 0; r < nrhs; ++r) {
    CgState& S = c->st_host[r];
    std::memset(&S, 0, sizeof(S));
    S.tol2 = opts->tol * opts->tol;
    S.maxiter = opts->maxiter;
    S.bb = bb[r];
  }
  SSH_CHECK(hipMemcpyAsync(c->st, c->st_host, nrhs * sizeof(CgState), hipMemcpyHostToDevice, s));
  // r = b - A u (or b for a zero guess), z = F F^T r, p = z
  if (opts->zero_guess) {
    SSH_CHECK(hipMemsetAsync(u_dev, 0, n * sizeof(double), s));
    SSH_CHECK(hipMemcpyAsync(c->r, b_dev, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  } else {
    SSH_CHECK(launch_apply(c, FPH_OP_MTM, nrhs, u_dev, c->r, s));
    hipLaunchKernelGGL(k_sub_from, dim3(grid_for(n)), dim3(256), 0, s, n, b_dev, c->r);
    SSH_CHECK(hipGetLastError());
  }
  rc = precondition();
  if (rc != FPH_OK) return rc;
  SSH_CHECK(hipMemcpyAsync(c->p, z, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  double* pc = c->p;   // the current direction
  double* pn = c->p2;  // receives the next one
  SSH_CHECK(dots(c, nrhs, c->r, c->r, s));
  if (pre) SSH_CHECK(dots(c, nrhs, c->r, c->z, s, c->part2));
  hipLaunchKernelGGL(k_cg_scalar, dim3(nrhs), dim3(256), 0, s, 0, kRedBlocks, kRedBlocks, (const double*)c->part,
                     p2, c->st);
  SSH_CHECK(hipGetLastError());
  const int matvecs = opts->zero_guess ? 0 : 1;
  const bool fused = mtm_fusable(c);
  CgState* sa = c->st;               // the current state
  CgState* sb = c->st + c->max_rhs;  // the fused CG's next state
  for (int it = 0;;) {
    for (int k = 0; k < chunk; ++k, ++it) {
      // p = z + beta p (beta = 0 at the start, where p already holds z), formed
      // inside the M launch into pn; q = M^T M p with the p . q partials per slice
      const double* pq = c->part2;
      if (fused) {
        // also finishes the previous step's scalars (sa -> sb)
        MtmCg<double> a;
        a.zv = z;
        a.pnew = pn;
        a.st_old = sa;
        a.st_new = sb;
        a.part_rr = c->part;
        a.part_rz = p2;
        a.nbz = pre ? kRedBlocks : kXrBlocks;
        a.from_state = k == 0;
        SSH_CHECK((launch_mtm_fused<double, true>(c, nrhs, pc, c->q, s, true, c->part3, a)));
        std::swap(sa, sb);
        pq = c->part3;
      } else {
        SSH_CHECK((launch_apply_op<double, 0, true>(c, nrhs, pc, c->tmp, s, nullptr, z, pn)));  // state in c->st
        SSH_CHECK((launch_apply_op<double, 1>(c, nrhs, c->tmp, c->q, s, pn, nullptr, nullptr, c->part2)));
      }
      // alpha, u += alpha p, r -= alpha q with the |r|^2 partials (into part:
      // the p.q partials are still being read by other blocks)
      hipLaunchKernelGGL(k_cg_xr<double>, dim3(kXrBlocks, nrhs), dim3(256), 0, s, d, sa, c->G.Ltau, pq,
                         (const double*)pn, (const double*)c->q, u_dev, c->r, c->part);
      SSH_CHECK(hipGetLastError());
      rc = precondition();
      if (rc != FPH_OK) return rc;
      if (pre) SSH_CHECK(dots(c, nrhs, c->r, c->z, s, c->part2));
      if (!fused || k + 1 == chunk) {  // the fused launch of the next step does it otherwise
        hipLaunchKernelGGL(k_cg_scalar, dim3(nrhs), dim3(256), 0, s, 2, kXrBlocks, pre ? kRedBlocks : kXrBlocks,
                           (const double*)c->part,
                           p2, sa);
        SSH_CHECK(hipGetLastError());
      }
      std::swap(pc, pn);
    }
    SSH_CHECK(hipMemcpyAsync(c->st_host, sa, nrhs * sizeof(CgState), hipMemcpyDeviceToHost, s));
    SSH_CHECK(hipStreamSynchronize(s));
    bool all = true;
    for (int r = 0; r < nrhs; ++r) all = all && c->st_host[r].done;
    if (all || it >= opts->maxiter) break;
  }
  // true residual and S_F = b . u
  SSH_CHECK(launch_apply(c, FPH_OP_MTM, nrhs, u_dev, c->r, s));
  hipLaunchKernelGGL(k_sub_from, dim3(grid_for(n)), dim3(256), 0, s, n, b_dev, c->r);
  SSH_CHECK(hipGetLastError());
  SSH_CHECK(dots(c, nrhs, c->r, c->r, s));
  rc = sum_host(rr);
  if (rc != FPH_OK) return rc;
  SSH_CHECK(dots(c, nrhs, b_dev, u_dev, s));
  rc = sum_host(act);
  if (rc != FPH_OK) return rc;
  if (stats_host) {
    for (int r = 0; r < nrhs; ++r) {
      const CgState& S = c->st_host[r];
      fph_pcg_stats_t& o = stats_host[r];
      std::memset(&o, 0, sizeof(o));
      o.iters = S.iters;
      o.outer_iters = 0;
      o.matvecs = matvecs + S.iters + 1;
      o.rel_resid = bb[r] > 0.0 ? std::sqrt(rr[r] / bb[r]) : std::sqrt(rr[r]);
      o.action = act[r];
      o.status = S.status;
      if (std::isfinite(o.rel_resid) && o.rel_resid < opts->tol) o.status |= FPH_ST_CONVERGED;
      else if (!(S.status & (FPH_ST_BREAKDOWN | FPH_ST_NONFINITE))) o.status |= FPH_ST_MAXITER;
    }
  }
  return FPH_OK;
}

}  // extern "C"

fph_handle_t fph::ssh_precond(fph_ssh_t c) { return c ? c->pc : nullptr; }

int fph::ssh_info(fph_ssh_t c, fph_lattice_t* lat, int32_t* max_rhs, double* g) {
  if (c == nullptr) return FPH_E_NULL;
  if (lat) {
    lat->L = c->G.L;
    lat->Ltau = c->G.Ltau;
    lat->dtau = c->G.dtau;
    lat->t = c->G.t;
    lat->mu = c->G.mu;
    lat->alpha = c->G.alpha;
  }
  if (max_rhs) *max_rhs = c->max_rhs;
  if (g) *g = c->G.g;
  return FPH_OK;
}
