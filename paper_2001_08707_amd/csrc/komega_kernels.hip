// komega_kernels.hip -- gfx950 kernels of one shifted Krylov iteration.
//
// One iteration n (Kawamura et al., K-omega, Sec. 2.2) is two launches, plus
// a third when every x^(k) is kept:
//
//  k_spmv  q = H r_n for the built-in operator, fused with the partial sums
//          of t = r_n^T q (COCG) / r_n^H q (CG) / r~_n^H q (BiCG).  Its work-
//          group 0 meanwhile finalises step n-1: the O(N_z) shift recurrences
//          (Eqs. EQ-SHIFTEDCG-PI, -alpha, -beta), the projected y/u update
//          (Eqs. EQ-SHIFTEDCG-y/u), the seed switch (Sec. 2.2.4), residual
//          norms and the convergence test.  Nothing in q = H r depends on them.
//  k_shift (whole-x mode) x^k += alpha^k p^k, p^k = r_n/pi^k + beta^k p^k
//          (Eqs. EQ-SHIFTEDCG-x/-p) with the coefficients of step n-1.
//  k_seed  every work-group re-derives alpha_n, gamma_n from the partial sums
//          of t (Eq. EQ-REC-ALPHA-N2) and applies r_{n+1} = (1 + gamma - alpha
//          A) r_n - gamma r_{n-1} with A r = z_s r - q (Eq. EQ-CG-RN-3REC),
//          fused with the partial sums of rho_{n+1}, ||r_{n+1}||^2, P r_{n+1}.
//
// After the last iteration of a batch k_finalize (one work-group per
// right-hand side) finalises the last step.  Reductions use neither atomics
// nor fences: each group writes its partial sums to its own slot and the
// consumer of the next launch adds the slots in slot order, so results are
// bitwise reproducible and identical in every group that re-derives them.
#include <float.h>
#include <limits.h>

#include "komega_internal.h"

namespace kw {

constexpr int NW = TPB / 64;  // waves per work-group
constexpr int XCD_COUNT = 8;  // accelerator complex dies of an MI355X, each with its own L2

// ------------------------------------------------------------- reductions
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sums K values over the work-group; the totals are valid in thread 0.
template <int K>
__device__ inline void block_sum(double (&v)[K]) {
  __shared__ double sh[K > 0 ? K * NW : 1];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) sh[k * NW + w] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double s = sh[k * NW];
#pragma unroll
      for (int j = 1; j < NW; ++j) s += sh[k * NW + j];
      v[k] = s;
    }
  }
  __syncthreads();
}

// Sums slots [0, n) of `part` (stride `stride` doubles, first `used` of
// each meaningful) in slot order into the LDS array `tot` (K values, zeros
// beyond `used`), visible to every thread on return.  Every work-group that
// calls this on the same slots obtains bitwise the same totals, which is
// what lets each group of k_seed re-derive alpha on its own.  The values are
// reduced four at a time so that few registers are held; each value's
// summation order (per thread over slots, then the block tree) does not
// depend on that grouping.
template <int K>
__device__ inline void reduce_slots(const double* part, int n, int stride, int used, double* tot) {
  constexpr int C = K < 4 ? K : 4;
  for (int k0 = 0; k0 < K; k0 += C) {
    double v[C];
#pragma unroll
    for (int c = 0; c < C; ++c) v[c] = 0.0;
    if (k0 < used) {
      for (int b = threadIdx.x; b < n; b += TPB) {
#pragma unroll
        for (int c = 0; c < C; ++c)
          if (k0 + c < used) v[c] += part[(size_t)b * stride + k0 + c];
      }
      block_sum<C>(v);
    }
    if (threadIdx.x == 0) {
#pragma unroll
      for (int c = 0; c < C; ++c)
        if (k0 + c < K) tot[k0 + c] = k0 + c < used ? v[c] : 0.0;
    }
  }
  __syncthreads();
}

// Layout of the partial-sum slots.
constexpr int SLOT_A = 2;                       // Re, Im of r.q
constexpr int SLOT_B = 3 + 2 * KOMEGA_MAX_NL;   // rho (2), nu (1), P r (2 nl)
__device__ inline double* slotsA(const DevSolver& ds, int rhs) {
  return reinterpret_cast<double*>(ds.partA) + (size_t)rhs * ds.maxblk * SLOT_A;
}
__device__ inline double* slotsB(const DevSolver& ds, int rhs) {
  return reinterpret_cast<double*>(ds.partB) + (size_t)rhs * ds.maxblk * SLOT_B;
}

// The rows and work share of one work-group.  Uniform layout: grid
// (LEAD + groups, nrhs), system r at rows r*M.  Batched layout: entry
// blockIdx.x of the work list names (system, group); the system's rows come
// from soff and its group count is stream_blocks of its size, so its
// grid-stride pattern and slot order equal those of a stand-alone solve.
// g < 0 marks the finaliser group of k_spmv / k_dot.  BATCH = false compiles
// the uniform layout only (operators that batched solvers reject).
struct Blk {
  int rhs, g, ng;
  int64_t off, M;
};
template <int LEAD, bool BATCH = true>
__device__ inline Blk blk_of(const DevSolver& ds, const int2* wl) {
  Blk b;
  if (BATCH && ds.soff) {
    const int2 e = wl[blockIdx.x];
    b.rhs = e.x;
    b.g = e.y;
    b.off = ds.soff[e.x];
    b.M = ds.soff[e.x + 1] - b.off;
    b.ng = (int)stream_blocks(b.M);
  } else {
    b.rhs = blockIdx.y;
    b.g = (int)blockIdx.x - LEAD;
    b.ng = (int)gridDim.x - LEAD;
    b.off = (int64_t)b.rhs * ds.M;
    b.M = ds.M;
  }
  return b;
}
// Partial-sum slots written for system rhs (uniform: the launch's count).
__device__ inline int nslots(const DevSolver& ds, int rhs, int uniform) {
  return ds.soff ? (int)stream_blocks(ds.soff[rhs + 1] - ds.soff[rhs]) : uniform;
}

__device__ inline void fail(RhsState* S, int code) {
  S->status = code;
  S->stop = 1;
  S->pending = 0;
  S->step_pending = 0;
}

// Inner product selected by the method: bilinear for COCG (App. A),
// conjugated otherwise (CG: Eq. EQ-REC-RHO; BiCG: shadow on the left).
template <class V, int DK>
__device__ inline zc mdot(V a, V b) {
  return DK == 0 ? VT<V>::bil(a, b) : VT<V>::ses(a, b);
}

__device__ inline double zabs(zc a) { return hypot(a.x, a.y); }

// ---------------------------------------------------- seed coefficients
// alpha_n = rho_n / (r^T A r - (beta_{n-1}/alpha_{n-1}) rho_n), r^T A r =
// z_s rho_n - r^T H r (Eq. EQ-REC-ALPHA-N2); gamma_n = alpha_n beta_{n-1}/alpha_{n-1};
// r_{n+1} = (1 + gamma - alpha z_s) r_n + alpha H r_n - gamma r_{n-1} (Eq. EQ-CG-RN-3REC).
// tm is the inner product of the memory vectors; the true value carries the
// memory scale sc twice (sc^2, or |sc|^2 for the conjugated CG product).
struct SeedCoef {
  zc alpha, gamma, cr, cq, co;
  int err;
};

__device__ inline SeedCoef seed_coef(const DevSolver& ds, const RhsState* S, zc tm) {
  SeedCoef c;
  const zc sc = S->sc, rho = S->rho, ba = S->ba, zs = S->zs;
  const zc f = (ds.method == KOMEGA_CG_R || ds.method == KOMEGA_CG_C) ? zmk(zabs2(sc), 0.0) : zmul(sc, sc);
  const zc t = zmul(f, tm);
  const zc den = zsub(zsub(zmul(zs, rho), t), zmul(ba, rho));
  c.err = !zfinite(den) ? KOMEGA_E_NONFINITE : (zzero(den) ? KOMEGA_E_BREAKDOWN : 0);
  if (c.err) return c;
  c.alpha = zdiv(rho, den);
  c.gamma = zmul(c.alpha, ba);
  c.cr = zmul(zsub(zadd(zmk(1.0, 0.0), c.gamma), zmul(c.alpha, zs)), sc);
  c.cq = zmul(c.alpha, sc);
  c.co = zneg(zmul(c.gamma, S->so));
  return c;
}

// A value every lane of the work-group holds (read from LDS, or computed
// from such values), moved to scalar registers: the per-shift loops then
// spend no vector registers on the step's scalars.
__device__ inline double uniform(double v) {
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readfirstlane((int)(u & 0xffffffffLL));
  const int hi = __builtin_amdgcn_readfirstlane((int)(u >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ inline zc uniform(zc v) { return zmk(uniform(v.x), uniform(v.y)); }

// ------------------------------------------------ finalisation of a step
// Run by one work-group after k_seed: reduces its partial sums (rho_{n+1},
// nu_{n+1} = ||r_{n+1}||^2, P r_{n+1}; the memory vector r_{n+1} has scale 1)
// and performs the O(N_z) part of the step: shift recurrences, projected
// update or whole-x coefficients, seed switch, residuals, convergence.
__device__ void finalize_step(const DevSolver& ds, int rhs, int nblkB) {
  __shared__ zc s_alpha, s_gamma, s_beta, s_zs, s_c0, s_c1, s_rho1;
  __shared__ zc s_pr[KOMEGA_MAX_NL];
  __shared__ double s_nu1;
  __shared__ int s_err, s_sw, s_best, s_it;
  __shared__ double s_bv[NW];
  __shared__ int s_bi[NW];
  __shared__ double s_mx[NW];
  __shared__ int s_tb;
  RhsState* S = ds.st + rhs;
  const int tid = threadIdx.x;
  const int nz = ds.nz, nl = ds.nl;
  const size_t base = (size_t)rhs * nz;

  __shared__ double red[SLOT_B];
  reduce_slots<SLOT_B>(slotsB(ds, rhs), nslots(ds, rhs, nblkB), SLOT_B, 3 + 2 * nl, red);
  if (tid == 0) {
    const int it = S->iter;
    s_it = it;
    s_err = INT_MAX;
    s_alpha = S->alpha;
    s_gamma = S->gamma;
    s_zs = S->zs;
    s_rho1 = zmk(red[0], red[1]);
    s_nu1 = red[2];
    s_beta = zdiv(s_rho1, S->rho);  // beta_n = rho_{n+1} / rho_n (Eq. EQ-REC-BETA)
    for (int l = 0; l < nl; ++l) s_pr[l] = zmk(red[3 + 2 * l], red[4 + 2 * l]);
    if (!zfinite(s_rho1) || !isfinite(s_nu1)) s_err = -1;
    // blocked whole-x update: index of this step in the block (-1: the first
    // step of a new generation)
    s_tb = (S->blk_gen == ds.blk_gen) ? S->blk_cnt : -1;
    if (nl == 0 && ds.xblk > 1 && s_tb >= ds.xblk) s_err = -2;
    if (ds.hist_cap > 0 && it < ds.hist_cap) {
      const size_t h = (size_t)rhs * ds.hist_cap + it;
      ds.h_alpha[h] = s_alpha;
      ds.h_beta[h] = s_beta;
      ds.h_zs[h] = s_zs;
      for (int l = 0; l < nl; ++l) ds.h_pr[h * nl + l] = s_pr[l];
    }
  }
  __syncthreads();
  if (s_err == -1 || s_err == -2) {
    if (tid == 0) {
      fail(S, s_err == -1 ? KOMEGA_E_NONFINITE : KOMEGA_E_STATE);
      S->blk_cnt = -1;  // the block is not applied
    }
    return;
  }
  const bool xb = nl == 0 && ds.xblk > 1;
  const int tb = s_tb < 0 ? 0 : s_tb;
  if (xb && s_tb < 0) {
    // a new block: no shift touched yet
    for (int k = tid; k < nz; k += TPB) ds.btouch[base + k] = 0;
  }
  const zc alpha = uniform(s_alpha), gamma = uniform(s_gamma), beta = uniform(s_beta), zs = uniform(s_zs);
  const zc one_g = uniform(zadd(zmk(1.0, 0.0), gamma));

  // Shift recurrences for the active shifts.
  double bv = DBL_MAX;
  int bi = INT_MAX;
  for (int k = tid; k < nz; k += TPB) {
    const size_t kk = base + k;
    if (!ds.active[kk]) {
      ds.apply[kk] = 0;
      if (xb) {  // an identity step: x, p unchanged
        ds.bstep[bstep_at(nz, rhs, tb, 0, k)] = zmk(0.0, 0.0);
        ds.bstep[bstep_at(nz, rhs, tb, 1, k)] = zmk(1.0, 0.0);
        ds.bstep[bstep_at(nz, rhs, tb, 2, k)] = zmk(0.0, 0.0);
      }
      continue;
    }
    const zc sigma = zsub(ds.z[k], zs);
    const zc pk = ds.pi[kk], pko = ds.pio[kk];
    // pi_{n+1} = (1 + gamma + alpha sigma) pi_n - gamma pi_{n-1}  (Eq. EQ-SHIFTEDCG-PI)
    const zc pn = zsub(zmul(zadd(one_g, zmul(alpha, sigma)), pk), zmul(gamma, pko));
    if (!zfinite(pn)) { atomicMin(&s_err, 2 * k); continue; }
    if (zzero(pn)) { atomicMin(&s_err, 2 * k + 1); continue; }
    const zc ratio = zdiv(pk, pn);
    const zc a_k = zmul(ratio, alpha);              // Eq. EQ-SHIFTEDCG-alpha
    const zc b_k = zmul(zmul(ratio, ratio), beta);  // Eq. EQ-SHIFTEDCG-beta
    if (nl > 0) {
      for (int l = 0; l < nl; ++l) {
        const size_t o = kk * nl + l;
        const zc uo = ds.u[o];
        ds.y[o] = zadd(ds.y[o], zmul(a_k, uo));                  // Eq. EQ-SHIFTEDCG-y
        ds.u[o] = zadd(zdiv(s_pr[l], pn), zmul(b_k, uo));        // Eq. EQ-SHIFTEDCG-u
      }
    } else if (xb) {
      // step tb of the block: x += a_k p, p = (1/pi_{n+1}) r_{n+1} + b_k p;
      // k_block_map composes the block's steps when it is applied
      ds.bstep[bstep_at(nz, rhs, tb, 0, k)] = a_k;
      ds.bstep[bstep_at(nz, rhs, tb, 1, k)] = b_k;
      ds.bstep[bstep_at(nz, rhs, tb, 2, k)] = zinv(pn);
      ds.btouch[kk] = 1;
    } else {
      ds.ak[kk] = a_k;
      ds.bk[kk] = b_k;
      ds.ck[kk] = zinv(pn);
      ds.apply[kk] = 1;
    }
    ds.pio[kk] = pk;
    ds.pi[kk] = pn;
    const double m = zabs(pn);
    if (m < bv || (m == bv && k < bi)) { bv = m; bi = k; }
  }
  // arg min |pi_{n+1}| over active shifts, lowest index on ties
  {
    const int w = tid >> 6, lane = tid & 63;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      double ov = __shfl_xor(bv, off, 64);
      int oi = __shfl_xor(bi, off, 64);
      if (ov < bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
    }
    if (lane == 0) { s_bv[w] = bv; s_bi[w] = bi; }
  }
  __syncthreads();
  if (tid == 0) {
    double b = s_bv[0];
    int i = s_bi[0];
    for (int j = 1; j < NW; ++j)
      if (s_bv[j] < b || (s_bv[j] == b && s_bi[j] < i)) { b = s_bv[j]; i = s_bi[j]; }
    s_best = i;
    s_sw = 0;
    if (s_err == INT_MAX && !(ds.flags & KOMEGA_F_NO_SWITCH) && i != INT_MAX && b < 1.0) {
      s_sw = 1;
      s_c1 = ds.pi[base + i];
      s_c0 = ds.pio[base + i];
    }
  }
  __syncthreads();
  if (s_err != INT_MAX) {
    if (tid == 0) {
      fail(S, (s_err & 1) ? KOMEGA_E_SHIFT_BREAKDOWN : KOMEGA_E_NONFINITE);
      S->blk_cnt = -1;  // a partly composed step: the block is not applied
    }
    return;
  }
  const int sw = s_sw;
  const zc c0 = s_c0, c1 = s_c1;
  // Seed switch (Sec. 2.2.4): residuals of the new seed are r / pi^seed, so
  // every pi is divided by the new seed's pi at both levels n and n+1.
  const double nu1 = s_nu1;
  const double nus = sw ? nu1 / zabs2(c1) : nu1;
  const double sq = sqrt(nus);
  const double bnorm = S->bnorm;
  double mx = 0.0;
  for (int k = tid; k < nz; k += TPB) {
    const size_t kk = base + k;
    if (ds.active[kk]) {
      zc p = ds.pi[kk];
      if (sw) {
        p = zdiv(p, c1);
        ds.pi[kk] = p;
        ds.pio[kk] = zdiv(ds.pio[kk], c0);
      }
      // ||r^k|| / ||b|| = ||r|| / (|pi^k| ||b||)  (Eq. EQ-COLLINEAR)
      const double r = sq / (zabs(p) * bnorm);
      ds.res[kk] = r;
      if (ds.freeze_tol > 0.0 && r < ds.freeze_tol) ds.active[kk] = 0;
      mx = fmax(mx, r);
    } else {
      mx = fmax(mx, ds.res[kk]);
    }
  }
  {
    const int w = tid >> 6, lane = tid & 63;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
    if (lane == 0) s_mx[w] = mx;
  }
  __syncthreads();
  if (tid == 0) {
    const int it = s_it;
    for (int j = 1; j < NW; ++j) mx = fmax(mx, s_mx[j]);
    zc a = alpha, b = beta, r1 = s_rho1;
    if (sw) {
      const zc q = zdiv(c0, c1);
      a = zmul(a, q);
      b = zmul(b, zmul(q, q));
      if (ds.method == KOMEGA_CG_R || ds.method == KOMEGA_CG_C)
        r1 = zscale(1.0 / zabs2(c1), r1);
      else
        r1 = zdiv(r1, zmul(c1, c1));
      S->zs = ds.z[s_best];
      S->seed = s_best;
      S->nswitch += 1;
      S->so = zdiv(S->sc, c0);
      S->sc = zinv(c1);
    } else {
      S->so = S->sc;
      S->sc = zmk(1.0, 0.0);
    }
    if (ds.hist_cap > 0 && it < ds.hist_cap) {
      const size_t h = (size_t)rhs * ds.hist_cap + it;
      ds.h_seed[h] = S->seed;
      ds.h_sw[2 * h] = sw ? c0 : zmk(1.0, 0.0);
      ds.h_sw[2 * h + 1] = sw ? c1 : zmk(1.0, 0.0);
      ds.h_nu[h] = nus;
    }
    S->rho = r1;
    S->nu = nus;
    S->ba = zdiv(b, a);
    S->iter = it + 1;
    S->maxres = mx;
    S->pending = (nl == 0 && !xb) ? 1 : 0;
    S->step_pending = 0;
    if (xb) {
      S->blk_gen = ds.blk_gen;
      S->blk_cnt = tb + 1;
    }
    if (mx < ds.tol || nus == 0.0) {
      S->status = KOMEGA_CONVERGED;
      S->stop = 1;
    } else if (zabs(r1) <= 16.0 * DBL_EPSILON * nus) {
      S->status = KOMEGA_E_BREAKDOWN;
      S->stop = 1;
    } else if (it + 1 >= ds.itermax) {
      S->status = KOMEGA_E_MAXITER;
      S->stop = 1;
    }
  }
}

// Work-group 0 of k_spmv / k_dot: clears the whole-x flag of the previous
// step (its k_shift has run) and finalises the step k_seed left behind.
__device__ inline void finaliser_group(const DevSolver& ds, int rhs, int nblkB) {
  __shared__ int sp;
  RhsState* S = ds.st + rhs;
  if (threadIdx.x == 0) {
    S->pending = 0;
    sp = S->step_pending;
  }
  __syncthreads();
  if (sp) finalize_step(ds, rhs, nblkB);
}

// Stand-alone finalisation (end of a batch of iterations, and the reverse-
// communication update): one work-group per right-hand side.  Like the
// finaliser group it first consumes the whole-x flag: the k_shift launched
// after it must apply only a step finalised here, never again the step the
// last iteration's k_shift has already applied (a system that stopped in that
// iteration has no new step).
__global__ __launch_bounds__(TPB) void k_finalize(DevSolver ds, int nblkB) {
  finaliser_group(ds, blockIdx.y, nblkB);
}

// ----------------------------------------------------------------- k_seed
// Prologue: re-derive alpha_n, gamma_n from the r.q partial sums of k_spmv
// (every group obtains the same bits).  Body: r_{n+1} = cr R + cq Q + co RO
// on the memory vectors (Eq. EQ-CG-RN-3REC); the shadow of BiCG uses the
// conjugated coefficients (App. B).  INPLACE (reverse communication): R <-
// r_{n+1}, RO <- old R.  Otherwise RO <- r_{n+1} and the host swaps R and RO.
template <class V, int DK, bool SH, int NL, bool INPLACE>
__global__ __launch_bounds__(TPB) void k_seed(DevSolver ds, Buffers bf, const void* Pv, int nblkA) {
  const Blk bk = blk_of<0>(ds, ds.wl_b);
  const int rhs = bk.rhs;
  RhsState* S = ds.st + rhs;
  if (S->stop) return;
  __shared__ double tv[2];
  reduce_slots<2>(slotsA(ds, rhs), nslots(ds, rhs, nblkA), SLOT_A, 2, tv);
  const SeedCoef c = seed_coef(ds, S, zmk(tv[0], tv[1]));
  if (bk.g == 0 && threadIdx.x == 0) {
    if (c.err) {
      fail(S, c.err);
    } else {
      S->alpha = c.alpha;
      S->gamma = c.gamma;
      S->step_pending = 1;
    }
  }
  if (c.err) return;
  const zc cr = c.cr, cq = c.cq, co = c.co;
  const int64_t M = bk.M, off = bk.off, ldp = ds.M;
  V* __restrict__ R = reinterpret_cast<V*>(bf.R) + off;
  const V* __restrict__ Q = reinterpret_cast<const V*>(bf.Q) + off;
  V* __restrict__ RO = reinterpret_cast<V*>(bf.RO) + off;
  V* __restrict__ RN = bf.RN ? reinterpret_cast<V*>(bf.RN) + off : nullptr;
  V* Rs = nullptr;
  const V* Qs = nullptr;
  V* ROs = nullptr;
  if (SH) {
    Rs = reinterpret_cast<V*>(bf.Rs) + off;
    Qs = reinterpret_cast<const V*>(bf.Qs) + off;
    ROs = reinterpret_cast<V*>(bf.ROs) + off;
  }
  // P is [nl][ds.M]: shared by uniform right-hand sides, column block of a
  // batched system
  const V* __restrict__ P = reinterpret_cast<const V*>(Pv) + (ds.soff ? off : 0);
  const int nl = ds.nl;
  constexpr int K = 3 + 2 * NL;
  double acc[K];
#pragma unroll
  for (int k = 0; k < K; ++k) acc[k] = 0.0;

  const int64_t stride = (int64_t)bk.ng * TPB;
  for (int64_t i = (int64_t)bk.g * TPB + threadIdx.x; i < M; i += stride) {
    const V r = R[i], q = Q[i], ro = RO[i];
    const V rn = VT<V>::add(VT<V>::add(VT<V>::lin(cr, r), VT<V>::lin(cq, q)), VT<V>::lin(co, ro));
    if (INPLACE) { RO[i] = r; R[i] = rn; } else if (RN) { RN[i] = rn; } else { RO[i] = rn; }
    zc rho;
    if (SH) {
      const V rs = Rs[i], qs = Qs[i], ros = ROs[i];
      const V rsn = VT<V>::add(VT<V>::add(VT<V>::lin(zconj(cr), rs), VT<V>::lin(zconj(cq), qs)),
                               VT<V>::lin(zconj(co), ros));
      if (INPLACE) { ROs[i] = rs; Rs[i] = rsn; } else { ROs[i] = rsn; }
      rho = VT<V>::ses(rsn, rn);
    } else {
      rho = mdot<V, DK>(rn, rn);
    }
    acc[0] += rho.x;
    acc[1] += rho.y;
    acc[2] += VT<V>::nrm(rn);
#pragma unroll
    for (int l = 0; l < NL; ++l) {
      if (l < nl) {
        const zc pr = VT<V>::bil(P[(size_t)l * ldp + i], rn);
        acc[3 + 2 * l] += pr.x;
        acc[4 + 2 * l] += pr.y;
      }
    }
  }
  block_sum<K>(acc);
  if (threadIdx.x == 0) {
    double* slot = slotsB(ds, rhs) + (size_t)bk.g * SLOT_B;
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (k < 3 + 2 * nl) slot[k] = acc[k];
  }
}

// ------------------------------------------------------------------- init
// Partial sums of rho_0 (method product of b, or r~_0^H b), ||b||^2 and P b.
template <class V, int DK, bool SH, int NL>
__global__ __launch_bounds__(TPB) void k_init(DevSolver ds, Buffers bf, const void* Pv) {
  const Blk bk = blk_of<0>(ds, ds.wl_b);
  const int rhs = bk.rhs;
  const int64_t M = bk.M, off = bk.off, ldp = ds.M;
  const V* __restrict__ R = reinterpret_cast<const V*>(bf.R) + off;
  const V* Rs = SH ? reinterpret_cast<const V*>(bf.Rs) + off : nullptr;
  const V* __restrict__ P = reinterpret_cast<const V*>(Pv) + (ds.soff ? off : 0);
  const int nl = ds.nl;
  constexpr int K = 3 + 2 * NL;
  double acc[K];
#pragma unroll
  for (int k = 0; k < K; ++k) acc[k] = 0.0;
  const int64_t stride = (int64_t)bk.ng * TPB;
  for (int64_t i = (int64_t)bk.g * TPB + threadIdx.x; i < M; i += stride) {
    const V r = R[i];
    const zc rho = SH ? VT<V>::ses(Rs[i], r) : mdot<V, DK>(r, r);
    acc[0] += rho.x;
    acc[1] += rho.y;
    acc[2] += VT<V>::nrm(r);
#pragma unroll
    for (int l = 0; l < NL; ++l) {
      if (l < nl) {
        const zc pr = VT<V>::bil(P[(size_t)l * ldp + i], r);
        acc[3 + 2 * l] += pr.x;
        acc[4 + 2 * l] += pr.y;
      }
    }
  }
  block_sum<K>(acc);
  if (threadIdx.x == 0) {
    double* slot = slotsB(ds, rhs) + (size_t)bk.g * SLOT_B;
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (k < 3 + 2 * nl) slot[k] = acc[k];
  }
}

// Sets every per-solve scalar from the reduced sums: seed z[0], pi_0 =
// pi_{-1} = 1, u_0 = P b, y_0 = 0 (Sec. 2.2.1, Eqs. EQ-SHIFTEDCG-PI and -u).
__global__ __launch_bounds__(TPB) void k_init_fin(DevSolver ds, int nblkB) {
  const int rhs = blockIdx.y;
  const int nl = ds.nl;
  __shared__ double sv[SLOT_B];
  reduce_slots<SLOT_B>(slotsB(ds, rhs), nslots(ds, rhs, nblkB), SLOT_B, 3 + 2 * nl, sv);
  RhsState* S = ds.st + rhs;
  const int nz = ds.nz;
  const size_t base = (size_t)rhs * nz;
  const double bnorm = sqrt(sv[2]);
  for (int k = threadIdx.x; k < nz; k += TPB) {
    const size_t kk = base + k;
    ds.pi[kk] = zmk(1.0, 0.0);
    ds.pio[kk] = zmk(1.0, 0.0);
    ds.active[kk] = 1;
    ds.apply[kk] = 0;
    ds.res[kk] = bnorm > 0.0 ? 1.0 : 0.0;
    for (int l = 0; l < nl; ++l) {
      ds.u[kk * nl + l] = zmk(sv[3 + 2 * l], sv[4 + 2 * l]);
      ds.y[kk * nl + l] = zmk(0.0, 0.0);
    }
  }
  if (threadIdx.x < nl) ds.pb[(size_t)rhs * nl + threadIdx.x] = zmk(sv[3 + 2 * threadIdx.x], sv[4 + 2 * threadIdx.x]);
  if (threadIdx.x == 0) {
    const zc rho = zmk(sv[0], sv[1]);
    S->rho = rho;
    S->nu = sv[2];
    S->bnorm = bnorm;
    S->ba = zmk(0.0, 0.0);
    S->zs = ds.z[0];
    S->sc = zmk(1.0, 0.0);
    S->so = zmk(1.0, 0.0);
    S->alpha = S->gamma = S->cr = S->cq = S->co = zmk(0.0, 0.0);
    S->seed = 0;
    S->iter = 0;
    S->nswitch = 0;
    S->pending = 0;
    S->step_pending = 0;
    S->blk_cnt = 0;
    S->blk_gen = 0;  // the host's generations start at 1
    S->maxres = bnorm > 0.0 ? 1.0 : 0.0;
    S->status = KOMEGA_OK;
    S->stop = 0;
    if (bnorm == 0.0) {
      S->status = KOMEGA_CONVERGED;
      S->stop = 1;
    } else if (!zfinite(rho) || !isfinite(sv[2])) {
      S->status = KOMEGA_E_NONFINITE;
      S->stop = 1;
    } else if (zabs(rho) <= 16.0 * DBL_EPSILON * sv[2]) {
      S->status = KOMEGA_E_BREAKDOWN;
      S->stop = 1;
    }
  }
}

// Storage of the whole-x vectors x^k, p^k: the vector type itself, or
// complex64 with double arithmetic (XS<cf>).
template <class X> struct XS {
  static __device__ inline X ld(X a) { return a; }
  static __device__ inline X st(X a) { return a; }
};
template <> struct XS<cf> {
  static __device__ inline zc ld(cf a) { return widen(a); }
  static __device__ inline cf st(zc a) { return narrow(a); }
  static __device__ inline cf st(double a) { return narrow(zmk(a, 0.0)); }
};

// Offset of x^k_i of system rhs (first row off, M rows) in [system][nz][rows]
// storage; for uniform right-hand sides off = rhs*M gives [nrhs][nz][M].
__device__ inline size_t xoff(const DevSolver& ds, int64_t off, int64_t M, int k, int64_t i) {
  return (size_t)ds.nz * off + (size_t)k * M + i;
}

// R <- b, RO <- 0, shadow R~ <- bshadow or conj(b), RO~ <- 0; whole-x mode:
// p^k <- b, x^k <- 0 for every shift.
template <class V, class X>
__global__ __launch_bounds__(TPB) void k_init_copy(DevSolver ds, Buffers bf, const V* __restrict__ b,
                                                   const V* __restrict__ bsh, X* __restrict__ x) {
  const Blk bk = blk_of<0>(ds, ds.wl_b);
  const int64_t M = bk.M, off = bk.off;
  const int64_t stride = (int64_t)bk.ng * TPB;
  V* R = reinterpret_cast<V*>(bf.R) + off;
  V* RO = reinterpret_cast<V*>(bf.RO) + off;
  const V* bb = b + off;
  const bool sh = bf.Rs != nullptr;
  for (int64_t i = (int64_t)bk.g * TPB + threadIdx.x; i < M; i += stride) {
    const V v = bb[i];
    R[i] = v;
    RO[i] = VT<V>::zero();
    if (sh) {
      reinterpret_cast<V*>(bf.Rs)[off + i] = bsh ? bsh[off + i] : VT<V>::conj(v);
      reinterpret_cast<V*>(bf.ROs)[off + i] = VT<V>::zero();
    }
    if (ds.nl == 0) {
      for (int k = 0; k < ds.nz; ++k) {
        const size_t o = xoff(ds, off, M, k, i);
        reinterpret_cast<X*>(bf.p)[o] = XS<X>::st(v);
        x[o] = XS<X>::st(VT<V>::zero());
      }
    }
  }
}

// Streaming access to x^k, p^k: plain, or nontemporal (the stream is touched
// once per iteration, far more data than the caches hold).
template <class X, bool NT> struct Stream {
  static __device__ inline X ld(const X* p) { return *p; }
  static __device__ inline void st(X* p, X v) { *p = v; }
};
template <> struct Stream<zc, true> {
  typedef double v2 __attribute__((ext_vector_type(2)));
  static __device__ inline zc ld(const zc* p) {
    const v2 v = __builtin_nontemporal_load(reinterpret_cast<const v2*>(p));
    return zmk(v.x, v.y);
  }
  static __device__ inline void st(zc* p, zc a) {
    const v2 v = {a.x, a.y};
    __builtin_nontemporal_store(v, reinterpret_cast<v2*>(p));
  }
};
template <> struct Stream<cf, true> {
  typedef float v2 __attribute__((ext_vector_type(2)));
  static __device__ inline cf ld(const cf* p) {
    const v2 v = __builtin_nontemporal_load(reinterpret_cast<const v2*>(p));
    cf r;
    r.x = v.x;
    r.y = v.y;
    return r;
  }
  static __device__ inline void st(cf* p, cf a) {
    const v2 v = {a.x, a.y};
    __builtin_nontemporal_store(v, reinterpret_cast<v2*>(p));
  }
};
template <> struct Stream<double, true> {
  static __device__ inline double ld(const double* p) { return __builtin_nontemporal_load(p); }
  static __device__ inline void st(double* p, double a) { __builtin_nontemporal_store(a, p); }
};

// The two updates of k_shift with every product and sum in an explicit fused
// multiply-add chain, so the compiler has no contraction choice left and
// every launch shape (shift block, streaming mode) rounds identically.
__device__ inline zc shift_x(zc x, zc a, zc p) {  // x + a p
  return zmk(fma(a.x, p.x, fma(-a.y, p.y, x.x)), fma(a.x, p.y, fma(a.y, p.x, x.y)));
}
__device__ inline zc shift_p(zc c, zc r, zc b, zc p) {  // c r + b p
  const double re = fma(c.x, r.x, fma(-c.y, r.y, fma(b.x, p.x, -b.y * p.y)));
  const double im = fma(c.x, r.y, fma(c.y, r.x, fma(b.x, p.y, b.y * p.x)));
  return zmk(re, im);
}
__device__ inline double shift_x(double x, zc a, double p) { return fma(a.x, p, x); }
__device__ inline double shift_p(zc c, double r, zc b, double p) { return fma(c.x, r, b.x * p); }

// ------------------------------------------------------------ k_shift
// x^k += alpha^k p^k;  p^k = (1/pi^k_{n+1}) r_{n+1} + beta^k p^k
// (Eqs. EQ-SHIFTEDCG-x, EQ-SHIFTEDCG-p) for SB shifts per thread and one row
// per thread.  Layout x, p: [system][nz][rows], rows contiguous.  X is the
// storage type of x, p (V, or complex64 with double arithmetic); NT selects
// nontemporal streaming.  SWAP puts the shift blocks on the fastest grid
// dimension, so the blocks sharing a row tile (and its r_{n+1}) run together.
template <class V, class X, int SB, bool NT, bool SWAP>
__global__ __launch_bounds__(TPB) void k_shift(DevSolver ds, const V* __restrict__ RN,
                                               X* __restrict__ Xv, X* __restrict__ Pd) {
  const unsigned bt = SWAP ? blockIdx.y : blockIdx.x;  // row tile (or work-list entry)
  const unsigned bs = SWAP ? blockIdx.x : blockIdx.y;  // shift block
  int rhs;
  int64_t M, off, i;
  if (ds.soff) {
    const int2 e = ds.wl_t[bt];
    rhs = e.x;
    off = ds.soff[rhs];
    M = ds.soff[rhs + 1] - off;
    i = (int64_t)e.y * TPB + threadIdx.x;
  } else {
    rhs = blockIdx.z;
    M = ds.M;
    off = (int64_t)rhs * M;
    i = (int64_t)bt * TPB + threadIdx.x;
  }
  if (!ds.st[rhs].pending) return;
  const int k0 = bs * SB;
  if (i >= M) return;
  const int nz = ds.nz;
  const V rn = RN[off + i];
#pragma unroll
  for (int j = 0; j < SB; ++j) {
    const int k = k0 + j;
    if (k >= nz) break;
    const size_t kk = (size_t)rhs * nz + k;
    if (!ds.apply[kk]) continue;
    const zc a = ds.ak[kk], b = ds.bk[kk], c = ds.ck[kk];
    const size_t o = xoff(ds, off, M, k, i);
    const auto p = XS<X>::ld(Stream<X, NT>::ld(Pd + o));
    const auto x = XS<X>::ld(Stream<X, NT>::ld(Xv + o));
    Stream<X, NT>::st(Xv + o, XS<X>::st(shift_x(x, a, p)));
    Stream<X, NT>::st(Pd + o, XS<X>::st(shift_p(c, rn, b, p)));
  }
}

// ---------------------------------------------------------- k_block_map
// The map of a block of cnt steps, x <- x + E p + sum_s F_s r_s and
// p <- G p + sum_s H_s r_s, for every touched shift, from the scalars of its
// steps (a_s = alpha^k, b_s = beta^k, c_s = 1/pi^k; a shift inactive in a
// step has a = 0, b = 1, c = 0).  Unrolling x += a_s p, p = c_s r_s + b_s p
// (Eqs. EQ-SHIFTEDCG-x/p) gives, backward over the steps with Q = 0, P = 1:
// F_s = c_s Q, H_s = c_s P, then Q = a_s + b_s Q, P = b_s P; at the end
// E = Q, G = P.  One thread per (system, shift); coefficients of steps past
// cnt are zero (k_shift_blk multiplies them by zero residuals).
__global__ __launch_bounds__(TPB) void k_block_map(DevSolver ds) {
  const int nz = ds.nz;
  const int64_t e = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (e >= (int64_t)ds.nrhs * nz) return;
  const int rhs = (int)(e / nz), k = (int)(e - (int64_t)rhs * nz);
  const RhsState* S = ds.st + rhs;
  const int cnt = (S->blk_gen == ds.blk_gen) ? S->blk_cnt : 0;
  if (cnt <= 0 || !ds.btouch[e]) return;
  zc* c = ds.bcoef + (size_t)e * bcoef_len();
  zc Q = zmk(0.0, 0.0), P = zmk(1.0, 0.0);
  for (int s = XBLK_MAX - 1; s >= cnt; --s) {
    c[2 + s] = zmk(0.0, 0.0);
    c[2 + XBLK_MAX + s] = zmk(0.0, 0.0);
  }
#pragma unroll 4
  for (int s = cnt - 1; s >= 0; --s) {
    const zc a = ds.bstep[bstep_at(nz, rhs, s, 0, k)];
    const zc b = ds.bstep[bstep_at(nz, rhs, s, 1, k)];
    const zc cs = ds.bstep[bstep_at(nz, rhs, s, 2, k)];
    c[2 + s] = zmul(cs, Q);
    c[2 + XBLK_MAX + s] = zmul(cs, P);
    Q = zadd(a, zmul(b, Q));
    P = zmul(b, P);
  }
  c[0] = Q;
  c[1] = P;
}

// ---------------------------------------------------------- k_shift_blk
// Applies cnt composed steps of Eqs. EQ-SHIFTEDCG-x/p at once:
//   x^k <- x^k + E p^k + sum_t F_t r_t,   p^k <- G p^k + sum_t H_t r_t,
// r_t the seed residual memory vector of step t (ring slot (slot0+t) % nb).
// x^k, p^k are read and written once per block instead of once per step; the
// r_t of a row stay in registers while a work-group runs through its shifts.
// The 2 + 2T coefficients of a shift and the touched flags are the same for
// every lane: they are read through the constant address space, i.e. by
// scalar loads into SGPRs (a broadcast from LDS of 2 + 2T complex values per
// shift and wave costs LDS return bandwidth and vector registers).  Grid:
// (row tiles or work-list entries, shift splits, right-hand sides).
__device__ inline zc cfma(zc a, zc b, zc c) {  // c + a b
  return zmk(fma(a.x, b.x, fma(-a.y, b.y, c.x)), fma(a.x, b.y, fma(a.y, b.x, c.y)));
}
__device__ inline double cfma(zc a, double b, double c) { return fma(a.x, b, c); }

template <class V, class X, int T, bool NT>
__global__ __launch_bounds__(TPB) void k_shift_blk(DevSolver ds, const V* __restrict__ ring, int64_t vr, int slot0,
                                                   int nb, X* __restrict__ Xv, X* __restrict__ Pd) {
  typedef const __attribute__((address_space(4))) double* kd_ptr;
  typedef const __attribute__((address_space(4))) int32_t* ki_ptr;
  int rhs;
  int64_t M, off, i;
  if (ds.soff) {
    const int2 e = ds.wl_t[blockIdx.x];
    rhs = e.x;
    off = ds.soff[rhs];
    M = ds.soff[rhs + 1] - off;
    i = (int64_t)e.y * TPB + threadIdx.x;
  } else {
    rhs = blockIdx.z;
    M = ds.M;
    off = (int64_t)rhs * M;
    i = (int64_t)blockIdx.x * TPB + threadIdx.x;
  }
  rhs = __builtin_amdgcn_readfirstlane(rhs);
  const RhsState* S = ds.st + rhs;
  const int cnt = (S->blk_gen == ds.blk_gen) ? S->blk_cnt : 0;
  if (cnt <= 0 || i >= M) return;  // no barrier below
  const int nz = ds.nz;
  // this work-group's shifts: split blockIdx.y of gridDim.y
  const int per = (nz + (int)gridDim.y - 1) / (int)gridDim.y;
  const int kb = (int)blockIdx.y * per, ke = min(nz, kb + per);
  V r[T];
#pragma unroll
  for (int t = 0; t < T; ++t) {
    r[t] = VT<V>::zero();
    if (t < cnt) {
      int sl = slot0 + t;
      if (sl >= nb) sl -= nb;
      r[t] = ring[(size_t)sl * vr + off + i];
    }
  }
  const size_t sbase = (size_t)rhs * nz;
  for (int k0 = kb; k0 < ke; k0 += 32) {
    const int nk = min(32, ke - k0);
    const ki_ptr tf = (ki_ptr)(ds.btouch + sbase + k0);
    uint32_t todo = 0;  // bit sk set if shift k0+sk was touched by the block
    for (int e = 0; e < nk; ++e) todo |= (tf[e] ? 1u : 0u) << e;
    todo = __builtin_amdgcn_readfirstlane(todo);
    while (todo) {
      const int sk = __builtin_ctz(todo);
      todo &= todo - 1;
      const size_t o = xoff(ds, off, M, k0 + sk, i);
      const auto p0 = XS<X>::ld(Stream<X, NT>::ld(Pd + o));
      auto xa = XS<X>::ld(Stream<X, NT>::ld(Xv + o));
      // coefficient j of the shift: doubles 2j, 2j+1 (E, G, F_0.., H_0..)
      const kd_ptr c = (kd_ptr)(ds.bcoef + (sbase + k0 + sk) * bcoef_len());
      auto pa = VT<V>::zero();
      xa = cfma(zmk(c[0], c[1]), p0, xa);
      pa = cfma(zmk(c[2], c[3]), p0, pa);
#pragma unroll
      for (int t = 0; t < T; ++t) {
        xa = cfma(zmk(c[2 * (2 + t)], c[2 * (2 + t) + 1]), r[t], xa);
        pa = cfma(zmk(c[2 * (2 + XBLK_MAX + t)], c[2 * (2 + XBLK_MAX + t) + 1]), r[t], pa);
      }
      Stream<X, NT>::st(Xv + o, XS<X>::st(xa));
      Stream<X, NT>::st(Pd + o, XS<X>::st(pa));
    }
  }
}

// -------------------------------------------------------------- operators
// Row kernels return (H v)_i given v_i (already loaded) and the vector base.
// One periodic cube of the stencil operator: its edges, on-site energies and
// size (a batched operator holds one cube per system).
struct Cube {
  int32_t Lx, Ly, Lz;
  double hop;
  const double* eps;
  int64_t M;
};
__device__ inline Cube cube_of(const DevOp& op, int sys, int64_t off) {
  Cube c;
  c.hop = op.hop;
  if (op.nsys) {
    c.Lx = op.sysL[3 * sys];
    c.Ly = op.sysL[3 * sys + 1];
    c.Lz = op.sysL[3 * sys + 2];
    c.eps = op.eps + off;
    c.M = (int64_t)c.Lx * c.Ly * c.Lz;
  } else {
    c.Lx = op.Lx;
    c.Ly = op.Ly;
    c.Lz = op.Lz;
    c.eps = op.eps;
    c.M = op.M;
  }
  return c;
}

template <class V>
__device__ inline V stencil_row(const Cube& op, const V* __restrict__ v, int64_t i, V vi) {
  int64_t x, y, z;
  if (op.M < ((int64_t)1 << 31)) {
    const uint32_t ii = (uint32_t)i, lx = (uint32_t)op.Lx, ly = (uint32_t)op.Ly;
    const uint32_t yz = ii / lx;
    x = ii - yz * lx;
    y = yz % ly;
    z = yz / ly;
  } else {
    const int64_t yz = i / op.Lx;
    x = i - yz * op.Lx;
    y = yz % op.Ly;
    z = yz / op.Ly;
  }
  const int64_t Lx = op.Lx, Ly = op.Ly, Lz = op.Lz, LxLy = Lx * Ly;
  const int64_t xm = (x == 0) ? i + Lx - 1 : i - 1;
  const int64_t xp = (x == Lx - 1) ? i - (Lx - 1) : i + 1;
  const int64_t ym = (y == 0) ? i + LxLy - Lx : i - Lx;
  const int64_t yp = (y == Ly - 1) ? i - (LxLy - Lx) : i + Lx;
  const int64_t zm = (z == 0) ? i + (Lz - 1) * LxLy : i - LxLy;
  const int64_t zp = (z == Lz - 1) ? i - (Lz - 1) * LxLy : i + LxLy;
  // neighbour sum in the order -x, +x, -y, +y, -z, +z
  V nb = VT<V>::add(v[xm], v[xp]);
  nb = VT<V>::add(nb, v[ym]);
  nb = VT<V>::add(nb, v[yp]);
  nb = VT<V>::add(nb, v[zm]);
  nb = VT<V>::add(nb, v[zp]);
  const double e = op.eps[i];
  if constexpr (sizeof(V) == 16) {
    return zmk(e * vi.x - op.hop * nb.x, e * vi.y - op.hop * nb.y);
  } else {
    return e * vi - op.hop * nb;
  }
}

// Lane sums by DPP moves (vector ALU, no LDS traffic).  dpp_move reads the
// double of another lane of the same row of 16 lanes, chosen by CTRL.
template <int CTRL>
__device__ inline double dpp_move(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)(b & 0xffffffffll), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, true);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}
// Sum over each aligned group of N lanes (N = 1, 2, 4, 8): for 8, lanes i
// and 7 - i (half-row mirror), then i xor 2, then i xor 1 within a quad; for
// 4 the last two steps, for 2 the last.  Every lane of the group ends with the
// same value, summed in the same order.  All 64 lanes must be active.
template <int N>
__device__ inline double lane_sum(double v) {
  static_assert(N == 1 || N == 2 || N == 4 || N == 8, "1, 2, 4 or 8 lanes");
  if constexpr (N == 8) v += dpp_move<0x141>(v);  // row_half_mirror
  if constexpr (N >= 4) v += dpp_move<0x4E>(v);   // quad_perm [2, 3, 0, 1]
  if constexpr (N >= 2) v += dpp_move<0xB1>(v);   // quad_perm [1, 0, 3, 2]
  return v;
}

// CSR row product for CSR_LPR lanes per row: lane j of the row (j = lane mod
// CSR_LPR) takes the row's entries j, j + CSR_LPR, ... and the partial sums
// are combined by lane_sum, so the column and value reads of a wave are
// contiguous.  Rows at or beyond M contribute zero but their lanes still take
// part in the sum.  On the 64^3 stencil as CSR (7 entries per row), per
// product: one right-hand side 18.9 us with 8 or 4 lanes, 20.7 us with 2;
// BiCG's two vectors (4 right-hand sides) 70.5 / 58 / 61 us with 8 / 4 / 2.
constexpr int CSR_LPR = 4;
template <class V, bool VALC>
__device__ inline V csr_row_lanes(const DevOp& op, const V* __restrict__ v, int64_t i, bool live, int sub) {
  V acc = VT<V>::zero();
  if (live) {
    const int64_t p0 = op.rowptr[i], p1 = op.rowptr[i + 1];
    for (int64_t p = p0 + sub; p < p1; p += CSR_LPR) {
      const V vj = v[op.col[p]];
      if constexpr (VALC) {
        const zc a = reinterpret_cast<const zc*>(op.val)[p];
        if constexpr (sizeof(V) == 16) acc = zadd(acc, zmul(a, vj));
        else acc = acc + a.x * vj;
      } else {
        const double a = reinterpret_cast<const double*>(op.val)[p];
        if constexpr (sizeof(V) == 16) acc = zadd(acc, zscale(a, vj));
        else acc = acc + a * vj;
      }
    }
  }
  if constexpr (sizeof(V) == 16) return zmk(lane_sum<CSR_LPR>(acc.x), lane_sum<CSR_LPR>(acc.y));
  else return lane_sum<CSR_LPR>(acc);
}

// Heisenberg: (H v)_s = [sum_b (J_b/4)(+1 parallel, -1 antiparallel)] v_s
//                      + sum_{b antiparallel} (J_b/2) v_{idx(s xor m_b)}
// with idx(t) = hi_off[t >> h] + lo_rank[t & (2^h - 1)].  Rewritten as
//     (H v)_s = (sum_b J_b / 4) v_s + sum_b (J_b/2) (g_b - v_s),
// g_b = v_{idx(s xor m_b)} for an antiparallel bond and g_b = v_s otherwise,
// so a parallel bond adds an exact zero and no per-bond weight or diagonal
// term is carried.  Bonds come in three lists by where their sites fall
// relative to the index split (low: both below h, high: both at or above h,
// cross: one each side).  A low bond keeps the high part u = s >> h, so its
// partner is hi_off[u] + lo_rank[l xor m] with hi_off[u] looked up once per
// row; a high bond keeps the low part l and reads hi_off[u xor m] +
// lo_rank[l]; only a cross bond needs both lookups.  Each list is taken in
// chunks whose target indices are formed first and whose gathers then issue
// together (predicated on antiparallel), so a row has a chunk's loads in
// flight at once.  The lists are LDS copies padded with null bonds (mask 0,
// coupling 0) to whole chunks; the index tables are LDS copies or global,
// fixed per instantiation so that every lookup compiles to a plain LDS or
// global access.

// The three padded lists in LDS: masks (u32) then halved couplings (f64) per list.
// Bond lists in the constant address space: their entries are the same for
// every lane, so the compiler reads them with scalar loads into SGPRs.
typedef const __attribute__((address_space(4))) uint32_t* kmask_ptr;
typedef const __attribute__((address_space(4))) double* kcoef_ptr;
struct HeisLists {
  kmask_ptr lm; kcoef_ptr lj; int nl;   // low: masks within the low h bits
  kmask_ptr hm; kcoef_ptr hj; int nh;   // high: masks within the high bits
  kmask_ptr cm; kcoef_ptr cj; int nc;   // cross: full state masks
};

template <int KIND, int CH, class V>
__device__ inline V heis_chunks(kmask_ptr bm, kcoef_ptr bj, int n, const V* __restrict__ v, uint32_t s,
                                int h, uint32_t hs, uint32_t ls, V vi, V nvi, const uint32_t* hi,
                                const uint16_t* lo, V acc) {
  const uint32_t lmask = (1u << h) - 1u, u = s >> h, l = s & lmask;
  for (int b0 = 0; b0 < n; b0 += CH) {
    uint32_t jj[CH];
    uint32_t anti = 0;
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const uint32_t m = bm[b0 + c];
      if (KIND == 0) {          // low bond: flips bits of l only
        anti |= (uint32_t)(__popc(l & m) == 1) << c;
        jj[c] = hs + (uint32_t)lo[l ^ m];
      } else if (KIND == 1) {   // high bond: flips bits of u only
        anti |= (uint32_t)(__popc(u & m) == 1) << c;
        jj[c] = hi[u ^ m] + ls;
      } else {                  // cross bond
        const uint32_t t = s ^ m;
        anti |= (uint32_t)(__popc(s & m) == 1) << c;
        jj[c] = hi[t >> h] + (uint32_t)lo[t & lmask];
      }
    }
    V g[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      g[c] = vi;
      if ((anti >> c) & 1u) g[c] = v[jj[c]];
    }
#pragma unroll
    for (int c = 0; c < CH; ++c) acc = VT<V>::add(acc, VT<V>::rs(bj[b0 + c], VT<V>::add(g[c], nvi)));
  }
  return acc;
}

template <class V>
__device__ inline V heis_row(const HeisLists& B, int h, double jq, const V* __restrict__ v, uint32_t s, V vi,
                             const uint32_t* hi, const uint16_t* lo) {
  const uint32_t hs = hi[s >> h], ls = lo[s & ((1u << h) - 1u)];
  const V nvi = VT<V>::rs(-1.0, vi);
  V acc = VT<V>::zero();
  acc = heis_chunks<0, HEIS_CH_LO>(B.lm, B.lj, B.nl, v, s, h, hs, ls, vi, nvi, hi, lo, acc);
  acc = heis_chunks<1, HEIS_CH_HI>(B.hm, B.hj, B.nh, v, s, h, hs, ls, vi, nvi, hi, lo, acc);
  acc = heis_chunks<2, HEIS_CH_CR>(B.cm, B.cj, B.nc, v, s, h, hs, ls, vi, nvi, hi, lo, acc);
  return VT<V>::add(VT<V>::rs(jq, vi), acc);
}

// ---------------------------------------- Heisenberg, one group at a time
// The basis is ordered by the high part u = s >> h; the rows of one u (a
// "group") are contiguous and ordered by the rank j of the low part l among
// h-bit values of equal popcount, so l = lo_state[koff[k] + j] with
// k = nup - popc(u).  Work-group b takes the rows [b M / G, (b+1) M / G) and
// walks the groups that overlap them.  For each group it stages the group's
// whole r segment in LDS (a group split between two work-groups is staged by
// both) together with the group's bond constants, and then, per row:
//  - low bonds (both sites below h) flip l only: the partner is in the same
//    group at rank lo_rank[l ^ m], read from LDS;
//  - high bonds flip u only: whether the pair is antiparallel depends on u
//    alone, and the partner of rank j is rank j of group u ^ m, a contiguous
//    read shared by the whole wave;
//  - cross bonds (one site each side) read rank lo_rank[l ^ bit] of group
//    u ^ bit': the only scattered global reads.
// Every bond list sits in LDS padded with null bonds to a multiple of the
// chunk, so each chunk is straight-line code whose reads issue together.
constexpr int LDS_ALIGN = 16;
constexpr int GRP_CH = 8;  // bonds per chunk in the group kernel
__host__ __device__ inline size_t heis_grp_table_bytes(int h) {
  return (((size_t)4 << h) + LDS_ALIGN - 1) / LDS_ALIGN * LDS_ALIGN;  // lo_rank + lo_state (uint16 each)
}
__host__ __device__ inline int grp_pad(int n) { return (n + GRP_CH - 1) / GRP_CH * GRP_CH; }
// per-bond LDS: low (mask 4 + J 8), high (partner offset 4 + weight 8 + diagonal share 8),
// cross (low bit 4 + high-side bit value 4 + partner offset 4 + J 8)
__host__ __device__ inline size_t heis_grp_bond_bytes(const DevOp& op) {
  return (size_t)grp_pad(op.nlo) * 12 + (size_t)grp_pad(op.nhb) * 20 + (size_t)grp_pad(op.ncr) * 20 + 64;
}

template <class V, int DK, bool SH, bool DOT>
__global__ __launch_bounds__(TPB) void k_spmv_heis_grp(DevSolver ds, DevOp op, Buffers bf, int nblkB) {
  extern __shared__ unsigned char smem[];
  const int rhs = blockIdx.y;
  int g0 = blockIdx.x, ngb = gridDim.x;
  if (DOT) {
    if (g0 == 0) {
      finaliser_group(ds, rhs, nblkB);
      return;
    }
    g0 -= 1;
    ngb -= 1;
    if (ds.st[rhs].stop) return;
  }
  const int64_t M = op.M;
  const V* __restrict__ R = reinterpret_cast<const V*>(bf.R) + (size_t)rhs * M;
  V* __restrict__ Q = reinterpret_cast<V*>(bf.Q) + (size_t)rhs * M;
  const V* Rs = SH ? reinterpret_cast<const V*>(bf.Rs) + (size_t)rhs * M : nullptr;
  V* Qs = SH ? reinterpret_cast<V*>(bf.Qs) + (size_t)rhs * M : nullptr;
  const int h = op.h;
  const int nt = 1 << h;
  const int nlo = grp_pad(op.nlo), nhb = grp_pad(op.nhb), ncr = grp_pad(op.ncr);
  // LDS carve-up: tables | bond constants | segment(s)
  uint16_t* slo = reinterpret_cast<uint16_t*>(smem);  // lo_rank
  uint16_t* sst = slo + nt;                             // lo_state
  unsigned char* pb = smem + heis_grp_table_bytes(h);
  double* lJ = reinterpret_cast<double*>(pb);            // low: coupling
  double* hw = lJ + nlo;                                 // high: weight J/2 (0 if parallel)
  double* hd = hw + nhb;                                 // high: +-J/4
  double* cJ = hd + nhb;                                 // cross: coupling
  uint32_t* lm = reinterpret_cast<uint32_t*>(cJ + ncr);  // low: mask
  uint32_t* hb = lm + nlo;                               // high: partner group offset
  uint32_t* ca = hb + nhb;                               // cross: low-side bit
  uint32_t* cu = ca + ncr;                               // cross: high-side bit value of u
  uint32_t* cb = cu + ncr;                               // cross: partner group offset
  V* seg = reinterpret_cast<V*>(pb + (heis_grp_bond_bytes(op) + LDS_ALIGN - 1) / LDS_ALIGN * LDS_ALIGN);
  V* segs = SH ? seg + op.segmax : nullptr;
  for (int e = threadIdx.x; e < nt; e += TPB) {
    slo[e] = op.lo_rank[e];
    sst[e] = op.lo_state[e];
  }
  for (int b = threadIdx.x; b < nlo; b += TPB) {
    lm[b] = b < op.nlo ? op.lo_m[b] : 0u;
    lJ[b] = b < op.nlo ? op.lo_J[b] : 0.0;
  }
  for (int b = threadIdx.x; b < ncr; b += TPB) {
    ca[b] = b < op.ncr ? (uint32_t)op.cr_a[b] : 0u;
    cJ[b] = b < op.ncr ? op.cr_J[b] : 0.0;
  }
  // this work-group's rows and the group holding the first of them
  const int64_t r0 = M * g0 / ngb, r1 = M * (g0 + 1) / ngb;
  int ulo = 0, uhi = op.ngroups;  // hi_off[ngroups] = M > r0
  while (uhi - ulo > 1) {
    const int mid = (ulo + uhi) >> 1;
    if ((int64_t)op.hi_off[mid] <= r0) ulo = mid;
    else uhi = mid;
  }
  zc t = zmk(0.0, 0.0);
  for (int uu = ulo; uu < op.ngroups; ++uu) {
    const uint32_t u = (uint32_t)uu;
    const int64_t gs = op.hi_off[u], ge = op.hi_off[u + 1];
    if (gs >= r1) break;
    const int size = (int)(ge - gs);
    if (size == 0) continue;
    __syncthreads();  // the previous group's segment and constants have been consumed
    for (int j = threadIdx.x; j < size; j += TPB) {
      seg[j] = R[gs + j];
      if (SH) segs[j] = Rs[gs + j];
    }
    for (int b = threadIdx.x; b < nhb; b += TPB) {
      const bool real = b < op.nhb;
      const uint32_t m = real ? op.hb_m[b] : 0u;
      const double J = real ? op.hb_J[b] : 0.0;
      const bool anti = __popc(u & m) == 1;
      hb[b] = anti ? op.hi_off[u ^ m] : 0u;
      hw[b] = anti ? 0.5 * J : 0.0;
      hd[b] = anti ? -0.25 * J : 0.25 * J;
    }
    for (int b = threadIdx.x; b < ncr; b += TPB) {
      const bool real = b < op.ncr;
      const int c = real ? op.cr_c[b] : 0;
      cu[b] = real ? ((u >> c) & 1u) : 0u;
      cb[b] = real ? op.hi_off[u ^ (1u << c)] : 0u;
    }
    __syncthreads();
    const uint32_t koff = op.lo_koff[op.nup - __popc(u)];
    double dhi = 0.0;  // the high bonds' share of the diagonal, the same for the whole group
    for (int b = 0; b < nhb; ++b) dhi += hd[b];
    const int j0 = (int)((r0 > gs ? r0 : gs) - gs), j1 = (int)((r1 < ge ? r1 : ge) - gs);
    for (int j = j0 + (int)threadIdx.x; j < j1; j += TPB) {
      const uint32_t l = sst[koff + j];
      V acc = VT<V>::zero(), accs = VT<V>::zero();
      double diag = dhi;
      // high bonds: rank j of the partner group (weight 0: parallel, no read)
      for (int b0 = 0; b0 < nhb; b0 += GRP_CH) {
        V g[GRP_CH], gh[GRP_CH];
        double w[GRP_CH];
#pragma unroll
        for (int c = 0; c < GRP_CH; ++c) {
          w[c] = hw[b0 + c];
          g[c] = VT<V>::zero();
          gh[c] = VT<V>::zero();
          if (w[c] != 0.0) {
            const int64_t p = (int64_t)hb[b0 + c] + j;
            g[c] = R[p];
            if (SH) gh[c] = Rs[p];
          }
        }
#pragma unroll
        for (int c = 0; c < GRP_CH; ++c) {
          acc = VT<V>::add(acc, VT<V>::rs(w[c], g[c]));
          if (SH) accs = VT<V>::add(accs, VT<V>::rs(w[c], gh[c]));
        }
      }
      // cross bonds: scattered rows of the neighbouring group
      for (int b0 = 0; b0 < ncr; b0 += GRP_CH) {
        V g[GRP_CH], gh[GRP_CH];
        double w[GRP_CH];
#pragma unroll
        for (int c = 0; c < GRP_CH; ++c) {
          const uint32_t a = ca[b0 + c];
          const double J = cJ[b0 + c];
          const bool anti = ((l >> a) & 1u) != cu[b0 + c];
          const int64_t p = (int64_t)cb[b0 + c] + slo[l ^ (1u << a)];
          w[c] = anti ? 0.5 * J : 0.0;
          diag += anti ? -0.25 * J : 0.25 * J;
          g[c] = VT<V>::zero();
          gh[c] = VT<V>::zero();
          if (w[c] != 0.0) {
            g[c] = R[p];
            if (SH) gh[c] = Rs[p];
          }
        }
#pragma unroll
        for (int c = 0; c < GRP_CH; ++c) {
          acc = VT<V>::add(acc, VT<V>::rs(w[c], g[c]));
          if (SH) accs = VT<V>::add(accs, VT<V>::rs(w[c], gh[c]));
        }
      }
      // low bonds: partner in the same group, from LDS
      for (int b0 = 0; b0 < nlo; b0 += GRP_CH) {
#pragma unroll
        for (int c = 0; c < GRP_CH; ++c) {
          const uint32_t m = lm[b0 + c];
          const double J = lJ[b0 + c];
          const bool anti = __popc(l & m) == 1;
          // a parallel bond's l ^ m lies in another popcount class, whose
          // rank may fall outside this segment: read the row itself instead
          const int p = anti ? (int)slo[l ^ m] : j;
          const double wc = anti ? 0.5 * J : 0.0;
          diag += anti ? -0.25 * J : 0.25 * J;
          acc = VT<V>::add(acc, VT<V>::rs(wc, seg[p]));
          if (SH) accs = VT<V>::add(accs, VT<V>::rs(wc, segs[p]));
        }
      }
      const V ri = seg[j];
      const V q = VT<V>::add(VT<V>::rs(diag, ri), acc);
      Q[gs + j] = q;
      if (SH) {
        const V rsi = segs[j];
        Qs[gs + j] = VT<V>::add(VT<V>::rs(diag, rsi), accs);
        if (DOT) t = zadd(t, VT<V>::ses(rsi, q));
      } else if (DOT) {
        t = zadd(t, mdot<V, DK>(ri, q));
      }
    }
  }
  if (DOT) {
    double v[2] = {t.x, t.y};
    block_sum<2>(v);
    if (threadIdx.x == 0) {
      double* slot = slotsA(ds, rhs) + (size_t)g0 * SLOT_A;
      slot[0] = v[0];
      slot[1] = v[1];
    }
  }
}

size_t heis_grp_lds_bytes(const DevOp& op, bool shadow) {
  return heis_grp_table_bytes(op.h) + (heis_grp_bond_bytes(op) + LDS_ALIGN - 1) / LDS_ALIGN * LDS_ALIGN +
         (size_t)op.segmax * 16 * (shadow ? 2 : 1);
}

// LDS of the Heisenberg row product: the two index tables (TLDS), or none.
__host__ __device__ inline size_t heis_row_lds_bytes(const DevOp& op, bool tlds) {
  return tlds ? 4 * ((size_t)1 << (op.L - op.h)) + 2 * ((size_t)1 << op.h) : 0;
}


// q = H r (and qs = H rs for BiCG).  With DOT (the solver loop) one group
// per system is the finaliser of the previous step and the others each write
// the partial inner product feeding alpha_n into their slot.  OPK selects
// the operator; VALC is its variant flag: complex values (CSR) or index
// tables staged in LDS (Heisenberg).  In the batched layout a stencil
// operator supplies one cube per system and a CSR operator acts on the whole
// concatenated vector (block diagonal).
template <class V, int DK, bool SH, bool DOT, int OPK, bool VALC>
__global__ __launch_bounds__(TPB) void k_spmv(DevSolver ds, DevOp op, Buffers bf, int nblkB) {
  extern __shared__ unsigned char smem[];
  constexpr bool BATCH = OPK != OP_HEIS;
  const Blk bk = blk_of<DOT ? 1 : 0, BATCH>(ds, ds.wl_a);
  const int rhs = bk.rhs;
  const int g = bk.g, ngroups = bk.ng;
  if (DOT) {
    if (g < 0) {
      finaliser_group(ds, rhs, nblkB);
      return;
    }
    // one value per wave (stop may be set during the launch; see k_spmv_csr_mr)
    if (__builtin_amdgcn_readfirstlane(ds.st[rhs].stop)) return;
  }
  const int64_t M = bk.M;
  const V* __restrict__ R = reinterpret_cast<const V*>(bf.R) + bk.off;
  V* __restrict__ Q = reinterpret_cast<V*>(bf.Q) + bk.off;
  const V* Rs = SH ? reinterpret_cast<const V*>(bf.Rs) + bk.off : nullptr;
  V* Qs = SH ? reinterpret_cast<V*>(bf.Qs) + bk.off : nullptr;
  // CSR rows are global in the batched layout
  const int64_t crow = (BATCH && ds.soff) ? bk.off : 0;
  const V* Rc = R - crow;
  const V* Rsc = SH ? Rs - crow : nullptr;
  Cube cube;
  if constexpr (OPK == OP_STENCIL) cube = cube_of(op, rhs, bk.off);

  HeisLists bl;
  uint32_t* shi = nullptr;
  uint16_t* slo = nullptr;
  if constexpr (OPK == OP_HEIS) {
    const int h = op.h;
    (void)h;
    bl.nl = heis_pad(op.nlo, HEIS_CH_LO);
    bl.nh = heis_pad(op.nhb, HEIS_CH_HI);
    bl.nc = heis_pad(op.ncr, HEIS_CH_CR);
    bl.lm = (kmask_ptr)op.rl_m;
    bl.lj = (kcoef_ptr)op.rl_j;
    bl.hm = bl.lm + bl.nl;
    bl.hj = bl.lj + bl.nl;
    bl.cm = bl.hm + bl.nh;
    bl.cj = bl.hj + bl.nh;
    unsigned char* p = smem;
    if constexpr (VALC) {
      const int nhi = 1 << (op.L - op.h), nlo = 1 << op.h;
      shi = reinterpret_cast<uint32_t*>(p);
      slo = reinterpret_cast<uint16_t*>(shi + nhi);
      for (int e = threadIdx.x; e < nhi; e += TPB) shi[e] = op.hi_off[e];
      for (int e = threadIdx.x; e < nlo; e += TPB) slo[e] = op.lo_rank[e];
    }
    __syncthreads();
  }

  int64_t tile0 = g, tstride = ngroups, tend = (M + TPB - 1) / TPB;
  if (ngroups >= 8 * XCD_COUNT) {
    // XCD-aware order for the operator products: work-groups
    // g and g + XCD_COUNT run on one XCD (round-robin dispatch of consecutive
    // work-groups); XCD x takes the x-th slice of the tiles and its
    // work-groups stride through that slice together, so the partners of
    // nearby rows (Heisenberg gathers, the stencil's neighbouring planes,
    // the columns of a banded CSR matrix) are read through one L2.  Every tile is still processed exactly once (any
    // XCD count).
    const int x = g % XCD_COUNT, k = g / XCD_COUNT;
    const int ngx = (ngroups - x + XCD_COUNT - 1) / XCD_COUNT;
    const int64_t t0 = tend * x / XCD_COUNT, t1 = tend * (x + 1) / XCD_COUNT;
    tile0 = t0 + k;
    tstride = ngx;
    tend = t1;
  }
  zc t = zmk(0.0, 0.0);
  if constexpr (OPK == OP_CSR) {
    // a tile of TPB rows in CSR_LPR passes of TPB / CSR_LPR rows
    const int sub = threadIdx.x & (CSR_LPR - 1);
    for (int64_t tile = tile0; tile < tend; tile += tstride) {
#pragma unroll 1
      for (int pass = 0; pass < CSR_LPR; ++pass) {
        const int64_t i = tile * TPB + pass * (TPB / CSR_LPR) + threadIdx.x / CSR_LPR;
        const bool live = i < M;
        const V q = csr_row_lanes<V, VALC>(op, Rc, i + crow, live, sub);
        V qs;
        if (SH) qs = csr_row_lanes<V, VALC>(op, Rsc, i + crow, live, sub);
        if (sub == 0 && live) {
          Q[i] = q;
          if (SH) Qs[i] = qs;
          if (DOT) {
            const zc d = SH ? VT<V>::ses(Rs[i], q) : mdot<V, DK>(R[i], q);
            t = zadd(t, d);
          }
        }
      }
    }
  } else
  for (int64_t slot = tile0; slot < tend; slot += tstride) {
    // Heisenberg: the operator's tile order (a permutation, read by a scalar
    // load), so the ragged last tile can come at any slot
    const int64_t tile = OPK == OP_HEIS ? (int64_t)((kmask_ptr)op.tile_order)[slot] : slot;
    const int64_t i = tile * TPB + threadIdx.x;
    if (i >= M) continue;
    const V ri = R[i];
    V q, qs;
    if constexpr (OPK == OP_STENCIL) {
      q = stencil_row<V>(cube, R, i, ri);
      if (SH) qs = stencil_row<V>(cube, Rs, i, Rs[i]);
    } else {
      const uint32_t s = op.states[i];
      if constexpr (VALC) {
        q = heis_row<V>(bl, op.h, op.jq, R, s, ri, shi, slo);
        if (SH) qs = heis_row<V>(bl, op.h, op.jq, Rs, s, Rs[i], shi, slo);
      } else {
        q = heis_row<V>(bl, op.h, op.jq, R, s, ri, op.hi_off, op.lo_rank);
        if (SH) qs = heis_row<V>(bl, op.h, op.jq, Rs, s, Rs[i], op.hi_off, op.lo_rank);
      }
    }
    Q[i] = q;
    if (SH) Qs[i] = qs;
    if (DOT) {
      const zc d = SH ? VT<V>::ses(Rs[i], q) : mdot<V, DK>(ri, q);
      t = zadd(t, d);
    }
  }
  if (DOT) {
    double v[2] = {t.x, t.y};
    block_sum<2>(v);
    if (threadIdx.x == 0) {
      double* slot = slotsA(ds, rhs) + (size_t)g * SLOT_A;
      slot[0] = v[0];
      slot[1] = v[1];
    }
  }
}

// CSR product for several right-hand sides of one matrix (uniform layout, no
// shadow system), with the grid and slots of k_spmv: grid (ng + 1, nrhs),
// group 0 of row r finalises system r's previous step.  The ng product groups
// of every row form one pool of G = nrhs ng groups; group gg = r ng + g takes
// tiles gg, gg + G, ... for every live right-hand side, 8 at a time, so the
// matrix is read once per 8 right-hand sides instead of once per right-hand
// side, and writes the partial inner product of each into its slot gg
// (G slots per system, as k_seed expects).  Rows: CSR_MR_LPR lanes per row,
// lane j taking the row's entries j, j + CSR_MR_LPR, ... (on the 64^3
// stencil as CSR, 7 entries per row, 16 right-hand sides: 8 lanes 123 us,
// 4 lanes 94 us, 2 lanes 79 us, 1 lane 101 us per product).
constexpr int CSR_MR_B = 8;
constexpr int CSR_MR_LPR = 2;
template <class V, int DK, bool VALC>
__global__ __launch_bounds__(TPB) void k_spmv_csr_mr(DevSolver ds, DevOp op, Buffers bf, int nblkB) {
  const int row = blockIdx.y;
  const int g = (int)blockIdx.x - 1, ng = (int)gridDim.x - 1;
  if (g < 0) {
    finaliser_group(ds, row, nblkB);
    return;
  }
  const int nr = ds.nrhs;
  const int64_t M = ds.M;
  const int64_t gg = (int64_t)row * ng + g, G = (int64_t)nr * ng;
  const int64_t ntile = (M + TPB - 1) / TPB;
  const int sub = threadIdx.x & (CSR_MR_LPR - 1);
  const V* __restrict__ R = reinterpret_cast<const V*>(bf.R);
  V* __restrict__ Q = reinterpret_cast<V*>(bf.Q);
  for (int r0 = 0; r0 < nr; r0 += CSR_MR_B) {
    bool on[CSR_MR_B];
    zc t[CSR_MR_B];
#pragma unroll
    for (int j = 0; j < CSR_MR_B; ++j) {
      // the finaliser groups may set stop during this launch: every lane of
      // a wave takes one value (the lane sums below need whole waves); a
      // system that stops meanwhile has its product discarded either way
      on[j] = r0 + j < nr && !__builtin_amdgcn_readfirstlane(ds.st[r0 + j].stop);
      t[j] = zmk(0.0, 0.0);
    }
    for (int64_t tile = gg; tile < ntile; tile += G) {
#pragma unroll 1
      for (int pass = 0; pass < CSR_MR_LPR; ++pass) {
        const int64_t i = tile * TPB + pass * (TPB / CSR_MR_LPR) + threadIdx.x / CSR_MR_LPR;
        const bool live = i < M;
        V acc[CSR_MR_B];
#pragma unroll
        for (int j = 0; j < CSR_MR_B; ++j) acc[j] = VT<V>::zero();
        if (live) {
          const int64_t p0 = op.rowptr[i], p1 = op.rowptr[i + 1];
          for (int64_t p = p0 + sub; p < p1; p += CSR_MR_LPR) {
            const int64_t c = op.col[p];
            V vj[CSR_MR_B];
#pragma unroll
            for (int j = 0; j < CSR_MR_B; ++j)
              if (on[j]) vj[j] = R[(int64_t)(r0 + j) * M + c];
            if constexpr (VALC) {
              const zc a = reinterpret_cast<const zc*>(op.val)[p];
#pragma unroll
              for (int j = 0; j < CSR_MR_B; ++j) {
                if (!on[j]) continue;
                if constexpr (sizeof(V) == 16) acc[j] = zadd(acc[j], zmul(a, vj[j]));
                else acc[j] = acc[j] + a.x * vj[j];
              }
            } else {
              const double a = reinterpret_cast<const double*>(op.val)[p];
#pragma unroll
              for (int j = 0; j < CSR_MR_B; ++j) {
                if (!on[j]) continue;
                if constexpr (sizeof(V) == 16) acc[j] = zadd(acc[j], zscale(a, vj[j]));
                else acc[j] = acc[j] + a * vj[j];
              }
            }
          }
        }
#pragma unroll
        for (int j = 0; j < CSR_MR_B; ++j) {
          if (!on[j]) continue;  // the same for every lane of the group
          V q;
          if constexpr (sizeof(V) == 16) q = zmk(lane_sum<CSR_MR_LPR>(acc[j].x), lane_sum<CSR_MR_LPR>(acc[j].y));
          else q = lane_sum<CSR_MR_LPR>(acc[j]);
          if (sub == 0 && live) {
            const int64_t o = (int64_t)(r0 + j) * M + i;
            Q[o] = q;
            t[j] = zadd(t[j], mdot<V, DK>(R[o], q));
          }
        }
      }
    }
#pragma unroll
    for (int j = 0; j < CSR_MR_B; ++j) {
      if (r0 + j >= nr) break;
      double v[2] = {t[j].x, t[j].y};
      block_sum<2>(v);
      if (threadIdx.x == 0 && on[j]) {
        double* slot = slotsA(ds, r0 + j) + (size_t)gg * SLOT_A;
        slot[0] = v[0];
        slot[1] = v[1];
      }
    }
  }
}

// Reverse-communication path: t = dual . q for caller-supplied q, with the
// same finaliser group 0 and slot layout as k_spmv.
template <class V, int DK>
__global__ __launch_bounds__(TPB) void k_dot(DevSolver ds, const V* __restrict__ dual,
                                             const V* __restrict__ q, int nblkB) {
  const Blk bk = blk_of<1>(ds, ds.wl_a);
  const int rhs = bk.rhs;
  if (bk.g < 0) {
    finaliser_group(ds, rhs, nblkB);
    return;
  }
  if (ds.st[rhs].stop) return;
  const int g = bk.g, ngroups = bk.ng;
  const int64_t M = bk.M;
  const V* d = dual + bk.off;
  const V* qq = q + bk.off;
  zc t = zmk(0.0, 0.0);
  const int64_t stride = (int64_t)ngroups * TPB;
  for (int64_t i = (int64_t)g * TPB + threadIdx.x; i < M; i += stride)
    t = zadd(t, mdot<V, DK>(d[i], qq[i]));
  double v[2] = {t.x, t.y};
  block_sum<2>(v);
  if (threadIdx.x == 0) {
    double* slot = slotsA(ds, rhs) + (size_t)g * SLOT_A;
    slot[0] = v[0];
    slot[1] = v[1];
  }
}

// ------------------------------------------------- Heisenberg set-up
// Basis state of rank i among L-bit integers with nup set bits, ascending:
// ascending order is the colex order of the bit-position sets, whose rank is
// sum_j C(c_j, j) over the positions c_1 < c_2 < ... (combinatorial number
// system).  Unranked greedily from the top position.
__global__ void k_heis_basis(uint32_t* states, int64_t M, int L, int nup, const int64_t* binom) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  int64_t rank = i;
  uint32_t s = 0;
  int c = L - 1;
  for (int j = nup; j >= 1; --j) {
    while (binom[c * 33 + j] > rank) --c;
    s |= 1u << c;
    rank -= binom[c * 33 + j];
    --c;
  }
  states[i] = s;
}

// lo_rank[l] = colex rank of l among h-bit integers of equal popcount.
__global__ void k_heis_lo(uint16_t* lo, int h, const int64_t* binom) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= (1 << h)) return;
  int64_t r = 0;
  int j = 0;
  for (int c = 0; c < h; ++c)
    if ((l >> c) & 1) { ++j; r += binom[c * 33 + j]; }
  lo[l] = (uint16_t)r;
}

// hi_off[u] = number of basis states whose high part is < u: exclusive scan
// of C(h, nup - popcount(u)) over u, by one work-group of 1024 threads.
__global__ __launch_bounds__(1024) void k_heis_hi(uint32_t* hi, int nhi, int h, int nup,
                                                  const int64_t* binom, int64_t* total) {
  __shared__ int64_t sh[1024];
  const int t = threadIdx.x;
  const int per = (nhi + 1023) / 1024;
  const int u0 = t * per;
  int64_t sum = 0;
  for (int u = u0; u < u0 + per && u < nhi; ++u) {
    const int need = nup - __popc((unsigned)u);
    sum += (need >= 0 && need <= h) ? binom[h * 33 + need] : 0;
  }
  sh[t] = sum;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    int64_t v = (t >= off) ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += v;
    __syncthreads();
  }
  int64_t run = sh[t] - sum;  // exclusive prefix of this chunk
  for (int u = u0; u < u0 + per && u < nhi; ++u) {
    hi[u] = (uint32_t)run;
    const int need = nup - __popc((unsigned)u);
    run += (need >= 0 && need <= h) ? binom[h * 33 + need] : 0;
  }
  if (t == 1023) {
    *total = sh[1023];
    hi[nhi] = (uint32_t)sh[1023];
  }
}

// Checks that idx(states[i]) == i for every i (two-table consistency).
__global__ void k_heis_check(DevOp op, int32_t* bad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= op.M) return;
  const uint32_t s = op.states[i];
  const uint32_t j = op.hi_off[s >> op.h] + (uint32_t)op.lo_rank[s & ((1u << op.h) - 1u)];
  if ((int64_t)j != i) atomicOr(bad, 1);
}

__global__ void k_heis_lookup(DevOp op, const uint32_t* st, int64_t* idx, int64_t n, int32_t* bad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t s = st[i];
  const bool fits = (op.L == 32) || (s >> op.L) == 0;
  if (!fits || __popc(s) != op.nup) {
    idx[i] = -1;
    atomicOr(bad, 1);
    return;
  }
  idx[i] = (int64_t)op.hi_off[s >> op.h] + (int64_t)op.lo_rank[s & ((1u << op.h) - 1u)];
}

struct Phases { zc w[32]; };

__global__ void k_heis_szq(DevOp op, Phases ph, const zc* v, zc* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= op.M) return;
  const uint32_t s = op.states[i];
  zc c = zmk(0.0, 0.0);
  for (int j = 0; j < op.L; ++j) {
    const double sz = ((s >> j) & 1u) ? 0.5 : -0.5;
    c = zadd(c, zscale(sz, ph.w[j]));
  }
  out[i] = zmul(c, v[i]);
}

// -------------------------------------------------------------- recalc
// Projected solution at new shifts from the recorded seed history, without
// operator products (Sec. 3.2.2 iv): the pi recurrence (Eq. EQ-SHIFTEDCG-PI)
// with the recorded alpha_n, beta_n and seed shift of every step, the y/u
// updates (Eqs. EQ-SHIFTEDCG-y/u) with the recorded P r_{n+1}, and the
// recorded switch factors (c0, c1), which rescale pi exactly as the solve
// did.  The freeze rule of the solve is applied.  One thread per new shift.
__global__ void k_recalc(DevSolver ds, int rhs, int nsteps, const zc* __restrict__ znew, int nzn, zc* y,
                         double* res) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nzn) return;
  const int nl = ds.nl;
  const size_t h0 = (size_t)rhs * ds.hist_cap;
  const double bnorm = ds.st[rhs].bnorm;
  zc u[KOMEGA_MAX_NL], yy[KOMEGA_MAX_NL];
#pragma unroll
  for (int l = 0; l < KOMEGA_MAX_NL; ++l) {
    u[l] = l < nl ? ds.pb[(size_t)rhs * nl + l] : zmk(0.0, 0.0);
    yy[l] = zmk(0.0, 0.0);
  }
  zc pi = zmk(1.0, 0.0), pio = zmk(1.0, 0.0), ba = zmk(0.0, 0.0);
  const zc zk = znew[k];
  double r = bnorm > 0.0 ? 1.0 : 0.0;
  bool active = true;
  for (int it = 0; it < nsteps && active; ++it) {
    const size_t h = h0 + it;
    const zc alpha = ds.h_alpha[h], beta = ds.h_beta[h], zs = ds.h_zs[h];
    const zc c0 = ds.h_sw[2 * h], c1 = ds.h_sw[2 * h + 1];
    const zc gamma = zmul(alpha, ba);
    const zc pn = zsub(zmul(zadd(zadd(zmk(1.0, 0.0), gamma), zmul(alpha, zsub(zk, zs))), pi), zmul(gamma, pio));
    if (!zfinite(pn) || zzero(pn)) { r = NAN; break; }
    const zc ratio = zdiv(pi, pn);
    const zc a_k = zmul(ratio, alpha);
    const zc b_k = zmul(zmul(ratio, ratio), beta);
#pragma unroll
    for (int l = 0; l < KOMEGA_MAX_NL; ++l) {
      if (l < nl) {
        yy[l] = zadd(yy[l], zmul(a_k, u[l]));
        u[l] = zadd(zdiv(ds.h_pr[h * nl + l], pn), zmul(b_k, u[l]));
      }
    }
    pio = pi;
    pi = pn;
    const bool sw = !(c0.x == 1.0 && c0.y == 0.0 && c1.x == 1.0 && c1.y == 0.0);
    zc a = alpha, b = beta;
    if (sw) {
      pi = zdiv(pi, c1);
      pio = zdiv(pio, c0);
      const zc q = zdiv(c0, c1);
      a = zmul(a, q);
      b = zmul(b, zmul(q, q));
    }
    ba = zdiv(b, a);
    r = sqrt(ds.h_nu[h]) / (zabs(pi) * bnorm);
    if (ds.freeze_tol > 0.0 && r < ds.freeze_tol) active = false;
  }
#pragma unroll
  for (int l = 0; l < KOMEGA_MAX_NL; ++l)
    if (l < nl) y[(size_t)k * nl + l] = yy[l];
  res[k] = r;
}

hipError_t launch_recalc(const DevSolver& ds, int rhs, int nsteps, const zc* znew, int nzn, zc* y, double* res,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_recalc, dim3((unsigned)((nzn + 63) / 64)), dim3(64), 0, st, ds, rhs, nsteps, znew, nzn, y,
                     res);
  return hipGetLastError();
}

// ------------------------------------------------------ contour moments
// s_{k,l} = sum_j w[k][j] x_{j,l}: the moment vectors of the contour-integral
// eigensolver (Sec. 4.1), with trapezoid weights w[k][j] = (z_j - gamma)^{k+1}/N
// supplied by the caller.  x: [nrhs][nz][M] (the kept solutions), s:
// [nrhs][nk][M].  Each x element is read once; one thread per row.
constexpr int MOM_MAXK = 16;

__global__ __launch_bounds__(TPB) void k_moments(const zc* __restrict__ X, int nz, int64_t M, int nk,
                                                 const zc* __restrict__ W, zc* __restrict__ S) {
  const int l = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (i >= M) return;
  zc acc[MOM_MAXK];
#pragma unroll
  for (int k = 0; k < MOM_MAXK; ++k) acc[k] = zmk(0.0, 0.0);
  const zc* x = X + (size_t)l * nz * M + i;
  for (int j = 0; j < nz; ++j) {
    const zc v = x[(size_t)j * M];
#pragma unroll
    for (int k = 0; k < MOM_MAXK; ++k)
      if (k < nk) acc[k] = zadd(acc[k], zmul(W[k * nz + j], v));
  }
  zc* s = S + (size_t)l * nk * M + i;
#pragma unroll
  for (int k = 0; k < MOM_MAXK; ++k)
    if (k < nk) s[(size_t)k * M] = acc[k];
}

hipError_t launch_moments(const void* x, int nz, int64_t M, int nrhs, int nk, const void* w, void* s,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_moments, dim3((unsigned)((M + TPB - 1) / TPB), (unsigned)nrhs), dim3(TPB), 0, st,
                     reinterpret_cast<const zc*>(x), nz, M, nk, reinterpret_cast<const zc*>(w),
                     reinterpret_cast<zc*>(s));
  return hipGetLastError();
}

// ------------------------------------------------------ gradient pieces
// Bond contraction for the derivative of F_k = a^H G(z_k) b with respect to
// the coupling of bond b: dF_k/dJ_b = a^H G (S_i . S_j) G b = w_k^H O_b x_k,
// with x_k = G(z_k) b and w_k = G(z_k)^H a = G(conj z_k) a for Hermitian H.
// O_b acts like one term of the Heisenberg product: (O_b x)_s = (+-1/4) x_s
// + (1/2)[antiparallel] x_{idx(s xor m_b)}.  One pass over rows per chunk of
// GRAD_CH bonds; per-group partial sums in slot order (deterministic).
constexpr int GRAD_CH = 8;

// Bond masks live in LDS padded with null bonds to a multiple of GRAD_CH (so
// the chunk is straight-line code); TLDS puts the index tables in LDS too.
template <bool TLDS>
__global__ __launch_bounds__(TPB) void k_bond_grad(DevOp op, const zc* __restrict__ W, const zc* __restrict__ X,
                                                   int64_t ldw, int64_t ldx, double* part) {
  extern __shared__ unsigned char smem[];
  const int k = blockIdx.y, g = blockIdx.x, G = gridDim.x;
  const int64_t M = op.M;
  const zc* w = W + (size_t)k * ldw;
  const zc* x = X + (size_t)k * ldx;
  const int nbp = (op.nb + GRAD_CH - 1) / GRAD_CH * GRAD_CH;
  uint32_t* sbm = reinterpret_cast<uint32_t*>(smem);
  for (int e = threadIdx.x; e < nbp; e += TPB) sbm[e] = e < op.nb ? op.bmask[e] : 0u;
  const uint32_t* hi = op.hi_off;
  const uint16_t* lo = op.lo_rank;
  if constexpr (TLDS) {
    const int nhi = 1 << (op.L - op.h), nlo = 1 << op.h;
    uint32_t* shi = reinterpret_cast<uint32_t*>(smem + (4 * (size_t)nbp + 15) / 16 * 16);
    uint16_t* slo = reinterpret_cast<uint16_t*>(shi + nhi);
    for (int e = threadIdx.x; e < nhi; e += TPB) shi[e] = op.hi_off[e];
    for (int e = threadIdx.x; e < nlo; e += TPB) slo[e] = op.lo_rank[e];
    hi = shi;
    lo = slo;
  }
  __syncthreads();
  const uint32_t lmask = (1u << op.h) - 1u;
  const int h = op.h;
  for (int b0 = 0; b0 < nbp; b0 += GRAD_CH) {
    double acc[2 * GRAD_CH];
#pragma unroll
    for (int c = 0; c < 2 * GRAD_CH; ++c) acc[c] = 0.0;
    for (int64_t i = (int64_t)g * TPB + threadIdx.x; i < M; i += (int64_t)G * TPB) {
      const uint32_t s = op.states[i];
      const zc wi = zconj(w[i]);
      const zc xi = x[i];
      uint32_t jj[GRAD_CH];
      double dw[GRAD_CH], ow[GRAD_CH];
#pragma unroll
      for (int c = 0; c < GRAD_CH; ++c) {
        // (a null or parallel bond's index stays inside the tables, unused)
        const uint32_t m = sbm[b0 + c];
        const bool anti = __popc(s & m) == 1;
        const uint32_t t = s ^ m;
        jj[c] = hi[t >> h] + (uint32_t)lo[t & lmask];
        dw[c] = anti ? -0.25 : 0.25;
        ow[c] = anti ? 0.5 : 0.0;
      }
      zc xp[GRAD_CH];
#pragma unroll
      for (int c = 0; c < GRAD_CH; ++c) {
        xp[c] = zmk(0.0, 0.0);
        if (ow[c] != 0.0) xp[c] = x[jj[c]];
      }
#pragma unroll
      for (int c = 0; c < GRAD_CH; ++c) {
        const zc ox = zadd(zscale(dw[c], xi), zscale(ow[c], xp[c]));
        const zc v = zmul(wi, ox);
        acc[2 * c] += v.x;
        acc[2 * c + 1] += v.y;
      }
    }
    block_sum<2 * GRAD_CH>(acc);
    if (threadIdx.x == 0) {
      for (int c = 0; c < GRAD_CH && b0 + c < op.nb; ++c) {
        double* slot = part + (((size_t)k * G + g) * op.nb + (b0 + c)) * 2;
        slot[0] = acc[2 * c];
        slot[1] = acc[2 * c + 1];
      }
    }
  }
}

__global__ void k_sum_groups(const double* part, int G, int nb, int nvec, zc* out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nvec * nb) return;
  const int k = e / nb, b = e % nb;
  double re = 0.0, im = 0.0;
  for (int g = 0; g < G; ++g) {
    const double* slot = part + (((size_t)k * G + g) * nb + b) * 2;
    re += slot[0];
    im += slot[1];
  }
  out[e] = zmk(re, im);
}

// Projection a_k^H x_k for n vector pairs (stride 0 reuses one a): the
// projected value F_k = a^H x^(k) (Sec. 2.2.3, G_ab = a^H x) and the
// products w_k^H x_k of the gradient.
// X: complex128, or complex64 (widened; products and sums in double)
template <class X>
__global__ __launch_bounds__(TPB) void k_dotc(const zc* __restrict__ A, int64_t lda, const X* __restrict__ Xv,
                                              int64_t ldx, int64_t M, double* part) {
  const int k = blockIdx.y, g = blockIdx.x, G = gridDim.x;
  const zc* a = A + (size_t)k * lda;
  const X* x = Xv + (size_t)k * ldx;
  double acc[2] = {0.0, 0.0};
  for (int64_t i = (int64_t)g * TPB + threadIdx.x; i < M; i += (int64_t)G * TPB) {
    const zc v = zmul(zconj(a[i]), XS<X>::ld(x[i]));
    acc[0] += v.x;
    acc[1] += v.y;
  }
  block_sum<2>(acc);
  if (threadIdx.x == 0) {
    double* slot = part + ((size_t)k * G + g) * 2;
    slot[0] = acc[0];
    slot[1] = acc[1];
  }
}

hipError_t launch_bond_grad(const DevOp& op, const void* w, int64_t ldw, const void* x, int64_t ldx, int32_t nvec,
                            double* part, int G, void* out, hipStream_t st) {
  const size_t nbp = (size_t)(op.nb + GRAD_CH - 1) / GRAD_CH * GRAD_CH;
  size_t lds = (4 * nbp + 15) / 16 * 16;
  if (op.tables_in_lds) {
    lds += sizeof(uint32_t) * ((size_t)1 << (op.L - op.h)) + sizeof(uint16_t) * ((size_t)1 << op.h);
    hipLaunchKernelGGL((k_bond_grad<true>), dim3((unsigned)G, (unsigned)nvec), dim3(TPB), lds, st, op,
                       reinterpret_cast<const zc*>(w), reinterpret_cast<const zc*>(x), ldw, ldx, part);
  } else {
    hipLaunchKernelGGL((k_bond_grad<false>), dim3((unsigned)G, (unsigned)nvec), dim3(TPB), lds, st, op,
                       reinterpret_cast<const zc*>(w), reinterpret_cast<const zc*>(x), ldw, ldx, part);
  }
  const int n = nvec * op.nb;
  hipLaunchKernelGGL(k_sum_groups, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, part, G, op.nb, nvec,
                     reinterpret_cast<zc*>(out));
  return hipGetLastError();
}

// ---------------------------------------------------------- bandwidth probe
// Streams n 16-byte elements with the access pattern of the whole-x update
// (nontemporal 16-byte loads and stores, grid-stride, PROBE_UNROLL
// independent elements per thread in flight): COPY copies src to dst,
// otherwise src is only read and each work-group writes the sum of the
// elements' first halves to dst[group] (so that the loads are not removed).
constexpr int PROBE_UNROLL = 4;
constexpr int PROBE_GROUPS = 4096;
template <bool COPY>
__global__ __launch_bounds__(TPB) void k_probe(const zc* __restrict__ src, zc* __restrict__ dst, int64_t n) {
  typedef double v2 __attribute__((ext_vector_type(2)));
  const int64_t step = (int64_t)gridDim.x * TPB * PROBE_UNROLL;
  double acc = 0.0;
  for (int64_t base = (int64_t)blockIdx.x * TPB * PROBE_UNROLL + threadIdx.x; base < n; base += step) {
    v2 v[PROBE_UNROLL];
#pragma unroll
    for (int u = 0; u < PROBE_UNROLL; ++u) {
      const int64_t i = base + (int64_t)u * TPB;
      if (i < n) v[u] = __builtin_nontemporal_load(reinterpret_cast<const v2*>(src) + i);
    }
#pragma unroll
    for (int u = 0; u < PROBE_UNROLL; ++u) {
      const int64_t i = base + (int64_t)u * TPB;
      if (i < n) {
        if (COPY) __builtin_nontemporal_store(v[u], reinterpret_cast<v2*>(dst) + i);
        else acc += v[u].x;
      }
    }
  }
  if (!COPY) {
    double t[1] = {acc};
    block_sum<1>(t);
    if (threadIdx.x == 0) dst[blockIdx.x] = zmk(t[0], 0.0);
  }
}

hipError_t launch_stream_probe(const void* src, void* dst, int64_t n, int32_t kind, hipStream_t st) {
  const zc* s = reinterpret_cast<const zc*>(src);
  zc* d = reinterpret_cast<zc*>(dst);
  if (kind == 0) hipLaunchKernelGGL(k_probe<true>, dim3(PROBE_GROUPS), dim3(TPB), 0, st, s, d, n);
  else hipLaunchKernelGGL(k_probe<false>, dim3(PROBE_GROUPS), dim3(TPB), 0, st, s, d, n);
  return hipGetLastError();
}
int32_t stream_probe_groups() { return PROBE_GROUPS; }

hipError_t launch_dotc(const void* a, int64_t lda, const void* x, int64_t ldx, int64_t M, int32_t n, double* part,
                       int G, void* out, int x32, hipStream_t st) {
  if (x32)
    hipLaunchKernelGGL((k_dotc<cf>), dim3((unsigned)G, (unsigned)n), dim3(TPB), 0, st,
                       reinterpret_cast<const zc*>(a), lda, reinterpret_cast<const cf*>(x), ldx, M, part);
  else
    hipLaunchKernelGGL((k_dotc<zc>), dim3((unsigned)G, (unsigned)n), dim3(TPB), 0, st,
                       reinterpret_cast<const zc*>(a), lda, reinterpret_cast<const zc*>(x), ldx, M, part);
  hipLaunchKernelGGL(k_sum_groups, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, part, G, 1, n,
                     reinterpret_cast<zc*>(out));
  return hipGetLastError();
}

// On-site energies: dF_k/deps_i = a^H G(z_k) e_i e_i^T G(z_k) b = conj(w_k[i]) x_k[i]
// with x_k = G(z_k) b, w_k = G(z_k)^H a.  The backward pass needs the
// contraction with the upstream gradient g over the shifts,
// out[i] = sum_k g_k conj(dF_k/deps_i) = sum_k g_k w_k[i] conj(x_k[i]),
// one row per thread, the shifts' coefficients staged in LDS in chunks.
constexpr int ONSITE_CH = 512;
__global__ __launch_bounds__(TPB) void k_onsite_grad(const zc* __restrict__ G, const zc* __restrict__ W, int64_t ldw,
                                                     const zc* __restrict__ X, int64_t ldx, int64_t M, int n,
                                                     zc* __restrict__ out) {
  __shared__ zc sg[ONSITE_CH];
  const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
  zc acc = zmk(0.0, 0.0);
  for (int k0 = 0; k0 < n; k0 += ONSITE_CH) {
    const int kn = n - k0 < ONSITE_CH ? n - k0 : ONSITE_CH;
    __syncthreads();
    for (int e = threadIdx.x; e < kn; e += TPB) sg[e] = G[k0 + e];
    __syncthreads();
    if (i < M) {
      for (int c = 0; c < kn; ++c) {
        const int k = k0 + c;
        const zc wx = zmul(W[(size_t)k * ldw + i], zconj(X[(size_t)k * ldx + i]));
        acc = zadd(acc, zmul(sg[c], wx));
      }
    }
  }
  if (i < M) out[i] = acc;
}

hipError_t launch_onsite_grad(const void* g, const void* w, int64_t ldw, const void* x, int64_t ldx, int64_t M,
                              int32_t n, void* out, hipStream_t st) {
  hipLaunchKernelGGL(k_onsite_grad, dim3((unsigned)((M + TPB - 1) / TPB)), dim3(TPB), 0, st,
                     reinterpret_cast<const zc*>(g), reinterpret_cast<const zc*>(w), ldw,
                     reinterpret_cast<const zc*>(x), ldx, M, n, reinterpret_cast<zc*>(out));
  return hipGetLastError();
}

// =================================================================== launch
int64_t spmv_blocks(const DevOp& op, int64_t M) {
  // every product takes any work-group count (one partial-sum slot each); the
  // Heisenberg row product runs best with one round of resident work-groups
  // (row_groups): at L = 24 on MI355X, 1488..1535 took 55.7..56.2 us, 1568
  // and more 60..63.5 us, since the work-groups past one round (and the
  // finaliser group) then run in a second round
  const int64_t b = stream_blocks(M);
  const int64_t cap = op.row_groups > 0 ? op.row_groups : 1792;
  return (op.kind == OP_HEIS && b > cap) ? cap : b;
}

// One round of resident work-groups of the row product on the current
// device (occupancy of its solver instance with the operator's LDS), less 32
// so that the finaliser group and a few more still fit; 1792 if the runtime
// cannot tell.
int heis_row_groups(const DevOp& op) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 1792;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 1792;
  const size_t lds = heis_row_lds_bytes(op, op.tables_in_lds != 0);
  const hipError_t e =
      op.tables_in_lds
          ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &per, reinterpret_cast<const void*>(&k_spmv<zc, 0, false, true, OP_HEIS, true>), TPB, lds)
          : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &per, reinterpret_cast<const void*>(&k_spmv<zc, 0, false, true, OP_HEIS, false>), TPB, lds);
  if (e != hipSuccess || per < 1 || cus < 1) return 1792;
  int g = per * cus - 32;
  if (g < 64) g = 64;
  if (g > MAXBLK) g = MAXBLK;
  return g;
}

// Product work-groups (= partial-sum slots per system) for several
// right-hand sides of one CSR matrix: one resident round of k_spmv_csr_mr
// (4 work-groups per CU at its 121-123 VGPRs: 1024 on MI355X), at most one per
// row tile, rounded up to a multiple of nrhs (the launch spreads them over
// the nrhs grid rows) and within MAXBLK.  On the 64^3 stencil as CSR with
// 16 right-hand sides: 256 work-groups 292 us, 1024: 123 us, 2048: 133 us.
// Returns 0 when no such count exists (the caller keeps its own).
int64_t csr_mr_groups(int64_t M, int nrhs) {
  static int resident = 0;
  if (resident == 0) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, reinterpret_cast<const void*>(&k_spmv_csr_mr<zc, 0, false>),
                                                     TPB, 0) == hipSuccess &&
        per > 0 && cus > 0)
      resident = per * cus;
    else
      resident = 1024;
  }
  if (nrhs < 2 || nrhs > MAXBLK) return 0;
  const int64_t ntile = (M + TPB - 1) / TPB;
  int64_t g = ntile < resident ? ntile : resident;
  if (g < nrhs) g = nrhs;
  g = (g + nrhs - 1) / nrhs * nrhs;
  if (g > MAXBLK) g = MAXBLK / nrhs * nrhs;
  return g;
}

static int nl_bucket(int nl) { return nl == 0 ? 0 : nl == 1 ? 1 : nl == 2 ? 2 : nl <= 4 ? 4 : 8; }

#define KW_NL_SWITCH(nl, ...) \
  switch (nl_bucket(nl)) {     \
    case 0: { constexpr int NLV = 0; __VA_ARGS__; } break; \
    case 1: { constexpr int NLV = 1; __VA_ARGS__; } break; \
    case 2: { constexpr int NLV = 2; __VA_ARGS__; } break; \
    case 4: { constexpr int NLV = 4; __VA_ARGS__; } break; \
    default: { constexpr int NLV = 8; __VA_ARGS__; } break; \
  }

// Method -> (vector type, inner product, shadow)
#define KW_METHOD_SWITCH(method, ...)                                      \
  switch (method) {                                                        \
    case KOMEGA_CG_R: { typedef double VV; constexpr int DKV = 1; constexpr bool SHV = false; __VA_ARGS__; } break; \
    case KOMEGA_CG_C: { typedef zc VV; constexpr int DKV = 1; constexpr bool SHV = false; __VA_ARGS__; } break;     \
    case KOMEGA_COCG: { typedef zc VV; constexpr int DKV = 0; constexpr bool SHV = false; __VA_ARGS__; } break;     \
    default: { typedef zc VV; constexpr int DKV = 1; constexpr bool SHV = true; __VA_ARGS__; } break;               \
  }

// Grid of the streaming kernels: (groups, nrhs), or the batched work list.
static dim3 grid_b(const DevSolver& ds, int64_t nblk) {
  return ds.soff ? dim3((unsigned)ds.nwl_b) : dim3((unsigned)nblk, (unsigned)ds.nrhs);
}
static dim3 grid_a(const DevSolver& ds, int64_t nblkA, bool lead) {
  return ds.soff ? dim3((unsigned)ds.nwl_a) : dim3((unsigned)(nblkA + (lead ? 1 : 0)), (unsigned)ds.nrhs);
}

hipError_t launch_init(const DevSolver& ds, const Buffers& bf, const void* b, const void* bshadow, void* x,
                       hipStream_t st) {
  const int64_t nblkB = ds.nblkB;
  const dim3 grid = grid_b(ds, nblkB);
  KW_METHOD_SWITCH(ds.method, {
    if (ds.x32) {
      hipLaunchKernelGGL((k_init_copy<VV, cf>), grid, dim3(TPB), 0, st, ds, bf,
                         reinterpret_cast<const VV*>(b), reinterpret_cast<const VV*>(bshadow),
                         reinterpret_cast<cf*>(x));
    } else {
      hipLaunchKernelGGL((k_init_copy<VV, VV>), grid, dim3(TPB), 0, st, ds, bf,
                         reinterpret_cast<const VV*>(b), reinterpret_cast<const VV*>(bshadow),
                         reinterpret_cast<VV*>(x));
    }
    KW_NL_SWITCH(ds.nl, hipLaunchKernelGGL((k_init<VV, DKV, SHV, NLV>), grid, dim3(TPB), 0, st, ds, bf, ds.P));
  });
  hipLaunchKernelGGL(k_init_fin, dim3(1, (unsigned)ds.nrhs), dim3(TPB), 0, st, ds, (int)nblkB);
  return hipGetLastError();
}

template <class V, int DK, bool SH, bool DOT>
static void spmv_dispatch(const DevSolver& ds, const DevOp& op, const Buffers& bf, dim3 grid, int nblkB,
                          hipStream_t st) {
  switch (op.kind) {
    case OP_STENCIL:
      hipLaunchKernelGGL((k_spmv<V, DK, SH, DOT, OP_STENCIL, false>), grid, dim3(TPB), 0, st, ds, op, bf, nblkB);
      break;
    case OP_CSR:
      if (op.complex_vals)
        hipLaunchKernelGGL((k_spmv<V, DK, SH, DOT, OP_CSR, true>), grid, dim3(TPB), 0, st, ds, op, bf, nblkB);
      else
        hipLaunchKernelGGL((k_spmv<V, DK, SH, DOT, OP_CSR, false>), grid, dim3(TPB), 0, st, ds, op, bf, nblkB);
      break;
    default:
      if (op.group_kernel) {
        const size_t glds = heis_grp_lds_bytes(op, SH);
        hipLaunchKernelGGL((k_spmv_heis_grp<V, DK, SH, DOT>), grid, dim3(TPB), glds, st, ds, op, bf, nblkB);
      } else if (op.tables_in_lds) {
        hipLaunchKernelGGL((k_spmv<V, DK, SH, DOT, OP_HEIS, true>), grid, dim3(TPB), heis_row_lds_bytes(op, true),
                           st, ds, op, bf, nblkB);
      } else {
        hipLaunchKernelGGL((k_spmv<V, DK, SH, DOT, OP_HEIS, false>), grid, dim3(TPB), heis_row_lds_bytes(op, false),
                           st, ds, op, bf, nblkB);
      }
      break;
  }
}

hipError_t launch_spmv(const DevSolver& ds, const DevOp& op, const Buffers& bf, bool with_dot, int64_t nblkA,
                       hipStream_t st) {
  const int nblkB = ds.nblkB;
  if (op.kind == OP_CSR && with_dot && !ds.soff && ds.nrhs > 1 && ds.method != KOMEGA_BICG &&
      nblkA % ds.nrhs == 0) {
    // several right-hand sides of one CSR matrix: the matrix is read once
    // per 8 of them (k_spmv_csr_mr), same slots
    const dim3 grid((unsigned)(nblkA / ds.nrhs + 1), (unsigned)ds.nrhs);
    KW_METHOD_SWITCH(ds.method, {
      if constexpr (!SHV) {
        if (op.complex_vals)
          hipLaunchKernelGGL((k_spmv_csr_mr<VV, DKV, true>), grid, dim3(TPB), 0, st, ds, op, bf, nblkB);
        else
          hipLaunchKernelGGL((k_spmv_csr_mr<VV, DKV, false>), grid, dim3(TPB), 0, st, ds, op, bf, nblkB);
      }
    });
    return hipGetLastError();
  }
  const dim3 grid = grid_a(ds, nblkA, with_dot);
  KW_METHOD_SWITCH(ds.method, {
    if (with_dot) spmv_dispatch<VV, DKV, SHV, true>(ds, op, bf, grid, nblkB, st);
    else spmv_dispatch<VV, DKV, SHV, false>(ds, op, bf, grid, nblkB, st);
  });
  return hipGetLastError();
}

hipError_t launch_op_apply(const DevOp& op, const void* v, void* out, int32_t nvec, int32_t is_complex,
                           hipStream_t st) {
  DevSolver ds{};
  ds.M = op.M;
  Buffers bf{};
  if (op.nsys) {
    // one cube per system: the operator's own work list, one launch per vector
    ds.soff = op.soff;
    ds.wl_a = op.wl;
    ds.nwl_a = op.nwl;
    ds.nrhs = op.nsys;
    const size_t es = is_complex ? 16 : 8;
    for (int32_t k = 0; k < nvec; ++k) {
      bf.R = const_cast<char*>(reinterpret_cast<const char*>(v)) + (size_t)k * op.M * es;
      bf.Q = reinterpret_cast<char*>(out) + (size_t)k * op.M * es;
      if (is_complex) spmv_dispatch<zc, 0, false, false>(ds, op, bf, dim3((unsigned)op.nwl), 0, st);
      else spmv_dispatch<double, 0, false, false>(ds, op, bf, dim3((unsigned)op.nwl), 0, st);
    }
    return hipGetLastError();
  }
  bf.R = const_cast<void*>(v);
  bf.Q = out;
  const dim3 grid((unsigned)spmv_blocks(op, op.M), (unsigned)nvec);
  if (is_complex) spmv_dispatch<zc, 0, false, false>(ds, op, bf, grid, 0, st);
  else spmv_dispatch<double, 0, false, false>(ds, op, bf, grid, 0, st);
  return hipGetLastError();
}

hipError_t launch_dot(const DevSolver& ds, const void* dual, const void* q, int64_t nblkA, hipStream_t st) {
  const int nblkB = ds.nblkB;
  const dim3 grid = grid_a(ds, nblkA, true);
  KW_METHOD_SWITCH(ds.method, {
    hipLaunchKernelGGL((k_dot<VV, DKV>), grid, dim3(TPB), 0, st, ds,
                       reinterpret_cast<const VV*>(dual), reinterpret_cast<const VV*>(q), nblkB);
  });
  return hipGetLastError();
}

hipError_t launch_seed(const DevSolver& ds, const Buffers& bf, bool inplace, int64_t nblkA, int64_t nblkB,
                       hipStream_t st) {
  const dim3 grid = grid_b(ds, nblkB);
  KW_METHOD_SWITCH(ds.method, {
    KW_NL_SWITCH(ds.nl, {
      if (inplace)
        hipLaunchKernelGGL((k_seed<VV, DKV, SHV, NLV, true>), grid, dim3(TPB), 0, st, ds, bf, ds.P, (int)nblkA);
      else
        hipLaunchKernelGGL((k_seed<VV, DKV, SHV, NLV, false>), grid, dim3(TPB), 0, st, ds, bf, ds.P, (int)nblkA);
    });
  });
  return hipGetLastError();
}

hipError_t launch_finalize(const DevSolver& ds, int64_t nblkB, hipStream_t st) {
  hipLaunchKernelGGL(k_finalize, dim3(1, (unsigned)ds.nrhs), dim3(TPB), 0, st, ds, (int)nblkB);
  return hipGetLastError();
}

template <class V, class X, int SB>
static void shift_launch(const DevSolver& ds, const Buffers& bf, hipStream_t st) {
  const unsigned nsb = (unsigned)((ds.nz + SB - 1) / SB);
  const unsigned ntile = ds.soff ? (unsigned)ds.nwl_t : (unsigned)((ds.M + TPB - 1) / TPB);
  // the y dimension holds at most 65535 blocks
  const bool swap = ds.shift_order == 1 && ntile <= 65535u;
  const dim3 grid = swap ? dim3(nsb, ntile, ds.soff ? 1u : (unsigned)ds.nrhs)
                         : dim3(ntile, nsb, ds.soff ? 1u : (unsigned)ds.nrhs);
  const V* R = reinterpret_cast<const V*>(bf.R);
  X* x = reinterpret_cast<X*>(bf.x);
  X* p = reinterpret_cast<X*>(bf.p);
  if (ds.shift_nt) {
    if (swap) hipLaunchKernelGGL((k_shift<V, X, SB, true, true>), grid, dim3(TPB), 0, st, ds, R, x, p);
    else hipLaunchKernelGGL((k_shift<V, X, SB, true, false>), grid, dim3(TPB), 0, st, ds, R, x, p);
  } else {
    if (swap) hipLaunchKernelGGL((k_shift<V, X, SB, false, true>), grid, dim3(TPB), 0, st, ds, R, x, p);
    else hipLaunchKernelGGL((k_shift<V, X, SB, false, false>), grid, dim3(TPB), 0, st, ds, R, x, p);
  }
}

template <class V, class X>
static void shift_sb(const DevSolver& ds, const Buffers& bf, hipStream_t st) {
  switch (ds.shift_block) {
    case 1: shift_launch<V, X, 1>(ds, bf, st); break;
    case 2: shift_launch<V, X, 2>(ds, bf, st); break;
    case 4: shift_launch<V, X, 4>(ds, bf, st); break;
    case 16: shift_launch<V, X, 16>(ds, bf, st); break;
    default: shift_launch<V, X, 8>(ds, bf, st); break;
  }
}

hipError_t launch_shift(const DevSolver& ds, const Buffers& bf, hipStream_t st) {
  if (ds.method == KOMEGA_CG_R) shift_sb<double, double>(ds, bf, st);
  else if (ds.x32) shift_sb<zc, cf>(ds, bf, st);
  else shift_sb<zc, zc>(ds, bf, st);
  return hipGetLastError();
}

template <class V, class X, int T>
static void shift_blk_launch(const DevSolver& ds, const void* ring, int64_t vr, int slot0, int nb, void* x, void* p,
                             hipStream_t st) {
  const int64_t ntile = ds.soff ? ds.nwl_t : (ds.M + TPB - 1) / TPB;
  const int64_t nsys = ds.soff ? 1 : ds.nrhs;
  // split the shifts so that the launch holds about five rounds of resident
  // work-groups (the last, partly filled round then costs little); the
  // residency of this instance is taken once from the runtime (3 work-groups
  // per CU for FP64 x at T = 32, 6 for complex64 x at T = 16)
  static int resident = 0;
  if (resident == 0) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, reinterpret_cast<const void*>(&k_shift_blk<V, X, T, true>),
                                                     TPB, 0) == hipSuccess &&
        per > 0 && cus > 0)
      resident = per * cus;
    else
      resident = 819;  // so that five rounds are about 4096 work-groups
  }
  int64_t split = (5 * (int64_t)resident + ntile * nsys - 1) / (ntile * nsys);
  const int64_t maxsplit = (ds.nz + XBLK_SHIFTS - 1) / XBLK_SHIFTS;
  if (split > maxsplit) split = maxsplit;
  if (split < 1) split = 1;
  const dim3 grid((unsigned)ntile, (unsigned)split, (unsigned)nsys);
  const V* R = reinterpret_cast<const V*>(ring);
  if (ds.shift_nt)
    hipLaunchKernelGGL((k_shift_blk<V, X, T, true>), grid, dim3(TPB), 0, st, ds, R, vr, slot0, nb,
                       reinterpret_cast<X*>(x), reinterpret_cast<X*>(p));
  else
    hipLaunchKernelGGL((k_shift_blk<V, X, T, false>), grid, dim3(TPB), 0, st, ds, R, vr, slot0, nb,
                       reinterpret_cast<X*>(x), reinterpret_cast<X*>(p));
}

template <class V, class X>
static void shift_blk_t(const DevSolver& ds, const void* ring, int64_t vr, int slot0, int nb, void* x, void* p,
                        hipStream_t st) {
  if (ds.xblk <= 4) shift_blk_launch<V, X, 4>(ds, ring, vr, slot0, nb, x, p, st);
  else if (ds.xblk <= 8) shift_blk_launch<V, X, 8>(ds, ring, vr, slot0, nb, x, p, st);
  else if (ds.xblk <= 16) shift_blk_launch<V, X, 16>(ds, ring, vr, slot0, nb, x, p, st);
  else shift_blk_launch<V, X, 32>(ds, ring, vr, slot0, nb, x, p, st);
}

hipError_t launch_shift_blk(const DevSolver& ds, const void* ring, int64_t vr, int slot0, int nb, void* x, void* p,
                            hipStream_t st) {
  const int64_t nmap = (int64_t)ds.nrhs * ds.nz;
  hipLaunchKernelGGL(k_block_map, dim3((unsigned)((nmap + TPB - 1) / TPB)), dim3(TPB), 0, st, ds);
  if (ds.method == KOMEGA_CG_R) shift_blk_t<double, double>(ds, ring, vr, slot0, nb, x, p, st);
  else if (ds.x32) shift_blk_t<zc, cf>(ds, ring, vr, slot0, nb, x, p, st);
  else shift_blk_t<zc, zc>(ds, ring, vr, slot0, nb, x, p, st);
  return hipGetLastError();
}


hipError_t launch_heis_setup(DevOp& op, const int64_t* binom, hipStream_t st) {
  uint32_t* states = const_cast<uint32_t*>(op.states);
  hipLaunchKernelGGL(k_heis_basis, dim3((unsigned)((op.M + 255) / 256)), dim3(256), 0, st, states, op.M,
                     op.L, op.nup, binom);
  const int nlo = 1 << op.h;
  hipLaunchKernelGGL(k_heis_lo, dim3((unsigned)((nlo + 255) / 256)), dim3(256), 0, st,
                     const_cast<uint16_t*>(op.lo_rank), op.h, binom);
  return hipGetLastError();
}

hipError_t launch_heis_hi(DevOp& op, const int64_t* binom, int64_t* total, hipStream_t st) {
  const int nhi = 1 << (op.L - op.h);
  hipLaunchKernelGGL(k_heis_hi, dim3(1), dim3(1024), 0, st, const_cast<uint32_t*>(op.hi_off), nhi, op.h,
                     op.nup, binom, total);
  return hipGetLastError();
}

hipError_t launch_heis_check(const DevOp& op, int32_t* bad, hipStream_t st) {
  hipLaunchKernelGGL(k_heis_check, dim3((unsigned)((op.M + 255) / 256)), dim3(256), 0, st, op, bad);
  return hipGetLastError();
}

hipError_t launch_heis_lookup(const DevOp& op, const uint32_t* states, int64_t* idx, int64_t n, int32_t* bad,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_heis_lookup, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, op, states, idx, n, bad);
  return hipGetLastError();
}

hipError_t launch_heis_szq(const DevOp& op, const zc* w, const void* v, void* out, hipStream_t st) {
  Phases ph;
  for (int j = 0; j < 32; ++j) ph.w[j] = j < op.L ? w[j] : zmk(0.0, 0.0);
  hipLaunchKernelGGL(k_heis_szq, dim3((unsigned)((op.M + 255) / 256)), dim3(256), 0, st, op, ph,
                     reinterpret_cast<const zc*>(v), reinterpret_cast<zc*>(out));
  return hipGetLastError();
}

}  // namespace kw
