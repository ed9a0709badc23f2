/*
 * komega_oracle.c -- plain FP64 CPU oracle of the shifted Krylov solver.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the independent reference against
 * which the GPU library is checked.  Only the test-suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it.  It shares no code, no
 * header and no table with the GPU library: it has its own operators, its
 * own spin basis (a brute-force scan) and its own index (binary search).
 *
 * What it computes (Kawamura et al., "K-omega: open-source library for the
 * shifted Krylov subspace method", Sec. 2):
 *   - the shifted linear systems (z_k I - H) x^(k) = b, k = 0..N_z-1
 *     (Sec. 1, Eq. EQ-SHIFT-EQ), rewritten as (A + sigma I) x = b with
 *     A = z_seed I - H and sigma = z_k - z_seed (Sec. 2.1, Eq. EQ-SHIFT-EQ2);
 *   - the seed system by the three-term CG recurrence (Sec. 2.2.1,
 *     Eqs. EQ-CG-RN-3REC and EQ-REC-ALPHA-N2, with beta_{-1}/alpha_{-1} = 0);
 *   - the shifted systems through the collinearity factors pi (Sec. 2.2.2,
 *     Eqs. EQ-COLLINEAR, EQ-SHIFTEDCG-PI, EQ-SHIFTEDCG-alpha/beta/x/p);
 *   - the projected variant y = P x (Sec. 2.2.3, Eqs. EQ-SHIFTEDCG-y/u, with
 *     the index of the u-update read as P applied to EQ-SHIFTEDCG-p);
 *   - seed switching to the shift of smallest |pi| after every update
 *     (Sec. 2.2.4);
 *   - the COCG form (bilinear x^T y products, Appendix A) and the BiCG form
 *     (shadow residual, Appendix B) through the same shifted equations.
 *
 * Arithmetic: IEEE binary64, C99 complex, compiled with -ffp-contract=off.
 * Every reduction runs sequentially in index order.  Row loops that write
 * disjoint outputs (operator application, elementwise vector updates) may be
 * split over OpenMP threads; that does not change any rounding, so results
 * do not depend on the thread count.
 */
#include <complex.h>
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

/* Number of threads the OpenMP row loops use (1 without OpenMP). */
int orc_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Status codes (same meaning as the library's, but defined independently). */
enum {
  ORC_OK = 0,
  ORC_CONVERGED = 1,
  ORC_E_INVALID = -1,
  ORC_E_BREAKDOWN = -2,
  ORC_E_SHIFT_BREAKDOWN = -3,
  ORC_E_MAXITER = -4,
  ORC_E_NONFINITE = -7
};

enum { ORC_CG_R = 0, ORC_CG_C = 1, ORC_COCG = 2, ORC_BICG = 3 };
enum { ORC_STENCIL3D = 1, ORC_CSR = 2, ORC_HEISENBERG = 3 };

/*
 * Operator description.  H must be real symmetric or Hermitian (Sec. 3.2.1 ii).
 *  STENCIL3D : Anderson tight-binding cube, site i = x + Lx*(y + Ly*z),
 *              H_ii = eps_i, H_ij = -hop for the 6 periodic neighbours.
 *  CSR       : H given row by row; values complex.
 *  HEISENBERG: H = sum_b J_b S_{bi[b]} . S_{bj[b]} for spin 1/2 (Sec. 4.2,
 *              Eq. eq:heisenberg with per-bond couplings), restricted to the
 *              states with nup up spins.  Site j is bit j, up = 1; the basis
 *              'states' is ascending (built by orc_heis_basis).
 */
typedef struct {
  int32_t kind;
  int32_t pad0;
  int64_t M;
  /* stencil */
  int32_t Lx, Ly, Lz, pad1;
  double hop;
  const double* eps;
  /* csr */
  const int64_t* rowptr;
  const int32_t* col;
  const cplx* val;
  /* heisenberg */
  int32_t L, nup, nb, pad2;
  const int32_t* bi;
  const int32_t* bj;
  const double* J;
  const uint32_t* states;
} orc_op;

static int popcount32(uint32_t s) {
  int c = 0;
  while (s) { c += (int)(s & 1u); s >>= 1; }
  return c;
}

/* Basis of the fixed-magnetisation sector: every L-bit integer with nup set
 * bits, ascending.  Returns the count; writes the states when out != NULL.
 * Brute force over all 2^L integers -- deliberately the simplest possible
 * enumeration. */
int64_t orc_heis_basis(int32_t L, int32_t nup, uint32_t* out) {
  if (L < 1 || L > 32 || nup < 0 || nup > L) return -1;
  int64_t n = 0;
  uint64_t end = (uint64_t)1 << L;
  for (uint64_t s = 0; s < end; ++s) {
    if (popcount32((uint32_t)s) == nup) {
      if (out) out[n] = (uint32_t)s;
      ++n;
    }
  }
  return n;
}

/* Position of state s in the ascending basis by binary search; -1 if absent. */
int64_t orc_heis_index(const uint32_t* states, int64_t M, uint32_t s) {
  int64_t lo = 0, hi = M - 1;
  while (lo <= hi) {
    int64_t mid = lo + (hi - lo) / 2;
    uint32_t v = states[mid];
    if (v == s) return mid;
    if (v < s) lo = mid + 1; else hi = mid - 1;
  }
  return -1;
}

/* out = H v.  Returns 0, or -1 for an unknown operator / missing basis state. */
int orc_apply(const orc_op* op, const cplx* v, cplx* out) {
  int64_t M = op->M;
  int bad = 0;
  if (op->kind == ORC_STENCIL3D) {
    int64_t Lx = op->Lx, Ly = op->Ly, Lz = op->Lz;
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < Lz; ++z) {
      for (int64_t y = 0; y < Ly; ++y) {
        for (int64_t x = 0; x < Lx; ++x) {
          int64_t i = x + Lx * (y + Ly * z);
          int64_t xm = (x + Lx - 1) % Lx, xp = (x + 1) % Lx;
          int64_t ym = (y + Ly - 1) % Ly, yp = (y + 1) % Ly;
          int64_t zm = (z + Lz - 1) % Lz, zp = (z + 1) % Lz;
          cplx nb = v[xm + Lx * (y + Ly * z)] + v[xp + Lx * (y + Ly * z)] +
                    v[x + Lx * (ym + Ly * z)] + v[x + Lx * (yp + Ly * z)] +
                    v[x + Lx * (y + Ly * zm)] + v[x + Lx * (y + Ly * zp)];
          out[i] = op->eps[i] * v[i] - op->hop * nb;
        }
      }
    }
    return 0;
  }
  if (op->kind == ORC_CSR) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < M; ++i) {
      cplx acc = 0.0;
      for (int64_t p = op->rowptr[i]; p < op->rowptr[i + 1]; ++p)
        acc += op->val[p] * v[op->col[p]];
      out[i] = acc;
    }
    return 0;
  }
  if (op->kind == ORC_HEISENBERG) {
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int64_t i = 0; i < M; ++i) {
      uint32_t s = op->states[i];
      double diag = 0.0;
      cplx off = 0.0;
      for (int b = 0; b < op->nb; ++b) {
        int bi = op->bi[b], bj = op->bj[b];
        uint32_t ui = (s >> bi) & 1u, uj = (s >> bj) & 1u;
        if (ui == uj) {
          /* S^z_i S^z_j = +1/4 on parallel spins */
          diag += 0.25 * op->J[b];
        } else {
          /* S^z_i S^z_j = -1/4; (S+S- + S-S+)/2 flips the pair with weight 1/2 */
          diag -= 0.25 * op->J[b];
          uint32_t t = s ^ ((1u << bi) | (1u << bj));
          int64_t j = orc_heis_index(op->states, M, t);
          if (j < 0) { bad = 1; continue; }
          off += 0.5 * op->J[b] * v[j];
        }
      }
      out[i] = diag * v[i] + off;
    }
    return bad ? -1 : 0;
  }
  return -1;
}

/* Excited vector out_s = [sum_j w_j (n_j(s) - 1/2)] v_s, i.e. S^z(q) v with
 * S^z(q) = sum_j e^{iqj} S^z_j (Sec. 4.2, Eq. eq:dynamicalspin); the phases
 * w_j = e^{iqj} are supplied by the caller. */
void orc_heis_szq(const uint32_t* states, int64_t M, int32_t L, const cplx* w,
                  const cplx* v, cplx* out) {
  for (int64_t i = 0; i < M; ++i) {
    cplx c = 0.0;
    for (int j = 0; j < L; ++j) {
      double sz = ((states[i] >> j) & 1u) ? 0.5 : -0.5;
      c += w[j] * sz;
    }
    out[i] = c * v[i];
  }
}

/* ------------------------------------------------------------------------ */
/* Inner products, sequential in index order.                               */
static cplx dot_bilinear(int64_t n, const cplx* x, const cplx* y) {
  cplx s = 0.0;
  for (int64_t i = 0; i < n; ++i) s += x[i] * y[i];
  return s;
}
static cplx dot_sesq(int64_t n, const cplx* x, const cplx* y) {
  cplx s = 0.0;
  for (int64_t i = 0; i < n; ++i) s += conj(x[i]) * y[i];
  return s;
}
static int finite_c(cplx a) { return isfinite(creal(a)) && isfinite(cimag(a)); }

/*
 * Arguments of one shifted solve.
 *   method    : ORC_CG_R / ORC_CG_C (shifted CG, Sec. 2.2), ORC_COCG (App. A),
 *               ORC_BICG (App. B).  CG needs real shifts.
 *   z[nz]     : shifts z_k.  The first seed is z[0] (Sec. 2.1: A = z_0 I - H).
 *   nl, P     : nl = 0 keeps the whole x^(k) (P = I); nl >= 1 keeps only
 *               y^(k) = P x^(k) with P an nl x M row-major matrix (Sec. 2.2.3).
 *   tol       : stop when max_k ||r^k|| / ||b|| < tol (2-norms).
 *   freeze_tol: a shift whose relative residual falls below freeze_tol stops
 *               being updated and leaves the seed choice (0 = never freeze).
 *   seed_switch: switch the seed to argmin |pi| after every update (Sec. 2.2.4).
 *   out       : nl >= 1: y[k*nl + l];  nl = 0: x[k*M + i].
 *   res[nz]   : final relative residual per shift.
 *   hist_*    : optional (may be NULL), itermax entries: alpha_n, beta_n and the
 *               seed shift of step n, and the seed index after step n.
 */
typedef struct {
  int32_t method;
  int32_t nz;
  const cplx* z;
  int32_t nl;
  int32_t itermax;
  const cplx* P;
  double tol;
  double freeze_tol;
  int32_t seed_switch;
  int32_t pad;
  cplx* out;
  double* res;
  int32_t iters;
  int32_t status;
  int32_t seed;
  int32_t nswitch;
  cplx* hist_alpha;
  cplx* hist_beta;
  cplx* hist_zseed;
  int32_t* hist_seed;
} orc_solve_args;

/* Inner product that defines rho and t for the method: x^T y for COCG
 * (App. A), x^H y for CG (Eq. EQ-REC-RHO) and for BiCG with the shadow on the
 * left (App. B). */
static cplx method_dot(int method, int64_t n, const cplx* x, const cplx* y) {
  return method == ORC_COCG ? dot_bilinear(n, x, y) : dot_sesq(n, x, y);
}

int orc_solve(const orc_op* op, int64_t M, const cplx* b, const cplx* bshadow,
              orc_solve_args* a) {
  const int method = a->method;
  const int nz = a->nz, nl = a->nl;
  const int bicg = (method == ORC_BICG);
  a->iters = 0; a->status = ORC_OK; a->seed = 0; a->nswitch = 0;
  if (M < 1 || nz < 1 || nl < 0 || a->itermax < 0) return a->status = ORC_E_INVALID;
  if (nl > 0 && a->P == NULL) return a->status = ORC_E_INVALID;
  if (method == ORC_CG_R || method == ORC_CG_C)
    for (int k = 0; k < nz; ++k)
      if (cimag(a->z[k]) != 0.0) return a->status = ORC_E_INVALID;

  const size_t vb = (size_t)M * sizeof(cplx);
  cplx* r = malloc(vb);
  cplx* r_old = calloc((size_t)M, sizeof(cplx));
  cplx* r_new = malloc(vb);
  cplx* q = malloc(vb);
  cplx *rs = NULL, *rs_old = NULL, *rs_new = NULL, *qs = NULL;
  if (bicg) {
    rs = malloc(vb); rs_old = calloc((size_t)M, sizeof(cplx));
    rs_new = malloc(vb); qs = malloc(vb);
  }
  cplx* pi = malloc(sizeof(cplx) * nz);
  cplx* pi_old = malloc(sizeof(cplx) * nz);
  unsigned char* active = malloc((size_t)nz);
  cplx* u = NULL;  /* projected search directions u^k (nz x nl)            */
  cplx* p = NULL;  /* full search directions p^k (nz x M)                  */
  cplx* Pr = NULL; /* P r_{n+1} (nl)                                       */
  if (nl > 0) { u = malloc(sizeof(cplx) * (size_t)nz * nl); Pr = malloc(sizeof(cplx) * nl); }
  else p = malloc(sizeof(cplx) * (size_t)nz * (size_t)M);

  int status = ORC_OK;

  /* ---- initialisation: x_0 = 0, r_0 = p_0 = b (Sec. 2.2.1), pi_0 = pi_{-1} = 1
   *      (Eq. EQ-SHIFTEDCG-PI), y_0 = 0, u_0 = P b (Eq. EQ-SHIFTEDCG-u). */
  memcpy(r, b, vb);
  if (bicg) {
    /* Shadow start: any vector not orthogonal to b (App. B); default conj(b). */
    for (int64_t i = 0; i < M; ++i) rs[i] = bshadow ? bshadow[i] : conj(b[i]);
  }
  cplx rho = method_dot(method, M, bicg ? rs : r, r);
  double nu = creal(dot_sesq(M, r, r));
  const double bnorm = sqrt(nu);
  for (int k = 0; k < nz; ++k) { pi[k] = 1.0; pi_old[k] = 1.0; active[k] = 1; }
  if (nl > 0) {
    for (int l = 0; l < nl; ++l) {
      cplx s = 0.0;
      for (int64_t i = 0; i < M; ++i) s += a->P[(size_t)l * M + i] * b[i];
      for (int k = 0; k < nz; ++k) { u[(size_t)k * nl + l] = s; a->out[(size_t)k * nl + l] = 0.0; }
    }
  } else {
    for (int k = 0; k < nz; ++k) {
      memcpy(p + (size_t)k * M, b, vb);
      memset(a->out + (size_t)k * M, 0, vb);
    }
  }
  for (int k = 0; k < nz; ++k) a->res[k] = bnorm > 0.0 ? 1.0 : 0.0;

  int seed = 0;
  cplx zs = a->z[0];
  cplx ba = 0.0; /* beta_{n-1}/alpha_{n-1}; starts at 0 (Sec. 2.2.1) */
  int n = 0;

  if (bnorm == 0.0) { status = ORC_CONVERGED; goto done; }
  if (!finite_c(rho) || !isfinite(nu)) { status = ORC_E_NONFINITE; goto done; }
  if (cabs(rho) <= 16.0 * DBL_EPSILON * nu) { status = ORC_E_BREAKDOWN; goto done; }

  for (n = 0; n < a->itermax; ++n) {
    /* q = H r_n (and H r~_n for BiCG): the caller-side product of Alg. 1. */
    if (orc_apply(op, r, q) != 0) { status = ORC_E_INVALID; break; }
    if (bicg && orc_apply(op, rs, qs) != 0) { status = ORC_E_INVALID; break; }

    /* alpha_n = rho_n / (r_n^T A r_n - (beta_{n-1}/alpha_{n-1}) rho_n)
     * (Eq. EQ-REC-ALPHA-N2) with A r = z_s r - H r. */
    cplx t = method_dot(method, M, bicg ? rs : r, q);
    cplx rAr = zs * rho - t;
    cplx den = rAr - ba * rho;
    if (!finite_c(den)) { status = ORC_E_NONFINITE; break; }
    if (den == 0.0) { status = ORC_E_BREAKDOWN; break; }
    cplx alpha = rho / den;
    cplx gamma = alpha * ba; /* alpha_n beta_{n-1} / alpha_{n-1} */

    /* r_{n+1} = (1 + gamma - alpha A) r_n - gamma r_{n-1}  (Eq. EQ-CG-RN-3REC) */
    cplx c_r = 1.0 + gamma - alpha * zs;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < M; ++i)
      r_new[i] = c_r * r[i] + alpha * q[i] - gamma * r_old[i];
    if (bicg) {
      /* shadow: conjugate coefficients and A^H = conj(z_s) I - H (App. B) */
      cplx c_rs = conj(c_r), ca = conj(alpha), cg = conj(gamma);
#pragma omp parallel for schedule(static)
      for (int64_t i = 0; i < M; ++i)
        rs_new[i] = c_rs * rs[i] + ca * qs[i] - cg * rs_old[i];
    }

    /* rho_{n+1}, the residual norm and the projection P r_{n+1} */
    cplx rho_new = method_dot(method, M, bicg ? rs_new : r_new, r_new);
    double nu_new = creal(dot_sesq(M, r_new, r_new));
    if (nl > 0)
      for (int l = 0; l < nl; ++l) {
        cplx s = 0.0;
        for (int64_t i = 0; i < M; ++i) s += a->P[(size_t)l * M + i] * r_new[i];
        Pr[l] = s;
      }
    if (!finite_c(rho_new) || !isfinite(nu_new)) { status = ORC_E_NONFINITE; break; }

    /* beta_n = rho_{n+1} / rho_n  (Eq. EQ-REC-BETA) */
    cplx beta = rho_new / rho;
    if (a->hist_alpha) a->hist_alpha[n] = alpha;
    if (a->hist_beta) a->hist_beta[n] = beta;
    if (a->hist_zseed) a->hist_zseed[n] = zs;

    /* Shifted systems (Eqs. EQ-SHIFTEDCG-PI, -alpha, -beta and -x/-p or -y/-u) */
    for (int k = 0; k < nz && status == ORC_OK; ++k) {
      if (!active[k]) continue;
      cplx sigma = a->z[k] - zs;
      cplx pn = (1.0 + gamma + alpha * sigma) * pi[k] - gamma * pi_old[k];
      if (!finite_c(pn)) { status = ORC_E_NONFINITE; break; }
      if (pn == 0.0) { status = ORC_E_SHIFT_BREAKDOWN; break; }
      cplx ratio = pi[k] / pn;
      cplx ak = ratio * alpha;
      cplx bk = ratio * ratio * beta;
      if (nl > 0) {
        for (int l = 0; l < nl; ++l) {
          cplx* yk = a->out + (size_t)k * nl + l;
          cplx* uk = u + (size_t)k * nl + l;
          *yk += ak * *uk;              /* y_{n+1} = y_n + alpha^k u_n       */
          *uk = Pr[l] / pn + bk * *uk;  /* u_{n+1} = P r_{n+1}/pi_{n+1} + beta^k u_n */
        }
      } else {
        cplx* xk = a->out + (size_t)k * M;
        cplx* pk = p + (size_t)k * M;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < M; ++i) {
          xk[i] += ak * pk[i];               /* x_{n+1} = x_n + alpha^k p_n */
          pk[i] = r_new[i] / pn + bk * pk[i]; /* p_{n+1} = r_{n+1}/pi_{n+1} + beta^k p_n */
        }
      }
      pi_old[k] = pi[k];
      pi[k] = pn;
    }
    if (status != ORC_OK) break;

    /* Seed switching (Sec. 2.2.4): the new seed is the active shift with the
     * smallest |pi_{n+1}| (largest residual); switch only if it is strictly
     * smaller than the current seed's, which is 1.  Residual vectors of the
     * new seed are r/pi^seed (Eq. EQ-COLLINEAR); every other quantity is
     * rescaled to match. */
    if (a->seed_switch) {
      int best = -1;
      double bmin = 0.0;
      for (int k = 0; k < nz; ++k) {
        if (!active[k]) continue;
        double m = cabs(pi[k]);
        if (best < 0 || m < bmin) { best = k; bmin = m; }
      }
      if (best >= 0 && bmin < 1.0) {
        cplx c1 = pi[best], c0 = pi_old[best];
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < M; ++i) { r_new[i] /= c1; r[i] /= c0; }
        if (bicg) {
          cplx d1 = conj(c1), d0 = conj(c0);
#pragma omp parallel for schedule(static)
          for (int64_t i = 0; i < M; ++i) { rs_new[i] /= d1; rs[i] /= d0; }
        }
        if (method == ORC_CG_R || method == ORC_CG_C)
          rho_new /= c1 * conj(c1);
        else
          rho_new /= c1 * c1;
        nu_new /= creal(c1 * conj(c1));
        alpha *= c0 / c1;
        beta *= (c0 / c1) * (c0 / c1);
        for (int k = 0; k < nz; ++k) {
          if (!active[k]) continue;
          pi[k] /= c1;
          pi_old[k] /= c0;
        }
        zs = a->z[best];
        seed = best;
        a->nswitch++;
      }
    }
    if (a->hist_seed) a->hist_seed[n] = seed;

    /* Advance n -> n+1 */
    { cplx* tmp = r_old; r_old = r; r = r_new; r_new = tmp; }
    if (bicg) { cplx* tmp = rs_old; rs_old = rs; rs = rs_new; rs_new = tmp; }
    rho = rho_new;
    nu = nu_new;
    ba = beta / alpha;

    /* Residual of every shift from collinearity: ||r^k|| = ||r|| / |pi^k| */
    double maxres = 0.0;
    for (int k = 0; k < nz; ++k) {
      if (active[k]) a->res[k] = sqrt(nu) / (cabs(pi[k]) * bnorm);
      if (a->res[k] > maxres) maxres = a->res[k];
    }
    if (a->freeze_tol > 0.0)
      for (int k = 0; k < nz; ++k)
        if (active[k] && a->res[k] < a->freeze_tol) active[k] = 0;
    if (maxres < a->tol) { status = ORC_CONVERGED; n++; break; }
    if (nu == 0.0) { status = ORC_CONVERGED; n++; break; }
    if (cabs(rho) <= 16.0 * DBL_EPSILON * nu) { status = ORC_E_BREAKDOWN; n++; break; }
  }
  if (status == ORC_OK) status = ORC_E_MAXITER;

done:
  a->iters = n;
  a->status = status;
  a->seed = seed;
  free(r); free(r_old); free(r_new); free(q);
  free(rs); free(rs_old); free(rs_new); free(qs);
  free(pi); free(pi_old); free(active); free(u); free(p); free(Pr);
  return status;
}

/* ------------------------------------------------------------------------ */
/* Lanczos tridiagonalisation of Hermitian H on b (the continued-fraction
 * method the paper compares against, Sec. 2.3).  Produces a[0..n-1] and
 * bet[0..n-2] with T_n = tridiag(bet, a, bet); stops early (returns the
 * number of steps made) if the Krylov space is exhausted.  Plain three-term
 * recurrence, no reorthogonalisation. */
int orc_lanczos(const orc_op* op, int64_t M, const cplx* b, int nsteps,
                double* a_out, double* b_out) {
  cplx* v = malloc(sizeof(cplx) * M);
  cplx* v_prev = calloc((size_t)M, sizeof(cplx));
  cplx* w = malloc(sizeof(cplx) * M);
  double nb = sqrt(creal(dot_sesq(M, b, b)));
  int made = 0;
  if (nb == 0.0) goto out;
  for (int64_t i = 0; i < M; ++i) v[i] = b[i] / nb;
  double bprev = 0.0;
  for (int j = 0; j < nsteps; ++j) {
    if (orc_apply(op, v, w) != 0) break;
    for (int64_t i = 0; i < M; ++i) w[i] -= bprev * v_prev[i];
    double aj = creal(dot_sesq(M, v, w));
    for (int64_t i = 0; i < M; ++i) w[i] -= aj * v[i];
    a_out[j] = aj;
    made = j + 1;
    double bj = sqrt(creal(dot_sesq(M, w, w)));
    if (j + 1 < nsteps) b_out[j] = bj;
    if (bj == 0.0) break;
    for (int64_t i = 0; i < M; ++i) { v_prev[i] = v[i]; v[i] = w[i] / bj; }
    bprev = bj;
  }
out:
  free(v); free(v_prev); free(w);
  return made;
}
