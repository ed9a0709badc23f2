/*
 * komega_hip.h -- C interface of the MI355X shifted Krylov solver.
 *
 * Solves the shifted linear systems
 *     (z_k I - H) x^(k) = b,   k = 0 .. nz-1
 * for a real-symmetric or Hermitian sparse H with one Krylov sequence
 * (Kawamura et al., K-omega, Sec. 1 Eq. EQ-SHIFT-EQ and Sec. 2).  Each
 * iteration is one product q = H r (Sec. 3.2.1 i), the seed recurrences
 * (Sec. 2.2.1, Eqs. EQ-CG-RN-3REC, EQ-REC-ALPHA-N2, EQ-REC-BETA), the
 * collinear-residual recurrences of every shift (Sec. 2.2.2, Eqs.
 * EQ-SHIFTEDCG-PI .. EQ-SHIFTEDCG-p), optionally only the projection
 * y = P x (Sec. 2.2.3, Eqs. EQ-SHIFTEDCG-y/u), and seed switching
 * (Sec. 2.2.4).  The call sequence follows the paper's library flow (Sec. 3.2.1
 * iii, Algorithm 1): create/init, then {q = H r; update} until converged,
 * then finalize.  Besides that reverse-communication flow the library has
 * built-in operators (3D Anderson stencil, CSR, spin-1/2 Heisenberg) that run
 * the whole iteration on the GPU without returning to the caller.
 *
 * Conventions (all calls):
 *  - Every call returns a komega_status: 0 = OK, 1 = CONVERGED, < 0 = error.
 *    komega_last_error() gives a message for the last error of the calling
 *    thread.
 *  - Complex numbers are two doubles (re, im), interleaved ("complex128").
 *  - Vector arguments (b, P, x, r, q, v, ...) are DEVICE pointers on the
 *    current HIP device.  Vectors are complex128 except for method
 *    KOMEGA_CG_R, which uses real double vectors throughout, and the kept
 *    solutions of KOMEGA_F_X32.  With nrhs > 1 the right-hand sides are
 *    stored one after another ([nrhs][M]).
 *  - Batched solvers (komega_create_batched) hold nrhs independent systems
 *    of uneven sizes M_r: every vector is the concatenation of the systems'
 *    pieces (system r on rows off_r = M_0 + ... + M_{r-1}), P is [nl][ndim]
 *    with system r using its own column block, kept solutions are
 *    x[r][k][i] at offset nz*off_r + k*M_r + i, and y is [nrhs][nz][nl].
 *  - Operator construction arrays (eps, CSR arrays, bonds, couplings) and the
 *    shift list are HOST pointers; the library copies them.
 *  - All device work is enqueued on the stream given at creation (NULL = the
 *    default stream).  Only komega_getstate, komega_getresidual,
 *    komega_getcoef, komega_solve and komega_get_timing wait for the stream.
 *  - A solver or operator handle must not be used from two threads at once;
 *    distinct handles are independent.
 */
#ifndef KOMEGA_HIP_H
#define KOMEGA_HIP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t komega_status;

enum {
  KOMEGA_OK = 0,
  KOMEGA_CONVERGED = 1,
  KOMEGA_E_INVALID = -1,         /* bad argument or size                       */
  KOMEGA_E_BREAKDOWN = -2,       /* seed breakdown: rho ~ 0 or alpha denominator = 0 */
  KOMEGA_E_SHIFT_BREAKDOWN = -3, /* pi^k_{n+1} = 0 for an active shift          */
  KOMEGA_E_MAXITER = -4,         /* itermax iterations without convergence      */
  KOMEGA_E_HIP = -5,             /* HIP runtime error                           */
  KOMEGA_E_STATE = -6,           /* call out of order (e.g. update before init) */
  KOMEGA_E_NONFINITE = -7,       /* a scalar became Inf/NaN                      */
  KOMEGA_E_NOMEM = -8            /* device allocation failed                    */
};

/* Methods of Table 1: the type of A + sigma I decides the method. */
enum {
  KOMEGA_CG_R = 0, /* real symmetric H, real shifts, real vectors (shifted CG)    */
  KOMEGA_CG_C = 1, /* Hermitian H, real shifts, complex vectors (shifted CG)      */
  KOMEGA_COCG = 2, /* real symmetric H, complex shifts (shifted COCG, App. A)     */
  KOMEGA_BICG = 3  /* Hermitian H, complex shifts (shifted BiCG, App. B)          */
};

/* Flags */
enum {
  KOMEGA_F_NO_SWITCH = 1u, /* keep z[0] as seed for the whole solve           */
  KOMEGA_F_HISTORY = 2u,   /* record alpha_n, beta_n, seeds, P r_n (getcoef)  */
  KOMEGA_F_GRAPH = 4u,     /* komega_iterate replays a captured HIP graph of two
                              iterations (built-in operators, timing off)      */
  KOMEGA_F_X32 = 8u        /* whole-x mode (nl = 0, complex methods): keep x^(k)
                              and p^(k) as complex64 (two floats); every scalar,
                              residual vector, product and inner product stays
                              double, and each x, p update is done in double and
                              rounded to nearest on store                      */
};

#define KOMEGA_MAX_NL 8    /* largest number of projection rows               */

typedef struct komega_solver komega_solver;
typedef struct komega_op komega_op;

typedef struct {
  int32_t method;     /* KOMEGA_CG_R / CG_C / COCG / BICG                       */
  int32_t nz;         /* number of shifts, >= 1                                 */
  int64_t ndim;       /* M, the dimension of H, >= 1                            */
  int32_t nl;         /* 0: keep every x^(k) (P = I); 1..KOMEGA_MAX_NL: keep only
                         y^(k) = P x^(k) for an nl x M matrix P (Sec. 2.2.3)   */
  int32_t nrhs;       /* independent right-hand sides sharing H, >= 1          */
  int32_t itermax;    /* iteration limit, >= 1                                  */
  uint32_t flags;     /* KOMEGA_F_*                                              */
  double tol;         /* converged when max_k ||r^k|| / ||b|| < tol             */
  double freeze_tol;  /* shift k stops being updated (and leaves the seed choice)
                         once ||r^k||/||b|| < freeze_tol; < 0 selects 1e-3*tol,
                         0 never freezes                                        */
  void* stream;       /* hipStream_t, NULL = default stream                     */
} komega_params;

/* Per right-hand side progress, filled by komega_getstate / komega_solve. */
typedef struct {
  int32_t status;     /* KOMEGA_OK while running, else the final status         */
  int32_t iter;       /* iterations done                                        */
  int32_t seed;       /* index of the current seed shift                        */
  int32_t nswitch;    /* number of seed switches so far                         */
  double maxres;      /* max_k ||r^k|| / ||b|| after the last iteration          */
} komega_iter;

/* ---------------------------------------------------------------- solver -- */

/* Create a solver.  z: HOST array of nz complex shifts (2*nz doubles); the
 * first seed is z[0] (Sec. 2.1, A = z_0 I - H).  CG methods need real shifts.
 * Errors: E_INVALID for bad sizes, nl > KOMEGA_MAX_NL, complex shifts with a
 * CG method; E_NOMEM; E_HIP. */
komega_status komega_create(komega_solver** s, const komega_params* p, const double* z);

/* Create a solver for p->nrhs independent systems (z_k I - H_r) x_r^(k) = b_r
 * of uneven sizes rows[r] >= 1 (HOST array), all with the shifts z.  p->ndim
 * must equal the total rows.  Each system runs its own Krylov sequence, seed
 * and convergence test (a converged system stops while the others go on), and
 * all of them advance in the same launches: one work-group list covers every
 * (system, row group) pair.  A system's arithmetic, reduction order included,
 * is exactly that of a stand-alone solver of its size, so its results agree
 * bit for bit.  Operators: komega_op_stencil3d_batch with the same sizes, a
 * CSR operator of dimension ndim that couples no two systems (checked), or a
 * callback (called with nvec = 1 on the concatenated vector; it must not
 * couple systems).  Vector layouts: see the conventions above.
 * Errors as komega_create, plus E_INVALID if the rows do not add up to ndim. */
komega_status komega_create_batched(komega_solver** s, const komega_params* p, const double* z,
                                    const int64_t* rows);

/* Start a solve (Sec. 2.2.1: x_0 = 0, r_0 = p_0 = b; Eq. EQ-SHIFTEDCG-PI:
 * pi_0 = pi_{-1} = 1; Eq. EQ-SHIFTEDCG-u: y_0 = 0, u_0 = P b).
 *   b       [nrhs][M] right-hand sides (device).  Copied; b may be freed after.
 *   bshadow [nrhs][M] BiCG shadow start r~_0 (App. B: any vector not
 *           orthogonal to b); NULL selects conj(b).  Ignored by other methods.
 *   P       [nl][M] projection rows (device), required iff nl > 0; must stay
 *           valid until finalize.  y_l = sum_i P[l][i] x_i (no conjugation:
 *           pass conj(a) to obtain a^H x).
 *   x       output (device), must stay valid until finalize:
 *           nl = 0: x[rhs][k][i], the whole solutions ([nrhs][nz][M]);
 *           nl > 0: y[rhs][k][l] ([nrhs][nz][nl]).
 *           The library zeroes it here and updates it in every iteration.
 * May be called again to start a new solve with the same handle. */
komega_status komega_init(komega_solver* s, const void* b, const void* bshadow,
                          const void* P, void* x);

/* Reverse-communication update (Algorithm 1): the caller has computed
 * q = H r (and qs = H rs for BiCG) for its own vectors r, rs ([nrhs][M],
 * device), which must hold b (resp. the shadow start) before the first
 * update.  The call performs one iteration: seed coefficients, the three-term
 * update that overwrites r (and rs) in place with the next residual, the
 * shifted recurrences, the solution or projection update and the seed switch.
 * After a seed switch r holds the new seed's residual up to a scalar factor
 * that the library tracks; the caller only ever applies H to it.
 * st: HOST array of nrhs entries, or NULL.  With st the call waits for the
 * stream and returns CONVERGED once every right-hand side has stopped (or the
 * first error status); without st it returns OK and does not wait.
 * Right-hand sides that have stopped are left unchanged. */
komega_status komega_update(komega_solver* s, const void* q, void* r,
                            const void* qs, void* rs, komega_iter* st);

/* Enqueue n iterations with a built-in (or callback) operator, using the
 * solver's own residual buffers.  Asynchronous; stopped right-hand sides are
 * skipped on the device, so extra iterations after convergence change
 * nothing. */
komega_status komega_iterate(komega_solver* s, const komega_op* op, int32_t n);

/* Iterate until every right-hand side has converged, failed or reached
 * itermax, checking the device status every `poll` iterations (<= 0: 16).
 * In a batched solver (without KOMEGA_F_GRAPH), systems found stopped at a
 * check are left out of later product and seed launches; komega_init and
 * komega_restore_state restore them.  st: HOST array of nrhs entries or NULL.
 * Returns CONVERGED if all right-hand sides converged, else the first error
 * status. */
komega_status komega_solve(komega_solver* s, const komega_op* op, int32_t poll,
                           komega_iter* st);

/* Copy the progress of every right-hand side (HOST st[nrhs]); waits. */
komega_status komega_getstate(komega_solver* s, komega_iter* st);

/* Relative residual norms ||r^k||/||b|| = ||r|| / (|pi^k| ||b||) (Sec. 3.2.1
 * iii b, Eq. EQ-COLLINEAR) into HOST res[nrhs][nz]; waits. */
komega_status komega_getresidual(komega_solver* s, double* res);

/* Recorded seed coefficients of right-hand side `rhs` (needs
 * KOMEGA_F_HISTORY; Sec. 3.2.2 iv: alpha_n, beta_n and P r_n allow
 * recalculation at new shifts).  HOST outputs, each NULL or of capacity
 * itermax: alpha[n], beta[n] (complex), zseed[n] = the seed shift used in step
 * n (complex), seed[n] = seed index after step n, sw[2n..2n+1] = (c0, c1)
 * complex rescale factors of a switch after step n (1, 1 without switch),
 * Pr[n][l] = P r_{n+1} before the switch (complex, nl per step).
 * *n receives the number of recorded steps.  Waits. */
komega_status komega_getcoef(komega_solver* s, int32_t rhs, double* alpha, double* beta,
                             double* zseed, int32_t* seed, double* sw, double* Pr,
                             int32_t* n);

/* Recalculation at new shifts without operator products (Sec. 3.2.2 iv: the
 * recorded alpha_n, beta_n and P r_n determine the projected solution at any
 * shift).  Needs KOMEGA_F_HISTORY and nl > 0.  For right-hand side `rhs`,
 * replays every recorded step for the nzn HOST shifts znew (2*nzn doubles):
 * the pi recurrence with the recorded seed shift of each step, the y/u
 * updates with the recorded P r_{n+1}, the recorded seed-switch rescales and
 * the solve's freeze rule.  y: DEVICE output [nzn][nl] complex; res: HOST
 * [nzn] residual ||r^k||/||b|| reached at the last recorded step, or NULL.
 * A new shift whose residual is still large needs a longer recorded run.
 * Waits for the stream. */
komega_status komega_recalc(komega_solver* s, int32_t rhs, int32_t nzn, const double* znew,
                            void* y, double* res);

/* Restart (Sec. 3.2.1 iii a: "for restart calculations, the initial values
 * of the coefficients and the vector should be inputted").  A snapshot holds
 * every scalar, per-shift array, residual vector, the projected y (nl > 0) or
 * the search directions p (nl = 0; the caller keeps its own x) and the
 * history.  state_size gives the byte count; save copies it to HOST memory;
 * restore loads it into a solver created with the same parameters, with the
 * projection P and output x of komega_init (whole-x mode: x must hold the
 * saved solutions).  Continuing a restored solve reproduces the uninterrupted
 * one bit for bit.  All three wait for the stream. */
komega_status komega_state_size(komega_solver* s, int64_t* bytes);
komega_status komega_save_state(komega_solver* s, void* host, int64_t bytes);
komega_status komega_restore_state(komega_solver* s, const void* host, int64_t bytes,
                                   const void* P, void* x);

/* Release everything the solver owns (Sec. 3.2.1 iii c).  NULL is a no-op. */
komega_status komega_finalize(komega_solver* s);

/* -------------------------------------------------------------- operators -- */

/* 3D Anderson tight-binding cube with periodic edges: site i = x + Lx*(y + Ly*z),
 * H_ii = eps[i], H_ij = -hop for the 6 neighbours.  Edges must be >= 3.
 * eps: HOST array of Lx*Ly*Lz doubles. */
komega_status komega_op_stencil3d(komega_op** op, int32_t Lx, int32_t Ly, int32_t Lz,
                                  double hop, const double* eps);

/* nsys independent Anderson cubes as one block-diagonal operator: cube r
 * has edges L[3r], L[3r+1], L[3r+2] (each >= 3), the rows after those of
 * cubes 0..r-1, and the on-site energies eps[off_r ..] (HOST array of all
 * cubes' sites, concatenated); hopping -hop inside each cube as in
 * komega_op_stencil3d.  For batched solvers with the same cube sizes. */
komega_status komega_op_stencil3d_batch(komega_op** op, int32_t nsys, const int32_t* L, double hop,
                                        const double* eps);

/* General sparse H in CSR form (HOST arrays): rowptr[M+1] (int64), col[nnz]
 * (int32), val[nnz] complex (complex_vals = 1, 2*nnz doubles) or real
 * (complex_vals = 0).  H must be Hermitian (real symmetric for COCG / CG_R). */
komega_status komega_op_csr(komega_op** op, int64_t M, const int64_t* rowptr,
                            const int32_t* col, const double* val, int32_t complex_vals);

/* Spin-1/2 Heisenberg model H = sum_b J[b] S_{bi[b]} . S_{bj[b]} (Sec. 4.2,
 * Eq. eq:heisenberg with per-bond couplings) on the sector with nup up spins
 * of an L-site system, applied matrix-free.  Site j is bit j of the state,
 * up = 1; the basis is every L-bit integer with nup set bits, ascending
 * (enumerated on the GPU).  1 <= L <= 32, 0 <= nup <= L, 1 <= nb <= 256, bonds
 * distinct sites.  HOST arrays bi, bj, J. */
komega_status komega_op_heisenberg(komega_op** op, int32_t L, int32_t nup, int32_t nb,
                                   const int32_t* bi, const int32_t* bj, const double* J);

/* User operator: fn(user, v, Hv, nvec, stream) must enqueue Hv = H v for nvec
 * vectors of length M ([nvec][M], complex128, or double for CG_R) on `stream`
 * and return 0 on success. */
typedef int32_t (*komega_apply_fn)(void* user, const void* v, void* Hv, int32_t nvec,
                                   int32_t is_complex, void* stream);
komega_status komega_op_callback(komega_op** op, int64_t M, komega_apply_fn fn, void* user);

/* Dimension M of the operator. */
komega_status komega_op_dim(const komega_op* op, int64_t* M);

/* out = H v for nvec vectors ([nvec][M] device; complex128 if is_complex,
 * else double), enqueued on `stream`. */
komega_status komega_op_apply(const komega_op* op, const void* v, void* out, int32_t nvec,
                              int32_t is_complex, void* stream);

/* Heisenberg operators only: copy the basis (M uint32 states, ascending) to
 * the device array `states`. */
komega_status komega_op_heisenberg_states(const komega_op* op, uint32_t* states, void* stream);

/* Heisenberg operators only: position of each of n states (device uint32) in
 * the basis by the two-table index, into device int64 idx.  Every state must
 * have nup set bits and fit in L bits (checked: E_INVALID otherwise). */
komega_status komega_op_heisenberg_lookup(const komega_op* op, const uint32_t* states,
                                          int64_t* idx, int64_t n, void* stream);

/* Heisenberg operators only: out_s = [sum_j w_j (n_j(s) - 1/2)] v_s, the
 * excitation S^z(q) v with S^z(q) = sum_j e^{iqj} S^z_j (Sec. 4.2, Eq.
 * eq:dynamicalspin); w: HOST array of L complex phases; v, out: device
 * complex128 [M]. */
komega_status komega_op_heisenberg_szq(const komega_op* op, const double* w, const void* v,
                                       void* out, void* stream);

/* Heisenberg operators only: choose the product kernel.  0 = automatic
 * (default), 1 = one row per thread with gathers through the two-table
 * index, 2 = one basis group (common high half of the state) per work-group
 * with the group's vector segment staged in LDS.  E_INVALID if the variant
 * does not fit the operator (variant 2 needs the LDS to hold the rank table
 * and two segments). */
komega_status komega_op_set_variant(komega_op* op, int32_t variant);

/* Heisenberg operators only: bond contractions for the coupling gradient of
 * spectra.  For k < n: out[k*nb + b] = w_k^H (S_{bi[b]} . S_{bj[b]}) x_k
 * (complex), where w_k = w + k*ldw and x_k = x + k*ldx are device complex128
 * vectors of length M.  With x_k = G(z_k) b and w_k = G(conj z_k) a this is
 * dF_k/dJ_b of F_k = a^H G(z_k) b (G = (zI - H)^-1, dG = G dH G; H of
 * Sec. 4.2, Eq. eq:heisenberg, linear in the couplings).  out is device
 * memory (n*nb complex).  Deterministic; uses stream-ordered scratch. */
komega_status komega_op_heisenberg_bond_grad(const komega_op* op, const void* w, int64_t ldw,
                                             const void* x, int64_t ldx, int32_t n, void* out,
                                             void* stream);

/* out[k] = a_k^H x_k for k < n, device complex128 vectors of length M with
 * a_k = a + k*lda (lda = 0: the same a for every k) and x_k = x + k*ldx: the
 * projection G_ab = a^H x of Sec. 2.2.3 for kept solutions.  out is device
 * memory (n complex).  Deterministic; uses stream-ordered scratch. */
komega_status komega_dotc(const void* a, int64_t lda, const void* x, int64_t ldx, int64_t M, int32_t n,
                          void* out, void* stream);

/* Gradient of spectra with respect to on-site energies (the diagonal of H).
 * For F_k = a^H G(z_k) b, G = (zI - H)^-1, dG = G dH G and dH/deps_i = e_i e_i^T
 * give dF_k/deps_i = conj(w_k[i]) x_k[i] with x_k = G(z_k) b and
 * w_k = G(z_k)^H a = G(conj z_k) a (H Hermitian; both from one shifted solve
 * when a = b, Sec. 2.1).  This call forms the contraction a backward pass
 * needs: out[i] = sum_k g[k] w_k[i] conj(x_k[i]) = sum_k g[k] conj(dF_k/deps_i)
 * for i < M, whose real part is the gradient of a real loss with upstream
 * gradient g (PyTorch's convention).  g: device complex128 [n]; w_k = w + k*ldw
 * and x_k = x + k*ldx: device complex128 vectors of length M; out: device
 * complex128 [M].  Deterministic (fixed order over k); enqueued on `stream`. */
komega_status komega_onsite_grad(const void* g, const void* w, int64_t ldw, const void* x, int64_t ldx,
                                 int64_t M, int32_t n, void* out, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): komega_dotc
 * with the same arguments, results and kernels, but its partial sums live in
 * a static device array of the library (4 MiB per device, held until the
 * process ends) instead of stream-ordered scratch, and the call allocates
 * nothing.  n may not exceed KOMEGA_NOALLOC_MAX_VECTORS (KOMEGA_E_INVALID
 * otherwise).  Every call on one device shares that array: calls that may
 * overlap on one device (other streams, other threads) race and must be
 * ordered by the caller.  The first call on a device looks up the array's
 * device address, so make it outside graph capture. */
#define KOMEGA_NOALLOC_MAX_VECTORS 4096
komega_status komega_dotc_noalloc(const void* a, int64_t lda, const void* x, int64_t ldx, int64_t M, int32_t n,
                                  void* out, void* stream);

/* As komega_dotc for complex64 x (KOMEGA_F_X32 solutions): the products and
 * the sums are formed in double. */
komega_status komega_dotc_c64(const void* a, int64_t lda, const void* x, int64_t ldx, int64_t M, int32_t n,
                              void* out, void* stream);

/* Moment vectors of the contour-integral eigensolver (Sec. 4.1):
 * s[l][k][i] = sum_j w[k][j] x[l][j][i] for k < nk (1 <= nk <= 16), with x the
 * kept solutions [nrhs][nz][M] (device complex128), w HOST complex weights
 * [nk][nz] (trapezoid rule on the contour: w[k][j] = (z_j - gamma)^{k+1}/nz for
 * nodes z_j = gamma + rho e^{2 pi i (j + 1/2)/nz}) and s device complex128
 * [nrhs][nk][M].  Reads x once.  Waits for the stream. */
komega_status komega_contour_moments(const void* x, int32_t nz, int64_t M, int32_t nrhs,
                                     int32_t nk, const double* w, void* s, void* stream);

/* Release an operator.  NULL is a no-op. */
komega_status komega_op_destroy(komega_op* op);

/* ------------------------------------------------------------ diagnostics -- */

/* Kernel classes for timing. */
enum {
  KOMEGA_K_SPMV = 0,  /* operator product + inner product r.q + seed scalars     */
  KOMEGA_K_SEED = 1,  /* three-term seed update + inner products + shift scalars */
  KOMEGA_K_SHIFT = 2, /* whole-solution shift update x^k, p^k                     */
  KOMEGA_K_DOT = 3,   /* inner product r.q of the reverse-communication path      */
  KOMEGA_K_NCLASS = 4
};

/* Record HIP events around every launch of the kernel classes in `mask`
 * (bit c = class c), on the solver's stream; 0 turns recording off. */
komega_status komega_set_timing(komega_solver* s, uint32_t mask);

/* Total device time (ms) and launch count of class `cls` since the last
 * reset (reset = 1 clears after reading).  Waits for the stream. */
komega_status komega_get_timing(komega_solver* s, int32_t cls, double* ms, int64_t* count,
                                int32_t reset);

/* Grid size (work-groups per right-hand side; for a batched solver, of the
 * whole launch, which shrinks as stopped systems leave it) used by class
 * `cls` for this solver and operator; lets callers count launches and bytes. */
komega_status komega_launch_info(const komega_solver* s, const komega_op* op, int32_t cls,
                                 int64_t* blocks, int64_t* threads);

/* Bandwidth probe (diagnostic; no counterpart in the paper).  Streams
 * `bytes` (a multiple of 16, >= 16) of device memory with the access pattern
 * of the whole-x update: 16-byte nontemporal loads (and stores), grid-stride
 * over komega_stream_probe_groups() work-groups.  kind 0 copies src to dst
 * (both `bytes` long, not overlapping); kind 1 only reads src and writes one
 * 16-byte partial sum per work-group to dst (komega_stream_probe_groups() x
 * 16 bytes).  Device pointers, enqueued on `stream`; time it with events to
 * obtain the bandwidth the HBM sustains for such streams. */
komega_status komega_stream_probe(const void* src, void* dst, int64_t bytes, int32_t kind, void* stream);
int32_t komega_stream_probe_groups(void);

/* Launch configuration of the whole-x update (results do not depend on it:
 * every element is computed by the same arithmetic).  Knobs:
 *   KOMEGA_T_SHIFT_BLOCK  shifts handled per thread: 1, 2 (default), 4, 8, 16
 *   KOMEGA_T_SHIFT_NT     1 (default): stream x^k, p^k with nontemporal loads
 *                         and stores; 0: ordinary cached accesses
 *   KOMEGA_T_SPMV_BLOCKS  work-groups of the built-in operator product per
 *                         right-hand side, 1..2048, 0 = automatic (default);
 *                         ignored by batched solvers.  The inner product r.Hr
 *                         is summed over these groups, so unlike the other
 *                         knobs this one changes rounding (not accuracy)
 *   KOMEGA_T_SHIFT_ORDER  whole-x update grid order: 0 (default) row tiles
 *                         fastest, 1 shift blocks fastest (the blocks of one
 *                         row tile, which share r_{n+1}, run together)
 *   KOMEGA_T_SHIFT_STEPS  steps of Eqs. EQ-SHIFTEDCG-x/p composed per block
 *                         before x^k, p^k are read and written, 1..32 (default
 *                         32; 16 with KOMEGA_F_X32): x^k <- x^k + E p^k +
 *                         sum_t F_t r_t and
 *                         p^k <- G p^k + sum_t H_t r_t with the scalars of the
 *                         block's steps, so x^k, p^k stream once per block.
 *                         1 applies every step at once.  Changes rounding (not
 *                         accuracy); the x^k in the caller's buffer are current
 *                         whenever komega_iterate / komega_solve return.  Graph
 *                         replay (KOMEGA_F_GRAPH) and reverse communication
 *                         apply every step at once.  E_STATE while a block is
 *                         pending (never between calls).
 * An autotuner can time the candidates with komega_set_timing and choose per
 * problem size.  Changing a knob discards captured graphs. */
enum {
  KOMEGA_T_SHIFT_BLOCK = 0,
  KOMEGA_T_SHIFT_NT = 1,
  KOMEGA_T_SPMV_BLOCKS = 2,
  KOMEGA_T_SHIFT_ORDER = 3,
  KOMEGA_T_SHIFT_STEPS = 4
};
komega_status komega_set_tuning(komega_solver* s, int32_t knob, int32_t value);
komega_status komega_get_tuning(const komega_solver* s, int32_t knob, int32_t* value);

const char* komega_strerror(komega_status code);
const char* komega_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* KOMEGA_HIP_H */
