// komega_internal.h -- device state, complex helpers and launch interface
// shared by the HIP kernels (komega_kernels.hip) and the C interface
// (komega_capi.hip).  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/komega_hip.h"

namespace kw {

// ------------------------------------------------------------------ complex
// Complex double as double2 (x = re, y = im): 16-byte aligned, so vector
// elements move with one dwordx4 load/store.
typedef double2 zc;

__host__ __device__ inline zc zmk(double re, double im) { zc a; a.x = re; a.y = im; return a; }
__host__ __device__ inline zc zadd(zc a, zc b) { return zmk(a.x + b.x, a.y + b.y); }
__host__ __device__ inline zc zsub(zc a, zc b) { return zmk(a.x - b.x, a.y - b.y); }
__host__ __device__ inline zc zneg(zc a) { return zmk(-a.x, -a.y); }
__host__ __device__ inline zc zconj(zc a) { return zmk(a.x, -a.y); }
__host__ __device__ inline zc zmul(zc a, zc b) { return zmk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__host__ __device__ inline zc zscale(double s, zc a) { return zmk(s * a.x, s * a.y); }
__host__ __device__ inline double zabs2(zc a) { return a.x * a.x + a.y * a.y; }
__host__ __device__ inline bool zfinite(zc a) { return isfinite(a.x) && isfinite(a.y); }
__host__ __device__ inline bool zzero(zc a) { return a.x == 0.0 && a.y == 0.0; }
// a / b by Smith's algorithm (no overflow of |b|^2 for large |b|).
__host__ __device__ inline zc zdiv(zc a, zc b) {
  if (fabs(b.x) >= fabs(b.y)) {
    double r = b.y / b.x, d = b.x + b.y * r;
    return zmk((a.x + a.y * r) / d, (a.y - a.x * r) / d);
  }
  double r = b.x / b.y, d = b.y + b.x * r;
  return zmk((a.x * r + a.y) / d, (a.y * r - a.x) / d);
}
__host__ __device__ inline zc zinv(zc b) { return zdiv(zmk(1.0, 0.0), b); }

// Complex float: storage of x^k, p^k in the complex64 whole-x mode.  All
// arithmetic on them is done in double; values are rounded to nearest on
// store.
typedef float2 cf;
__host__ __device__ inline zc widen(cf a) { return zmk((double)a.x, (double)a.y); }
__host__ __device__ inline cf narrow(zc a) { cf r; r.x = (float)a.x; r.y = (float)a.y; return r; }

// ------------------------------------------------- vector element traits
// V = zc for complex vectors, double for the real-vector CG method.  The
// scalar coefficients are always complex; with real vectors they are real
// by construction (real shifts, real H, real b) and only .x is used.
template <class V> struct VT;
template <> struct VT<zc> {
  static __device__ inline zc lin(zc c, zc v) { return zmul(c, v); }
  static __device__ inline zc rs(double c, zc v) { return zscale(c, v); }
  static __device__ inline zc add(zc a, zc b) { return zadd(a, b); }
  static __device__ inline zc bil(zc a, zc b) { return zmul(a, b); }           // a b
  static __device__ inline zc ses(zc a, zc b) { return zmul(zconj(a), b); }    // conj(a) b
  static __device__ inline double nrm(zc a) { return zabs2(a); }
  static __device__ inline zc conj(zc a) { return zconj(a); }
  static __device__ inline zc zero() { return zmk(0.0, 0.0); }
  static __device__ inline zc of(double re) { return zmk(re, 0.0); }
};
template <> struct VT<double> {
  static __device__ inline double lin(zc c, double v) { return c.x * v; }
  static __device__ inline double rs(double c, double v) { return c * v; }
  static __device__ inline double add(double a, double b) { return a + b; }
  static __device__ inline zc bil(double a, double b) { return zmk(a * b, 0.0); }
  static __device__ inline zc ses(double a, double b) { return zmk(a * b, 0.0); }
  static __device__ inline double nrm(double a) { return a * a; }
  static __device__ inline double conj(double a) { return a; }
  static __device__ inline double zero() { return 0.0; }
  static __device__ inline double of(double re) { return re; }
};

// ------------------------------------------------------------ solver state
// One record per right-hand side, in device memory.  "Memory scale": the
// residual vectors in memory are R_mem with true r_n = sc * R_mem and true
// r_{n-1} = so * RO_mem.  A seed switch divides the true residuals by pi of
// the new seed (Eq. EQ-COLLINEAR); the library folds that division into sc/so
// instead of rescaling the vectors.
struct alignas(16) RhsState {
  zc rho;     // rho_n of the current seed (true vectors)
  zc ba;      // beta_{n-1} / alpha_{n-1}   (0 at n = 0)
  zc zs;      // current seed shift
  zc sc, so;  // memory scales of r_n and r_{n-1}
  zc alpha;   // alpha_n   (set by the SpMV-side finalisation)
  zc gamma;   // alpha_n beta_{n-1} / alpha_{n-1}
  zc cr, cq, co;  // r_{n+1} = cr R + cq Q + co RO (memory vectors)
  double nu;      // ||r_n||^2
  double bnorm;   // ||b||
  double maxres;  // max_k ||r^k|| / ||b||
  double pad0;
  int32_t seed, iter, status, stop;
  int32_t nswitch;
  int32_t pending;       // whole-x coefficients ak/bk/ck of the last step await k_shift
  int32_t step_pending;  // k_seed has run; its shift step has not been finalised yet
  int32_t blk_cnt;       // whole-x steps accumulated in the current block (blocked update)
  uint32_t blk_gen;      // block generation those steps belong to
};

// Everything the kernels need, passed by value.
struct DevSolver {
  int32_t method, nz, nl, nrhs;
  int64_t M;
  int32_t itermax;
  uint32_t flags;
  double tol, freeze_tol;
  int32_t maxblk;     // partial-sum slots per right-hand side
  int32_t nblkB;      // uniform layout: work-groups per system of init / seed (sys_blocks)
  int32_t hist_cap;
  const zc* z;        // [nz]
  RhsState* st;       // [nrhs]
  zc* pi;             // [nrhs][nz]  pi_n
  zc* pio;            // [nrhs][nz]  pi_{n-1}
  int32_t* active;    // [nrhs][nz]
  double* res;        // [nrhs][nz]
  zc* ak;             // [nrhs][nz]  alpha^k_n        (whole-x mode)
  zc* bk;             // [nrhs][nz]  beta^k_n
  zc* ck;             // [nrhs][nz]  1 / pi^k_{n+1}
  int32_t* apply;     // [nrhs][nz]  shift updated in the last step
  zc* u;              // [nrhs][nz][nl]
  zc* y;              // [nrhs][nz][nl]  caller's projected output
  const void* P;      // [nl][M]  (V elements)
  zc* partA;          // [nrhs][maxblk]          partial r.q of k_spmv / k_dot
  zc* partB;          // [nrhs][maxblk][2 + NL]  partial rho, nu, P r of k_seed / init
  // history (KOMEGA_F_HISTORY), capacity hist_cap steps per right-hand side
  zc* h_alpha;        // [nrhs][cap]
  zc* h_beta;
  zc* h_zs;
  zc* h_sw;           // [nrhs][cap][2]
  int32_t* h_seed;    // [nrhs][cap]
  zc* h_pr;           // [nrhs][cap][nl]
  double* h_nu;       // [nrhs][cap]  ||r_{n+1}||^2 of the seed after the step
  zc* pb;             // [nrhs][nl]   P b (u_0)
  // Batched systems of uneven size.  soff == nullptr: nrhs right-hand sides
  // of M rows each, stored one after another (system r at rows r*M) and
  // launched on (groups, nrhs) grids.  Otherwise system r occupies rows
  // [soff[r], soff[r+1]) of every vector (M is then the total), and each
  // launch is a 1-D grid over a work list of (system, work-group) pairs.
  const int64_t* soff;  // [nrhs+1]
  const int2* wl_a;     // k_spmv / k_dot: (system, group); group -1 finalises
  const int2* wl_b;     // k_seed / k_init / k_init_copy: (system, group)
  const int2* wl_t;     // k_shift: (system, row tile of TPB rows)
  int32_t nwl_a, nwl_b, nwl_t;
  int32_t x32;          // whole-x mode keeps x^k, p^k as complex64
  int32_t shift_block;  // shifts per thread of k_shift (1, 2, 4, 8 or 16)
  int32_t shift_nt;     // k_shift streams x, p with nontemporal loads/stores
  int32_t spmv_blk;     // product work-groups per right-hand side (0: automatic)
  int32_t shift_order;  // k_shift grid: 0 row tiles fastest, 1 shift blocks fastest
  // Blocked whole-x update: xblk > 1 steps of Eqs. EQ-SHIFTEDCG-x/p are
  // composed into one linear map per shift before x^k, p^k are touched:
  // after t steps x = x0 + E p0 + sum_s F_s r_s, p = G p0 + sum_s H_s r_s
  // (r_s the seed residual memory vectors of those steps).  xblk <= 1: the
  // per-step update (k_shift).
  int32_t xblk;
  uint32_t blk_gen;     // current block generation (the host bumps it after each application)
  zc* bcoef;            // [nrhs][nz][2 + 2 XBLK_MAX]  E, G, F_0.., H_0..
  int32_t* btouch;      // [nrhs][nz]  shift updated in the current block
  zc* bstep;            // [nrhs][XBLK_MAX][3][nz]  alpha^k, beta^k, 1/pi^k of each step of the block
};

// Operator description passed to kernels.
enum OpKind { OP_STENCIL = 1, OP_CSR = 2, OP_HEIS = 3, OP_CALLBACK = 4 };

struct DevOp {
  int32_t kind;
  int64_t M;
  // stencil
  int32_t Lx, Ly, Lz;
  double hop;
  const double* eps;
  // csr
  const int64_t* rowptr;
  const int32_t* col;
  const void* val;
  int32_t complex_vals;
  // heisenberg
  int32_t L, nup, nb, h;       // h = number of low bits in the index split
  const uint32_t* states;      // [M]
  const uint32_t* hi_off;      // [2^(L-h)]
  const uint16_t* lo_rank;     // [2^h]  rank of l among h-bit values of its popcount
  const uint16_t* lo_state;    // [2^h]  inverse: lo_state[lo_koff[k] + j] = j-th value of popcount k
  const uint32_t* lo_koff;     // [h+2]  lo_koff[k] = number of h-bit values of popcount < k
  const uint32_t* bmask;       // [nb]  (1<<i)|(1<<j)
  const double* bJ;            // [nb]  J_b
  double jq;                   // sum_b J_b / 4 (the diagonal of a state with every bond parallel)
  int32_t tables_in_lds;
  // Bonds split by where their two sites fall relative to the index split:
  // low (both < h), high (both >= h), cross (one each side).
  int32_t nlo, nhb, ncr;
  const uint32_t* lo_m;        // [nlo] mask within the low h bits
  const double* lo_J;
  const uint32_t* hb_m;        // [nhb] mask within the high L-h bits
  const double* hb_J;
  const int32_t* cr_a;         // [ncr] low-side bit position
  const int32_t* cr_c;         // [ncr] high-side bit position (within the high bits)
  const double* cr_J;
  // the three lists again for the row product, each padded with null bonds to
  // whole chunks (HEIS_CH_*), one after another: masks (cross bonds as full
  // state masks) and halved couplings, read by the product as wave-uniform
  // scalar loads
  const uint32_t* rl_m;
  const double* rl_j;
  int32_t ngroups;             // 2^(L-h) high parts; hi_off has ngroups+1 entries
  int32_t segmax;              // largest group size C(h, floor(h/2)) (or smaller)
  int32_t group_kernel;        // 1: use the group-at-a-time product (segment in LDS)
  int32_t row_groups;          // default work-groups of the row product: one resident round
  const uint32_t* tile_order;  // [ceil(M / TPB)] order in which the row product takes its tiles
  // batched stencil: nsys independent cubes, block-diagonal, cube r on rows
  // [soff[r], soff[r+1]) with edges sysL[3r..3r+2]; eps concatenated
  int32_t nsys;
  const int32_t* sysL;         // [nsys][3]
  const int64_t* soff;         // [nsys+1]
  const int2* wl;              // (cube, group) work list of a stand-alone apply
  int32_t nwl;
};

constexpr int TPB = 256;            // threads per block of the streaming kernels
constexpr int HEIS_CH_LO = 12;      // bonds per chunk of the row product, low list
constexpr int HEIS_CH_HI = 12;      // high list
constexpr int HEIS_CH_CR = 2;       // cross list (short on chains: two bonds on a ring)
__host__ __device__ inline int heis_pad(int n, int ch) { return (n + ch - 1) / ch * ch; }
constexpr int MAXBLK = 2048;        // partial-sum slots per right-hand side
constexpr int SHIFT_BLOCK = 2;      // default shifts per thread in the whole-x update
constexpr int XBLK_MAX = 32;        // most steps composed by the blocked whole-x update
// steps composed per block unless tuned: with complex64 x, p the kept
// residuals are a larger share of the bytes and 16 steps measured faster
constexpr int XBLK_DEFAULT = 32;
constexpr int XBLK_DEFAULT_X32 = 16;
constexpr int XBLK_SHIFTS = 16;     // granule of the blocked update's shift split over work-groups
__host__ __device__ inline int bcoef_len() { return 2 + 2 * XBLK_MAX; }
// scalar q (0: alpha^k, 1: beta^k, 2: 1/pi^k_{n+1}) of step t of the block, shift k
__host__ __device__ inline size_t bstep_at(int nz, int rhs, int t, int q, int k) {
  return (((size_t)rhs * XBLK_MAX + t) * 3 + q) * nz + k;
}
constexpr int HEIS_CHUNK = 8;       // bonds whose gathers are issued together

// ----------------------------------------------------------- launchers
// All return hipError_t; they validate nothing (the C interface does).
struct Buffers {
  void* R; void* Q; void* RO;      // seed residual r_n, q = H r_n, r_{n-1}
  void* Rs; void* Qs; void* ROs;   // BiCG shadow counterparts (or null)
  void* p;                         // [nrhs][nz][M] search directions (whole x)
  void* x;                         // [nrhs][nz][M] caller output (whole x)
  void* RN;                        // when set, k_seed writes r_{n+1} here (ring of residuals)
};

// Work-group counts: k_spmv / k_dot use 1 + nblkA groups (group 0 finalises
// the previous step), k_seed uses nblkB groups; each writes one partial-sum
// slot per row group.
hipError_t launch_init(const DevSolver& ds, const Buffers& bf, const void* b,
                       const void* bshadow, void* x, hipStream_t st);
hipError_t launch_spmv(const DevSolver& ds, const DevOp& op, const Buffers& bf, bool with_dot,
                       int64_t nblkA, hipStream_t st);
hipError_t launch_dot(const DevSolver& ds, const void* dual, const void* q, int64_t nblkA,
                      hipStream_t st);
hipError_t launch_seed(const DevSolver& ds, const Buffers& bf, bool inplace, int64_t nblkA,
                       int64_t nblkB, hipStream_t st);
hipError_t launch_finalize(const DevSolver& ds, int64_t nblkB, hipStream_t st);
hipError_t launch_shift(const DevSolver& ds, const Buffers& bf, hipStream_t st);
// Applies the accumulated block: steps t < blk_cnt use the residual memory
// vector in ring slot (slot0 + t) % nb (slots of vr elements each).
hipError_t launch_shift_blk(const DevSolver& ds, const void* ring, int64_t vr, int slot0, int nb, void* x, void* p,
                            hipStream_t st);
hipError_t launch_op_apply(const DevOp& op, const void* v, void* out, int32_t nvec,
                           int32_t is_complex, hipStream_t st);
hipError_t launch_heis_setup(DevOp& op, const int64_t* binom_dev, hipStream_t st);
hipError_t launch_heis_hi(DevOp& op, const int64_t* binom_dev, int64_t* total, hipStream_t st);
hipError_t launch_heis_lookup(const DevOp& op, const uint32_t* states, int64_t* idx, int64_t n,
                              int32_t* bad, hipStream_t st);
hipError_t launch_heis_szq(const DevOp& op, const zc* w, const void* v, void* out,
                           hipStream_t st);
hipError_t launch_heis_check(const DevOp& op, int32_t* bad, hipStream_t st);

hipError_t launch_recalc(const DevSolver& ds, int rhs, int nsteps, const zc* znew, int nzn, zc* y, double* res,
                         hipStream_t st);
hipError_t launch_moments(const void* x, int nz, int64_t M, int nrhs, int nk, const void* w, void* s,
                          hipStream_t st);
hipError_t launch_bond_grad(const DevOp& op, const void* w, int64_t ldw, const void* x, int64_t ldx, int32_t nvec,
                            double* part, int G, void* out, hipStream_t st);
hipError_t launch_onsite_grad(const void* g, const void* w, int64_t ldw, const void* x, int64_t ldx, int64_t M,
                              int32_t n, void* out, hipStream_t st);
hipError_t launch_stream_probe(const void* src, void* dst, int64_t n, int32_t kind, hipStream_t st);
int32_t stream_probe_groups();
hipError_t launch_dotc(const void* a, int64_t lda, const void* x, int64_t ldx, int64_t M, int32_t n, double* part,
                       int G, void* out, int x32, hipStream_t st);

int64_t spmv_blocks(const DevOp& op, int64_t M);
int heis_row_groups(const DevOp& op);
int64_t csr_mr_groups(int64_t M, int nrhs);
size_t heis_grp_lds_bytes(const DevOp& op, bool shadow);

// Work-groups (and partial-sum slots) of the streaming kernels for M rows.
// Host and device use the same count, so a batched system reduces its slots
// exactly as a stand-alone solve of the same size does.
__host__ __device__ inline int64_t stream_blocks(int64_t M) {
  int64_t b = (M + TPB - 1) / TPB;
  if (b > MAXBLK) b = MAXBLK;
  return b < 1 ? 1 : b;
}

// Work-groups per system of the streaming kernels (init, seed) and of the
// default product in the uniform layout of nsys systems: stream_blocks, but
// at most about 4096 over all systems of a launch.  Every seed work-group
// first sums all of its system's product partial sums, so the work-group
// count multiplies that prologue; past a few thousand work-groups more of
// them stream no faster.
__host__ __device__ inline int64_t sys_blocks(int64_t M, int nsys) {
  const int64_t b = stream_blocks(M);
  int64_t cap = nsys > 1 ? (4096 + nsys - 1) / nsys : MAXBLK;
  if (cap < 64) cap = 64;
  return b < cap ? b : cap;
}

}  // namespace kw
