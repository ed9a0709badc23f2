// komega_capi.hip -- the C interface of include/komega_hip.h: handles, device
// buffers, the host side of the iteration loop, operators, diagnostics.
// Every call validates its arguments on the host before any kernel is
// launched, so kernels never see sizes they were not written for.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>

#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "komega_internal.h"

using namespace kw;

// ----------------------------------------------------------------- errors
static thread_local std::string g_err;

static komega_status set_err(komega_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIPCHK(call)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      return set_err(KOMEGA_E_HIP, "%s failed: %s", #call, hipGetErrorString(e_));       \
  } while (0)

template <class T>
static komega_status dalloc(T** p, size_t count, std::vector<void*>& owned) {
  *p = nullptr;
  if (count == 0) return KOMEGA_OK;
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, count * sizeof(T));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return set_err(KOMEGA_E_NOMEM, "device allocation of %zu bytes failed: %s", count * sizeof(T),
                   hipGetErrorString(e));
  }
  owned.push_back(q);
  *p = reinterpret_cast<T*>(q);
  return KOMEGA_OK;
}

#define TRY(x)                           \
  do {                                   \
    komega_status s_ = (x);              \
    if (s_ != KOMEGA_OK) return s_;      \
  } while (0)

// ---------------------------------------------------------------- handles
struct komega_op {
  DevOp d{};
  int version = 0;  // bumped whenever d changes (cached graphs become stale)
  std::vector<int64_t> h_soff;    // batched stencil: first row of every cube
  std::vector<int64_t> h_rowptr;  // CSR: host copy for the block-diagonal check
  std::vector<int32_t> h_col;
  std::vector<void*> owned;
  komega_apply_fn fn = nullptr;
  void* user = nullptr;
  ~komega_op() {
    for (void* p : owned) (void)hipFree(p);
  }
};

struct komega_solver {
  komega_params p{};
  DevSolver ds{};
  hipStream_t stream = nullptr;
  Buffers bf{};
  std::vector<void*> owned;
  RhsState* h_state = nullptr;  // pinned mirror of ds.st
  int initialized = 0;
  int mode = 0;                 // 0 none yet, 1 reverse communication, 2 built-in loop
  size_t es = 16;               // bytes per vector element
  size_t xes = 16;              // bytes per element of x^k, p^k
  bool batched = false;         // systems of uneven size (komega_create_batched)
  std::vector<int64_t> h_soff;  // batched: first row of every system, and the total
  // batched: the full product / seed work lists, and the systems currently
  // left out of them (stopped, see retire_stopped)
  std::vector<int2> wla_full, wlb_full;
  std::vector<char> retired;
  int nretired = 0;
  int64_t vrows = 0;            // rows of each residual-sized buffer
  const komega_op* csr_checked = nullptr;  // CSR operator found block diagonal
  int csr_checked_version = -1;
  // timing
  uint32_t tmask = 0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[KOMEGA_K_NCLASS];
  std::vector<hipEvent_t> pool;
  double acc_ms[KOMEGA_K_NCLASS] = {0, 0, 0, 0};
  int64_t acc_n[KOMEGA_K_NCLASS] = {0, 0, 0, 0};
  // Whole-x mode keeps the seed residuals in a ring of XBLK_MAX + 2 slots:
  // iteration `it` of the built-in loop reads r_it (slot it), r_{it-1} and
  // writes r_{it+1} (slot it+1), so the residuals of a block of composed
  // steps stay available until the block is applied.
  void* ring = nullptr;
  int64_t it = 0;                  // built-in-loop iterations since init
  bool step_pending_host = false;  // a seed update ran and its step is not finalised yet
  int blk_steps = 0;               // steps composed into the current block
  int blk_slot0 = 0;               // ring slot of the residual of the block's first step
  // captured two-iteration graphs (KOMEGA_F_GRAPH), keyed by operator,
  // operator version and buffer parity
  hipStream_t cap_stream = nullptr;
  struct GraphEntry {
    const komega_op* op;
    int version;
    void* R;  // buffer holding r_n when the graph starts
    hipGraphExec_t exec;
  };
  std::vector<GraphEntry> graphs;
  void drop_graphs() {
    for (auto& g : graphs) (void)hipGraphExecDestroy(g.exec);
    graphs.clear();
  }
  ~komega_solver() {
    drop_graphs();
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    for (auto& v : ev)
      for (auto& pr : v) { (void)hipEventDestroy(pr.first); (void)hipEventDestroy(pr.second); }
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    for (void* q : owned) (void)hipFree(q);
    if (h_state) (void)hipHostFree(h_state);
  }
};

// Records an event pair around the launches of one kernel class when the
// class is selected for timing.
struct Timed {
  komega_solver* s;
  int cls;
  hipEvent_t a = nullptr, b = nullptr;
  Timed(komega_solver* s_, int cls_) : s(s_), cls(cls_) {
    if (!(s->tmask & (1u << cls))) return;
    a = take();
    b = take();
    if (a && b) (void)hipEventRecord(a, s->stream);
  }
  hipEvent_t take() {
    if (!s->pool.empty()) {
      hipEvent_t e = s->pool.back();
      s->pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  ~Timed() {
    if (a && b) {
      (void)hipEventRecord(b, s->stream);
      s->ev[cls].emplace_back(a, b);
    } else {
      if (a) s->pool.push_back(a);
      if (b) s->pool.push_back(b);
    }
  }
};

static bool is_cg(int m) { return m == KOMEGA_CG_R || m == KOMEGA_CG_C; }

constexpr int RING = XBLK_MAX + 2;
static void* ring_slot(const komega_solver* s, int64_t j) {
  const int64_t m = ((j % RING) + RING) % RING;
  return reinterpret_cast<unsigned char*>(s->ring) + (size_t)m * (size_t)s->vrows * s->es;
}
static void ring_point(komega_solver* s) {
  s->bf.R = ring_slot(s, s->it);
  s->bf.RO = ring_slot(s, s->it - 1);
}
// The blocked whole-x update applies (the built-in loop, not graph replay).
static bool blocked(const komega_solver* s) {
  return s->p.nl == 0 && s->ds.xblk > 1 && !(s->p.flags & KOMEGA_F_GRAPH);
}

// ------------------------------------------------------------------ solver
static int64_t host_stream_blocks(int64_t M) { return stream_blocks(M); }

// Shared by komega_create and komega_create_batched; rows == nullptr is the
// uniform layout.
static komega_status create_solver(komega_solver** out, const komega_params* p, const double* z,
                                   const int64_t* rows) {
  if (!out || !p || !z) return set_err(KOMEGA_E_INVALID, "null argument");
  *out = nullptr;
  if (p->method < KOMEGA_CG_R || p->method > KOMEGA_BICG)
    return set_err(KOMEGA_E_INVALID, "unknown method %d", p->method);
  if (p->nz < 1 || p->ndim < 1 || p->nrhs < 1 || p->itermax < 1)
    return set_err(KOMEGA_E_INVALID, "nz, ndim, nrhs and itermax must be >= 1");
  if (p->nl < 0 || p->nl > KOMEGA_MAX_NL)
    return set_err(KOMEGA_E_INVALID, "nl must be in [0, %d]", KOMEGA_MAX_NL);
  if (p->nrhs > 65535) return set_err(KOMEGA_E_INVALID, "nrhs must be <= 65535");
  if (!(p->tol >= 0.0)) return set_err(KOMEGA_E_INVALID, "tol must be >= 0");
  const bool x32 = (p->flags & KOMEGA_F_X32) != 0;
  if (x32 && (p->nl != 0 || p->method == KOMEGA_CG_R))
    return set_err(KOMEGA_E_INVALID, "KOMEGA_F_X32 needs whole-x mode (nl = 0) and complex vectors");
  for (int k = 0; k < p->nz; ++k) {
    if (!std::isfinite(z[2 * k]) || !std::isfinite(z[2 * k + 1]))
      return set_err(KOMEGA_E_INVALID, "shift %d is not finite", k);
    if (is_cg(p->method) && z[2 * k + 1] != 0.0)
      return set_err(KOMEGA_E_INVALID, "shifted CG needs real shifts (shift %d is complex)", k);
  }
  std::vector<int64_t> soff;
  std::vector<int2> wla, wlb, wlt;
  if (rows) {
    soff.resize((size_t)p->nrhs + 1);
    soff[0] = 0;
    for (int r = 0; r < p->nrhs; ++r) {
      if (rows[r] < 1) return set_err(KOMEGA_E_INVALID, "system %d has %lld rows", r, (long long)rows[r]);
      soff[r + 1] = soff[r] + rows[r];
    }
    if (soff[p->nrhs] != p->ndim)
      return set_err(KOMEGA_E_INVALID, "ndim %lld != total rows %lld of the systems", (long long)p->ndim,
                     (long long)soff[p->nrhs]);
    // work lists: finalisers first (they are on the critical path), then the
    // row groups of every system in system order
    for (int r = 0; r < p->nrhs; ++r) wla.push_back(make_int2(r, -1));
    for (int r = 0; r < p->nrhs; ++r) {
      const int64_t M = soff[r + 1] - soff[r];
      const int nb = (int)host_stream_blocks(M);
      for (int g = 0; g < nb; ++g) {
        wla.push_back(make_int2(r, g));
        wlb.push_back(make_int2(r, g));
      }
      const int64_t nt = (M + TPB - 1) / TPB;
      for (int64_t t = 0; t < nt; ++t) wlt.push_back(make_int2(r, (int)t));
    }
    if (wla.size() > 0x7fffffff / 2 || wlt.size() > 0x7fffffff / 2)
      return set_err(KOMEGA_E_INVALID, "too many systems or rows for one launch");
  }
  komega_solver* s = new (std::nothrow) komega_solver();
  if (!s) return set_err(KOMEGA_E_NOMEM, "host allocation failed");
  s->p = *p;
  s->stream = reinterpret_cast<hipStream_t>(p->stream);
  s->es = (p->method == KOMEGA_CG_R) ? 8 : 16;
  s->xes = x32 ? 8 : s->es;
  s->batched = rows != nullptr;
  s->h_soff = soff;
  const size_t nr = (size_t)p->nrhs, nz = (size_t)p->nz, nl = (size_t)p->nl;
  // rows of each residual-sized buffer: the systems are concatenated
  const size_t VR = rows ? (size_t)p->ndim : nr * (size_t)p->ndim;
  s->vrows = (int64_t)VR;
  DevSolver& d = s->ds;
  d.method = p->method;
  d.nz = p->nz;
  d.nl = p->nl;
  d.nrhs = p->nrhs;
  d.M = p->ndim;
  d.itermax = p->itermax;
  d.flags = p->flags;
  d.tol = p->tol;
  d.freeze_tol = p->freeze_tol < 0.0 ? 1e-3 * p->tol : p->freeze_tol;
  d.maxblk = MAXBLK;
  d.nblkB = (int32_t)(rows ? stream_blocks(p->ndim) : sys_blocks(p->ndim, p->nrhs));
  d.hist_cap = (p->flags & KOMEGA_F_HISTORY) ? p->itermax : 0;
  d.x32 = x32 ? 1 : 0;
  d.shift_block = SHIFT_BLOCK;  // measured best on MI355X for 32..1024 shifts
  d.shift_nt = 1;
  // graph replay applies every step at once
  d.xblk = (p->flags & KOMEGA_F_GRAPH) ? 1 : (x32 ? XBLK_DEFAULT_X32 : XBLK_DEFAULT);
  d.blk_gen = 1;

  komega_status rc = KOMEGA_OK;
  auto A = [&](auto** ptr, size_t cnt) {
    if (rc == KOMEGA_OK) rc = dalloc(ptr, cnt, s->owned);
  };
  zc* zd;
  A(&zd, nz);
  d.z = zd;
  A(&d.st, nr);
  A(&d.pi, nr * nz);
  A(&d.pio, nr * nz);
  A(&d.active, nr * nz);
  A(&d.res, nr * nz);
  A(&d.ak, nr * nz);
  A(&d.bk, nr * nz);
  A(&d.ck, nr * nz);
  A(&d.apply, nr * nz);
  A(&d.u, nr * nz * (nl ? nl : 1));
  A(&d.partA, nr * MAXBLK);                               // 2 doubles per slot
  A(&d.partB, nr * MAXBLK * (2 + KOMEGA_MAX_NL));         // >= 3 + 2*MAX_NL doubles per slot
  if (d.hist_cap > 0) {
    const size_t cap = (size_t)d.hist_cap;
    A(&d.h_alpha, nr * cap);
    A(&d.h_beta, nr * cap);
    A(&d.h_zs, nr * cap);
    A(&d.h_sw, nr * cap * 2);
    A(&d.h_seed, nr * cap);
    A(&d.h_pr, nr * cap * (nl ? nl : 1));
    A(&d.h_nu, nr * cap);
  }
  A(&d.pb, nr * (nl ? nl : 1));
  unsigned char* Q;
  A(&Q, VR * s->es);
  s->bf.Q = Q;
  if (p->nl == 0) {
    // whole x: the residual ring (its slots are R and RO), block coefficients
    unsigned char* ring;
    A(&ring, (size_t)RING * VR * s->es);
    s->ring = ring;
    A(&d.bcoef, nr * nz * (size_t)bcoef_len());
    A(&d.btouch, nr * nz);
    A(&d.bstep, nr * nz * (size_t)(3 * XBLK_MAX));
  } else {
    unsigned char *R, *RO;
    A(&R, VR * s->es);
    A(&RO, VR * s->es);
    s->bf.R = R; s->bf.RO = RO;
  }
  if (p->method == KOMEGA_BICG) {
    unsigned char *Rs, *Qs, *ROs;
    A(&Rs, VR * s->es);
    A(&Qs, VR * s->es);
    A(&ROs, VR * s->es);
    s->bf.Rs = Rs; s->bf.Qs = Qs; s->bf.ROs = ROs;
  }
  if (p->nl == 0) {
    unsigned char* pp;
    A(&pp, nz * VR * s->xes);
    s->bf.p = pp;
  }
  int64_t* soffd = nullptr;
  int2 *wlad = nullptr, *wlbd = nullptr, *wltd = nullptr;
  if (rows) {
    A(&soffd, soff.size());
    A(&wlad, wla.size());
    A(&wlbd, wlb.size());
    A(&wltd, wlt.size());
  }
  if (rc != KOMEGA_OK) { delete s; return rc; }
  if (s->ring) ring_point(s);
  std::vector<zc> zh(nz);
  for (size_t k = 0; k < nz; ++k) zh[k] = zmk(z[2 * k], z[2 * k + 1]);
  hipError_t e = hipMemcpy(zd, zh.data(), nz * sizeof(zc), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(d.st, 0, nr * sizeof(RhsState));
  if (rows) {
    if (e == hipSuccess) e = hipMemcpy(soffd, soff.data(), soff.size() * sizeof(int64_t), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(wlad, wla.data(), wla.size() * sizeof(int2), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(wlbd, wlb.data(), wlb.size() * sizeof(int2), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(wltd, wlt.data(), wlt.size() * sizeof(int2), hipMemcpyHostToDevice);
    d.soff = soffd;
    d.wl_a = wlad;
    d.wl_b = wlbd;
    d.wl_t = wltd;
    d.nwl_a = (int32_t)wla.size();
    d.nwl_b = (int32_t)wlb.size();
    d.nwl_t = (int32_t)wlt.size();
    s->wla_full = wla;
    s->wlb_full = wlb;
    s->retired.assign(nr, 0);
  }
  if (e == hipSuccess) e = hipHostMalloc((void**)&s->h_state, nr * sizeof(RhsState), hipHostMallocDefault);
  if (e != hipSuccess) {
    delete s;
    return set_err(KOMEGA_E_HIP, "solver set-up failed: %s", hipGetErrorString(e));
  }
  *out = s;
  return KOMEGA_OK;
}

extern "C" komega_status komega_create(komega_solver** out, const komega_params* p, const double* z) {
  return create_solver(out, p, z, nullptr);
}

extern "C" komega_status komega_create_batched(komega_solver** out, const komega_params* p, const double* z,
                                               const int64_t* rows) {
  if (!rows) return set_err(KOMEGA_E_INVALID, "null rows");
  return create_solver(out, p, z, rows);
}

// Batched solves: the product and seed work lists without the entries of the
// systems marked in s->retired, uploaded in place (the lists only shrink, so
// the buffers of the full lists hold them), in stream order.
static komega_status upload_lists(komega_solver* s) {
  std::vector<int2> a, b;
  a.reserve(s->wla_full.size());
  b.reserve(s->wlb_full.size());
  for (const int2& e : s->wla_full)
    if (!s->retired[(size_t)e.x]) a.push_back(e);
  for (const int2& e : s->wlb_full)
    if (!s->retired[(size_t)e.x]) b.push_back(e);
  if (a.empty() || b.empty()) return KOMEGA_OK;  // every system stopped: nothing is launched
  HIPCHK(hipMemcpyAsync(const_cast<int2*>(s->ds.wl_a), a.data(), a.size() * sizeof(int2), hipMemcpyHostToDevice,
                        s->stream));
  HIPCHK(hipMemcpyAsync(const_cast<int2*>(s->ds.wl_b), b.data(), b.size() * sizeof(int2), hipMemcpyHostToDevice,
                        s->stream));
  HIPCHK(hipStreamSynchronize(s->stream));  // the host vectors go out of scope
  s->ds.nwl_a = (int32_t)a.size();
  s->ds.nwl_b = (int32_t)b.size();
  return KOMEGA_OK;
}

// Full lists again (init, restore: stop flags are reset or replaced).
static komega_status restore_lists(komega_solver* s) {
  if (!s->batched || s->nretired == 0) return KOMEGA_OK;
  std::fill(s->retired.begin(), s->retired.end(), (char)0);
  s->nretired = 0;
  return upload_lists(s);
}

// Retire systems that have stopped from the product and seed work lists, so
// later launches do not dispatch work-groups that would only exit.  A system
// is retired once its state shows no step left to finalise or to apply
// (pending, step_pending clear): from then on no kernel of those lists has
// work for it.  Not with captured graphs (their grids are fixed).  Reads the
// host mirror that collect() has just filled.
static komega_status retire_stopped(komega_solver* s) {
  if (!s->batched || (s->p.flags & KOMEGA_F_GRAPH)) return KOMEGA_OK;
  bool changed = false;
  for (size_t r = 0; r < (size_t)s->p.nrhs; ++r) {
    const RhsState& h = s->h_state[r];
    if (!s->retired[r] && h.stop && !h.pending && !h.step_pending) {
      s->retired[r] = 1;
      ++s->nretired;
      changed = true;
    }
  }
  return changed ? upload_lists(s) : KOMEGA_OK;
}

extern "C" komega_status komega_init(komega_solver* s, const void* b, const void* bshadow, const void* P,
                                     void* x) {
  if (!s || !b || !x) return set_err(KOMEGA_E_INVALID, "null argument");
  if (s->p.nl > 0 && !P) return set_err(KOMEGA_E_INVALID, "projected mode (nl > 0) needs P");
  s->drop_graphs();
  s->ds.P = P;
  s->ds.y = s->p.nl > 0 ? reinterpret_cast<zc*>(x) : nullptr;
  s->bf.x = x;
  if (s->ring) {
    s->it = 0;
    ring_point(s);
    s->step_pending_host = false;
    s->blk_steps = 0;
  }
  TRY(restore_lists(s));
  // The reverse-communication path keeps its shadow in the caller's rs; the
  // built-in path starts from bshadow or conj(b).
  HIPCHK(launch_init(s->ds, s->bf, b, s->p.method == KOMEGA_BICG ? bshadow : nullptr, x, s->stream));
  s->initialized = 1;
  s->mode = 0;
  return KOMEGA_OK;
}

static komega_status collect(komega_solver* s, komega_iter* st, bool* all_stopped) {
  const size_t nr = (size_t)s->p.nrhs;
  HIPCHK(hipMemcpyAsync(s->h_state, s->ds.st, nr * sizeof(RhsState), hipMemcpyDeviceToHost, s->stream));
  HIPCHK(hipStreamSynchronize(s->stream));
  bool all = true, conv = true;
  komega_status first_err = KOMEGA_OK;
  for (size_t r = 0; r < nr; ++r) {
    const RhsState& h = s->h_state[r];
    if (st) {
      st[r].status = h.status;
      st[r].iter = h.iter;
      st[r].seed = h.seed;
      st[r].nswitch = h.nswitch;
      st[r].maxres = h.maxres;
    }
    if (!h.stop) all = false;
    if (h.status != KOMEGA_CONVERGED) conv = false;
    if (h.status < 0 && first_err == KOMEGA_OK) first_err = h.status;
  }
  if (all_stopped) *all_stopped = all;
  if (!all) return KOMEGA_OK;
  if (conv) return KOMEGA_CONVERGED;
  return first_err != KOMEGA_OK ? first_err : KOMEGA_OK;
}

extern "C" komega_status komega_update(komega_solver* s, const void* q, void* r, const void* qs, void* rs,
                                       komega_iter* st) {
  if (!s || !q || !r) return set_err(KOMEGA_E_INVALID, "null argument");
  if (!s->initialized) return set_err(KOMEGA_E_STATE, "komega_update before komega_init");
  if (s->mode == 2) return set_err(KOMEGA_E_STATE, "solve already driven by komega_iterate");
  const bool bicg = s->p.method == KOMEGA_BICG;
  if (bicg && (!qs || !rs)) return set_err(KOMEGA_E_INVALID, "BiCG needs the shadow vectors qs, rs");
  s->mode = 1;
  Buffers b = s->bf;
  b.R = r;
  b.Q = const_cast<void*>(q);
  b.RN = nullptr;
  if (bicg) { b.Rs = rs; b.Qs = const_cast<void*>(qs); }
  const int64_t nblk = s->ds.nblkB;
  // the caller holds r: every step is applied to x at once (no blocks)
  DevSolver ds = s->ds;
  ds.xblk = 0;
  {
    Timed t(s, KOMEGA_K_DOT);
    HIPCHK(launch_dot(ds, bicg ? rs : r, q, nblk, s->stream));
  }
  {
    Timed t(s, KOMEGA_K_SEED);
    HIPCHK(launch_seed(ds, b, true, nblk, nblk, s->stream));
  }
  HIPCHK(launch_finalize(ds, nblk, s->stream));
  if (s->p.nl == 0) {
    Timed t(s, KOMEGA_K_SHIFT);
    HIPCHK(launch_shift(ds, b, s->stream));
  }
  if (!st) return KOMEGA_OK;
  bool all = false;
  komega_status rc = collect(s, st, &all);
  if (rc < 0 && rc != KOMEGA_E_MAXITER && rc != KOMEGA_E_BREAKDOWN && rc != KOMEGA_E_SHIFT_BREAKDOWN &&
      rc != KOMEGA_E_NONFINITE)
    return rc;
  return all ? rc : KOMEGA_OK;
}

static komega_status check_op(komega_solver* s, const komega_op* op) {
  if (!op) return set_err(KOMEGA_E_INVALID, "null operator");
  if (op->d.M != s->p.ndim)
    return set_err(KOMEGA_E_INVALID, "operator dimension %lld != solver dimension %lld",
                   (long long)op->d.M, (long long)s->p.ndim);
  if (s->p.method == KOMEGA_CG_R && op->d.kind == OP_CSR && op->d.complex_vals)
    return set_err(KOMEGA_E_INVALID, "KOMEGA_CG_R needs a real operator");
  if (op->d.nsys && (!s->batched || op->h_soff != s->h_soff))
    return set_err(KOMEGA_E_INVALID, "a batched operator needs a batched solver with the same systems");
  if (!s->batched) return KOMEGA_OK;
  // batched systems: the product must not couple two systems
  switch (op->d.kind) {
    case OP_STENCIL:
      if (!op->d.nsys && s->p.nrhs > 1)
        return set_err(KOMEGA_E_INVALID, "batched systems need a batched stencil (one cube per system)");
      return KOMEGA_OK;
    case OP_CALLBACK:
      return KOMEGA_OK;  // the caller's product acts on the concatenated vector
    case OP_CSR: {
      if (s->csr_checked == op && s->csr_checked_version == op->version) return KOMEGA_OK;
      for (int r = 0; r < s->p.nrhs; ++r) {
        const int64_t lo = s->h_soff[r], hi = s->h_soff[r + 1];
        for (int64_t i = lo; i < hi; ++i)
          for (int64_t q = op->h_rowptr[i]; q < op->h_rowptr[i + 1]; ++q)
            if (op->h_col[q] < lo || op->h_col[q] >= hi)
              return set_err(KOMEGA_E_INVALID, "CSR row %lld couples system %d to column %d of another system",
                             (long long)i, r, op->h_col[q]);
      }
      s->csr_checked = op;
      s->csr_checked_version = op->version;
      return KOMEGA_OK;
    }
    default:
      return set_err(KOMEGA_E_INVALID, "batched systems take stencil, CSR or callback operators");
  }
}

// Partial-sum slots per system, i.e. product work-groups per right-hand side
// (the shared-matrix CSR product spreads this many over all right-hand
// sides): the tuning knob when set (uniform layout), else the operator's own
// choice.
static int64_t spmv_count(const komega_solver* s, const komega_op* op) {
  if (s->ds.spmv_blk > 0 && !s->batched) return s->ds.spmv_blk;
  if (op->d.kind == OP_CSR && !s->batched && s->p.nrhs > 1 && s->p.method != KOMEGA_BICG) {
    // several right-hand sides of one CSR matrix: the shared-matrix product
    const int64_t g = csr_mr_groups(s->p.ndim, s->p.nrhs);
    if (g > 0) return g;
  }
  const int64_t b = spmv_blocks(op->d, s->p.ndim);
  if (s->batched) return b;
  const int64_t cap = sys_blocks(s->p.ndim, s->p.nrhs);
  return b < cap ? b : cap;
}

// One iteration on the solver's own buffers: product (its group 0 finalises
// the previous step), whole-x update of the previous step, seed update.
// The block holds one more finalised step (its residual is r_it).
static void note_step(komega_solver* s) {
  if (s->blk_steps == 0) s->blk_slot0 = (int)(((s->it % RING) + RING) % RING);
  ++s->blk_steps;
}

static komega_status apply_block(komega_solver* s, hipStream_t st) {
  {
    Timed t(s, KOMEGA_K_SHIFT);
    HIPCHK(launch_shift_blk(s->ds, s->ring, s->vrows, s->blk_slot0, RING, s->bf.x, s->bf.p, st));
  }
  ++s->ds.blk_gen;
  s->blk_steps = 0;
  return KOMEGA_OK;
}

static komega_status one_iteration(komega_solver* s, const komega_op* op, hipStream_t st) {
  const bool bicg = s->p.method == KOMEGA_BICG;
  Buffers& b = s->bf;
  if (s->ring) b.RN = ring_slot(s, s->it + 1);
  const int64_t nblkB = s->ds.nblkB;
  int64_t nblkA;
  if (op->d.kind == OP_CALLBACK) {
    nblkA = s->ds.nblkB;
    {
      Timed t(s, KOMEGA_K_SPMV);
      const int32_t cplx = s->p.method != KOMEGA_CG_R;
      const int32_t nvec = s->batched ? 1 : s->p.nrhs;  // batched: one concatenated vector
      if (op->fn(op->user, b.R, b.Q, nvec, cplx, st) != 0)
        return set_err(KOMEGA_E_INVALID, "operator callback failed");
      if (bicg && op->fn(op->user, b.Rs, b.Qs, nvec, cplx, st) != 0)
        return set_err(KOMEGA_E_INVALID, "operator callback failed");
    }
    Timed t(s, KOMEGA_K_DOT);
    HIPCHK(launch_dot(s->ds, bicg ? b.Rs : b.R, b.Q, nblkA, st));
  } else {
    nblkA = spmv_count(s, op);
    Timed t(s, KOMEGA_K_SPMV);
    HIPCHK(launch_spmv(s->ds, op->d, b, true, nblkA, st));
  }
  if (s->p.nl == 0) {
    if (blocked(s)) {
      // the product's finaliser group has composed step it-1 into the block
      if (s->step_pending_host) note_step(s);
      if (s->blk_steps >= s->ds.xblk) TRY(apply_block(s, st));
    } else {
      Timed t(s, KOMEGA_K_SHIFT);
      HIPCHK(launch_shift(s->ds, b, st));
    }
  }
  s->step_pending_host = false;
  {
    Timed t(s, KOMEGA_K_SEED);
    HIPCHK(launch_seed(s->ds, b, false, nblkA, nblkB, st));
  }
  s->step_pending_host = true;
  if (s->ring) {
    ++s->it;
    ring_point(s);
    b.RN = nullptr;
  } else {
    std::swap(b.R, b.RO);
  }
  if (bicg) std::swap(b.Rs, b.ROs);
  return KOMEGA_OK;
}

// Finalises the last step of a batch and applies its whole-x update; a
// partly filled block is applied only if apply_partial (komega_solve keeps
// filling it between its convergence checks).
static komega_status finish_batch(komega_solver* s, bool apply_partial) {
  HIPCHK(launch_finalize(s->ds, s->ds.nblkB, s->stream));
  if (s->p.nl == 0) {
    if (blocked(s)) {
      if (s->step_pending_host) note_step(s);
      if (s->blk_steps >= (apply_partial ? 1 : s->ds.xblk)) TRY(apply_block(s, s->stream));
    } else {
      Timed t(s, KOMEGA_K_SHIFT);
      HIPCHK(launch_shift(s->ds, s->bf, s->stream));
    }
  }
  s->step_pending_host = false;
  return KOMEGA_OK;
}

// Two iterations captured once (buffer roles return to the start) and
// replayed on the solver's stream.  Captured on a private stream, since the
// caller's stream may be the legacy default stream, which cannot capture.
static komega_status graph_for(komega_solver* s, const komega_op* op, hipGraphExec_t* exec) {
  for (auto& g : s->graphs)
    if (g.op == op && g.version == op->version && g.R == s->bf.R) {
      *exec = g.exec;
      return KOMEGA_OK;
    }
  if (!s->cap_stream) HIPCHK(hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking));
  const uint32_t saved_mask = s->tmask;
  s->tmask = 0;
  void* R0 = s->bf.R;
  const Buffers saved_bf = s->bf;
  const int64_t saved_it = s->it;
  const bool saved_pending = s->step_pending_host;
  HIPCHK(hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal));
  komega_status rc = one_iteration(s, op, s->cap_stream);
  if (rc == KOMEGA_OK) rc = one_iteration(s, op, s->cap_stream);
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamEndCapture(s->cap_stream, &graph);
  s->tmask = saved_mask;
  s->bf = saved_bf;  // the launches of the graph advance the state
  s->it = saved_it;
  s->step_pending_host = saved_pending;
  if (rc != KOMEGA_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (e != hipSuccess) return set_err(KOMEGA_E_HIP, "graph capture failed: %s", hipGetErrorString(e));
  hipGraphExec_t ge = nullptr;
  e = hipGraphInstantiate(&ge, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return set_err(KOMEGA_E_HIP, "graph instantiation failed: %s", hipGetErrorString(e));
  s->graphs.push_back({op, op->version, R0, ge});
  *exec = ge;
  return KOMEGA_OK;
}

static komega_status iterate_steps(komega_solver* s, const komega_op* op, int32_t n, bool apply_partial) {
  if (!s) return set_err(KOMEGA_E_INVALID, "null solver");
  if (!s->initialized) return set_err(KOMEGA_E_STATE, "komega_iterate before komega_init");
  if (s->mode == 1) return set_err(KOMEGA_E_STATE, "solve already driven by komega_update");
  TRY(check_op(s, op));
  if (n < 0) return set_err(KOMEGA_E_INVALID, "n must be >= 0");
  if (n == 0) return KOMEGA_OK;
  s->mode = 2;
  const bool graphs = (s->p.flags & KOMEGA_F_GRAPH) && s->tmask == 0 && op->d.kind != OP_CALLBACK;
  if (graphs) {
    while (n >= 2) {
      hipGraphExec_t ge = nullptr;
      TRY(graph_for(s, op, &ge));
      HIPCHK(hipGraphLaunch(ge, s->stream));
      // the host side of the two replayed iterations
      if (s->ring) {
        s->it += 2;
        ring_point(s);
      }
      s->step_pending_host = true;
      n -= 2;
    }
  }
  for (int32_t i = 0; i < n; ++i) TRY(one_iteration(s, op, s->stream));
  return finish_batch(s, apply_partial);
}

extern "C" komega_status komega_iterate(komega_solver* s, const komega_op* op, int32_t n) {
  return iterate_steps(s, op, n, true);
}

extern "C" komega_status komega_solve(komega_solver* s, const komega_op* op, int32_t poll, komega_iter* st) {
  if (!s) return set_err(KOMEGA_E_INVALID, "null solver");
  if (poll <= 0) poll = 16;
  TRY(check_op(s, op));
  komega_status rc = KOMEGA_OK;
  for (;;) {
    bool all = false;
    rc = collect(s, st, &all);
    if (rc == KOMEGA_E_HIP || all) break;
    TRY(retire_stopped(s));
    // a whole-x block may stay partly filled across the checks
    rc = iterate_steps(s, op, poll, false);
    if (rc != KOMEGA_OK) break;
  }
  if (rc == KOMEGA_E_HIP) return rc;
  // x^k current on return: apply what the last block holds
  if (s->initialized && s->p.nl == 0 && blocked(s) && s->blk_steps > 0) TRY(apply_block(s, s->stream));
  return rc;
}

extern "C" komega_status komega_getstate(komega_solver* s, komega_iter* st) {
  if (!s || !st) return set_err(KOMEGA_E_INVALID, "null argument");
  bool all = false;
  komega_status rc = collect(s, st, &all);
  return rc == KOMEGA_E_HIP ? rc : KOMEGA_OK;
}

extern "C" komega_status komega_getresidual(komega_solver* s, double* res) {
  if (!s || !res) return set_err(KOMEGA_E_INVALID, "null argument");
  HIPCHK(hipMemcpyAsync(res, s->ds.res, sizeof(double) * s->p.nrhs * s->p.nz, hipMemcpyDeviceToHost,
                        s->stream));
  HIPCHK(hipStreamSynchronize(s->stream));
  return KOMEGA_OK;
}

extern "C" komega_status komega_getcoef(komega_solver* s, int32_t rhs, double* alpha, double* beta,
                                        double* zseed, int32_t* seed, double* sw, double* Pr, int32_t* n) {
  if (!s || !n) return set_err(KOMEGA_E_INVALID, "null argument");
  if (s->ds.hist_cap == 0) return set_err(KOMEGA_E_STATE, "history was not requested (KOMEGA_F_HISTORY)");
  if (rhs < 0 || rhs >= s->p.nrhs) return set_err(KOMEGA_E_INVALID, "rhs out of range");
  komega_iter it[1];
  std::vector<komega_iter> all((size_t)s->p.nrhs);
  TRY(komega_getstate(s, all.data()));
  it[0] = all[(size_t)rhs];
  const int32_t cnt = it[0].iter < s->ds.hist_cap ? it[0].iter : s->ds.hist_cap;
  const size_t off = (size_t)rhs * s->ds.hist_cap;
  const size_t nl = (size_t)(s->p.nl ? s->p.nl : 1);
  if (cnt > 0) {
    if (alpha) HIPCHK(hipMemcpy(alpha, s->ds.h_alpha + off, sizeof(zc) * cnt, hipMemcpyDeviceToHost));
    if (beta) HIPCHK(hipMemcpy(beta, s->ds.h_beta + off, sizeof(zc) * cnt, hipMemcpyDeviceToHost));
    if (zseed) HIPCHK(hipMemcpy(zseed, s->ds.h_zs + off, sizeof(zc) * cnt, hipMemcpyDeviceToHost));
    if (seed) HIPCHK(hipMemcpy(seed, s->ds.h_seed + off, sizeof(int32_t) * cnt, hipMemcpyDeviceToHost));
    if (sw) HIPCHK(hipMemcpy(sw, s->ds.h_sw + 2 * off, sizeof(zc) * 2 * cnt, hipMemcpyDeviceToHost));
    if (Pr && s->p.nl > 0)
      HIPCHK(hipMemcpy(Pr, s->ds.h_pr + off * nl, sizeof(zc) * nl * cnt, hipMemcpyDeviceToHost));
  }
  *n = cnt;
  return KOMEGA_OK;
}

extern "C" komega_status komega_recalc(komega_solver* s, int32_t rhs, int32_t nzn, const double* znew, void* y,
                                       double* res) {
  if (!s || !znew || !y || nzn < 1) return set_err(KOMEGA_E_INVALID, "bad argument");
  if (s->ds.hist_cap == 0) return set_err(KOMEGA_E_STATE, "history was not requested (KOMEGA_F_HISTORY)");
  if (s->p.nl == 0) return set_err(KOMEGA_E_STATE, "recalculation needs the projected mode (nl > 0)");
  if (rhs < 0 || rhs >= s->p.nrhs) return set_err(KOMEGA_E_INVALID, "rhs out of range");
  if (!s->initialized) return set_err(KOMEGA_E_STATE, "no solve to recalculate from");
  std::vector<komega_iter> it((size_t)s->p.nrhs);
  TRY(komega_getstate(s, it.data()));
  const int32_t n = it[(size_t)rhs].iter < s->ds.hist_cap ? it[(size_t)rhs].iter : s->ds.hist_cap;
  std::vector<zc> zh(nzn);
  for (int k = 0; k < nzn; ++k) {
    if (!std::isfinite(znew[2 * k]) || !std::isfinite(znew[2 * k + 1]))
      return set_err(KOMEGA_E_INVALID, "shift %d is not finite", k);
    zh[k] = zmk(znew[2 * k], znew[2 * k + 1]);
  }
  zc* zd = nullptr;
  double* rd = nullptr;
  HIPCHK(hipMallocAsync((void**)&zd, sizeof(zc) * nzn, s->stream));
  HIPCHK(hipMallocAsync((void**)&rd, sizeof(double) * nzn, s->stream));
  hipError_t e = hipMemcpyAsync(zd, zh.data(), sizeof(zc) * nzn, hipMemcpyHostToDevice, s->stream);
  if (e == hipSuccess) e = launch_recalc(s->ds, rhs, n, zd, nzn, reinterpret_cast<zc*>(y), rd, s->stream);
  if (e == hipSuccess && res) e = hipMemcpyAsync(res, rd, sizeof(double) * nzn, hipMemcpyDeviceToHost, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  (void)hipFreeAsync(zd, s->stream);
  (void)hipFreeAsync(rd, s->stream);
  if (e != hipSuccess) return set_err(KOMEGA_E_HIP, "recalculation failed: %s", hipGetErrorString(e));
  return KOMEGA_OK;
}

// ------------------------------------------------------------ save/restore
// Snapshot layout: header, then the device pieces in a fixed order.
namespace {
struct SnapHeader {
  char magic[8];
  int32_t version, method, nz, nl, nrhs, itermax, mode, hist_cap;
  uint32_t flags, pad;
  int64_t M;
  uint64_t layout;  // hash of the batched row partition (0: uniform)
};

// FNV-1a over the system offsets, so a snapshot only loads into a solver with
// the same partition of rows.
uint64_t layout_hash(const komega_solver* s) {
  if (!s->batched) return 0;
  uint64_t h = 1469598103934665603ull;
  for (int64_t v : s->h_soff) {
    for (int b = 0; b < 8; ++b) {
      h ^= (uint64_t)((v >> (8 * b)) & 0xff);
      h *= 1099511628211ull;
    }
  }
  return h;
}

struct Piece {
  void* dev;
  size_t bytes;
};

std::vector<Piece> snapshot_pieces(komega_solver* s) {
  const size_t nr = (size_t)s->p.nrhs, nz = (size_t)s->p.nz, nl = (size_t)s->p.nl;
  const size_t vb = (size_t)s->vrows * s->es;
  DevSolver& d = s->ds;
  std::vector<Piece> v = {
      {d.st, nr * sizeof(RhsState)},       {d.pi, nr * nz * sizeof(zc)},     {d.pio, nr * nz * sizeof(zc)},
      {d.active, nr * nz * sizeof(int32_t)}, {d.res, nr * nz * sizeof(double)}, {d.ak, nr * nz * sizeof(zc)},
      {d.bk, nr * nz * sizeof(zc)},        {d.ck, nr * nz * sizeof(zc)},     {d.apply, nr * nz * sizeof(int32_t)},
      {d.u, nr * nz * (nl ? nl : 1) * sizeof(zc)}, {d.pb, nr * (nl ? nl : 1) * sizeof(zc)},
      {s->bf.R, vb},                       {s->bf.RO, vb}};
  if (s->p.method == KOMEGA_BICG) {
    v.push_back({s->bf.Rs, vb});
    v.push_back({s->bf.ROs, vb});
  }
  if (nl > 0) v.push_back({d.y, nr * nz * nl * sizeof(zc)});
  else v.push_back({s->bf.p, nz * (size_t)s->vrows * s->xes});
  if (d.hist_cap > 0) {
    const size_t cap = (size_t)d.hist_cap;
    v.push_back({d.h_alpha, nr * cap * sizeof(zc)});
    v.push_back({d.h_beta, nr * cap * sizeof(zc)});
    v.push_back({d.h_zs, nr * cap * sizeof(zc)});
    v.push_back({d.h_sw, nr * cap * 2 * sizeof(zc)});
    v.push_back({d.h_seed, nr * cap * sizeof(int32_t)});
    v.push_back({d.h_pr, nr * cap * (nl ? nl : 1) * sizeof(zc)});
    v.push_back({d.h_nu, nr * cap * sizeof(double)});
  }
  return v;
}
}  // namespace

extern "C" komega_status komega_state_size(komega_solver* s, int64_t* bytes) {
  if (!s || !bytes) return set_err(KOMEGA_E_INVALID, "null argument");
  if (!s->initialized) return set_err(KOMEGA_E_STATE, "nothing to save before komega_init");
  size_t n = sizeof(SnapHeader);
  for (const Piece& p : snapshot_pieces(s)) n += p.bytes;
  *bytes = (int64_t)n;
  return KOMEGA_OK;
}

extern "C" komega_status komega_save_state(komega_solver* s, void* host, int64_t bytes) {
  int64_t need = 0;
  TRY(komega_state_size(s, &need));
  if (!host || bytes < need) return set_err(KOMEGA_E_INVALID, "buffer too small (%lld < %lld)", (long long)bytes,
                                            (long long)need);
  SnapHeader h{};
  memcpy(h.magic, "KOMEGA01", 8);
  h.version = 1;
  h.method = s->p.method; h.nz = s->p.nz; h.nl = s->p.nl; h.nrhs = s->p.nrhs; h.itermax = s->p.itermax;
  h.mode = s->mode; h.hist_cap = s->ds.hist_cap; h.flags = s->p.flags; h.M = s->p.ndim;
  h.layout = layout_hash(s);
  unsigned char* out = reinterpret_cast<unsigned char*>(host);
  memcpy(out, &h, sizeof h);
  size_t off = sizeof h;
  for (const Piece& p : snapshot_pieces(s)) {
    HIPCHK(hipMemcpyAsync(out + off, p.dev, p.bytes, hipMemcpyDeviceToHost, s->stream));
    off += p.bytes;
  }
  HIPCHK(hipStreamSynchronize(s->stream));
  return KOMEGA_OK;
}

extern "C" komega_status komega_restore_state(komega_solver* s, const void* host, int64_t bytes, const void* P,
                                              void* x) {
  if (!s || !host || !x) return set_err(KOMEGA_E_INVALID, "null argument");
  if (s->p.nl > 0 && !P) return set_err(KOMEGA_E_INVALID, "projected mode needs P");
  SnapHeader h;
  if (bytes < (int64_t)sizeof h) return set_err(KOMEGA_E_INVALID, "snapshot too small");
  memcpy(&h, host, sizeof h);
  if (memcmp(h.magic, "KOMEGA01", 8) != 0 || h.version != 1) return set_err(KOMEGA_E_INVALID, "not a snapshot");
  if (h.method != s->p.method || h.nz != s->p.nz || h.nl != s->p.nl || h.nrhs != s->p.nrhs || h.M != s->p.ndim ||
      h.hist_cap != s->ds.hist_cap || h.layout != layout_hash(s) ||
      ((h.flags ^ s->p.flags) & KOMEGA_F_X32) != 0)
    return set_err(KOMEGA_E_INVALID, "snapshot was taken from a solver with other parameters");
  s->drop_graphs();
  s->ds.P = P;
  s->ds.y = s->p.nl > 0 ? reinterpret_cast<zc*>(x) : nullptr;
  s->bf.x = x;
  s->initialized = 1;
  int64_t need = 0;
  TRY(komega_state_size(s, &need));
  if (bytes < need) return set_err(KOMEGA_E_INVALID, "snapshot truncated");
  const unsigned char* in = reinterpret_cast<const unsigned char*>(host);
  size_t off = sizeof h;
  for (const Piece& p : snapshot_pieces(s)) {
    HIPCHK(hipMemcpyAsync(p.dev, in + off, p.bytes, hipMemcpyHostToDevice, s->stream));
    off += p.bytes;
  }
  HIPCHK(hipStreamSynchronize(s->stream));
  TRY(restore_lists(s));
  s->mode = h.mode;
  s->step_pending_host = false;
  s->blk_steps = 0;
  // the snapshot's block generations belong to the saving solver: continue
  // past all of them, so no restored count is taken for a block of this one
  {
    const RhsState* rs = reinterpret_cast<const RhsState*>(in + sizeof h);
    uint32_t g = s->ds.blk_gen;
    for (int r = 0; r < s->p.nrhs; ++r) {
      RhsState v;
      memcpy(&v, rs + r, sizeof v);
      if (v.blk_gen >= g) g = v.blk_gen + 1;
    }
    s->ds.blk_gen = g;
  }
  return KOMEGA_OK;
}

extern "C" komega_status komega_finalize(komega_solver* s) {
  if (!s) return KOMEGA_OK;
  (void)hipStreamSynchronize(s->stream);
  delete s;
  return KOMEGA_OK;
}

// --------------------------------------------------------------- timing
extern "C" komega_status komega_set_timing(komega_solver* s, uint32_t mask) {
  if (!s) return set_err(KOMEGA_E_INVALID, "null solver");
  s->tmask = mask;
  return KOMEGA_OK;
}

extern "C" komega_status komega_get_timing(komega_solver* s, int32_t cls, double* ms, int64_t* count,
                                           int32_t reset) {
  if (!s || cls < 0 || cls >= KOMEGA_K_NCLASS) return set_err(KOMEGA_E_INVALID, "bad argument");
  HIPCHK(hipStreamSynchronize(s->stream));
  for (auto& pr : s->ev[cls]) {
    float t = 0.f;
    HIPCHK(hipEventElapsedTime(&t, pr.first, pr.second));
    s->acc_ms[cls] += t;
    s->acc_n[cls] += 1;
    s->pool.push_back(pr.first);
    s->pool.push_back(pr.second);
  }
  s->ev[cls].clear();
  if (ms) *ms = s->acc_ms[cls];
  if (count) *count = s->acc_n[cls];
  if (reset) { s->acc_ms[cls] = 0.0; s->acc_n[cls] = 0; }
  return KOMEGA_OK;
}

extern "C" komega_status komega_launch_info(const komega_solver* s, const komega_op* op, int32_t cls,
                                            int64_t* blocks, int64_t* threads) {
  if (!s || !blocks || !threads) return set_err(KOMEGA_E_INVALID, "null argument");
  *threads = TPB;
  if (s->batched) {
    switch (cls) {
      case KOMEGA_K_SPMV:
      case KOMEGA_K_DOT: *blocks = s->ds.nwl_a; return KOMEGA_OK;
      case KOMEGA_K_SEED: *blocks = s->ds.nwl_b; return KOMEGA_OK;
      case KOMEGA_K_SHIFT:
        *blocks = (int64_t)s->ds.nwl_t * ((s->p.nz + s->ds.shift_block - 1) / s->ds.shift_block);
        return KOMEGA_OK;
      default: return set_err(KOMEGA_E_INVALID, "unknown kernel class");
    }
  }
  switch (cls) {
    case KOMEGA_K_SPMV: {
      if (!op) return set_err(KOMEGA_E_INVALID, "SPMV needs the operator");
      const int64_t n = spmv_count(s, op);
      // the shared-matrix CSR product (same condition as launch_spmv) spreads
      // its n work-groups over the nrhs grid rows
      const bool shared = op->d.kind == OP_CSR && s->p.nrhs > 1 && s->p.method != KOMEGA_BICG &&
                          n % s->p.nrhs == 0;
      *blocks = (shared ? n / s->p.nrhs : n) + 1;  // + the finaliser group
      break;
    }
    case KOMEGA_K_SEED:
      *blocks = s->ds.nblkB;
      break;
    case KOMEGA_K_DOT:
      *blocks = s->ds.nblkB + 1;
      break;
    case KOMEGA_K_SHIFT:
      *blocks = ((s->p.ndim + TPB - 1) / TPB) * ((s->p.nz + s->ds.shift_block - 1) / s->ds.shift_block);
      break;
    default:
      return set_err(KOMEGA_E_INVALID, "unknown kernel class");
  }
  return KOMEGA_OK;
}

extern "C" komega_status komega_set_tuning(komega_solver* s, int32_t knob, int32_t value) {
  if (!s) return set_err(KOMEGA_E_INVALID, "null solver");
  switch (knob) {
    case KOMEGA_T_SHIFT_BLOCK:
      if (value != 1 && value != 2 && value != 4 && value != 8 && value != 16)
        return set_err(KOMEGA_E_INVALID, "shift block must be 1, 2, 4, 8 or 16");
      s->ds.shift_block = value;
      break;
    case KOMEGA_T_SHIFT_NT:
      if (value != 0 && value != 1) return set_err(KOMEGA_E_INVALID, "nontemporal flag must be 0 or 1");
      s->ds.shift_nt = value;
      break;
    case KOMEGA_T_SPMV_BLOCKS:
      if (value < 0 || value > MAXBLK) return set_err(KOMEGA_E_INVALID, "product work-groups must be in [0, %d]", MAXBLK);
      s->ds.spmv_blk = value;
      break;
    case KOMEGA_T_SHIFT_ORDER:
      if (value != 0 && value != 1) return set_err(KOMEGA_E_INVALID, "shift order must be 0 or 1");
      s->ds.shift_order = value;
      break;
    case KOMEGA_T_SHIFT_STEPS:
      if (value < 1 || value > XBLK_MAX)
        return set_err(KOMEGA_E_INVALID, "whole-x steps per block must be in [1, %d]", XBLK_MAX);
      if (s->blk_steps > 0) return set_err(KOMEGA_E_STATE, "a block of steps is pending");
      s->ds.xblk = (s->p.flags & KOMEGA_F_GRAPH) ? 1 : value;
      break;
    default:
      return set_err(KOMEGA_E_INVALID, "unknown tuning knob %d", knob);
  }
  s->drop_graphs();  // captured launches carry the old configuration
  return KOMEGA_OK;
}

extern "C" komega_status komega_get_tuning(const komega_solver* s, int32_t knob, int32_t* value) {
  if (!s || !value) return set_err(KOMEGA_E_INVALID, "null argument");
  switch (knob) {
    case KOMEGA_T_SHIFT_BLOCK: *value = s->ds.shift_block; return KOMEGA_OK;
    case KOMEGA_T_SHIFT_STEPS: *value = s->ds.xblk; return KOMEGA_OK;
    case KOMEGA_T_SHIFT_NT: *value = s->ds.shift_nt; return KOMEGA_OK;
    case KOMEGA_T_SPMV_BLOCKS: *value = s->ds.spmv_blk; return KOMEGA_OK;
    case KOMEGA_T_SHIFT_ORDER: *value = s->ds.shift_order; return KOMEGA_OK;
    default: return set_err(KOMEGA_E_INVALID, "unknown tuning knob %d", knob);
  }
}

// ------------------------------------------------------------- operators
extern "C" komega_status komega_op_stencil3d(komega_op** out, int32_t Lx, int32_t Ly, int32_t Lz, double hop,
                                             const double* eps) {
  if (!out || !eps) return set_err(KOMEGA_E_INVALID, "null argument");
  *out = nullptr;
  if (Lx < 3 || Ly < 3 || Lz < 3) return set_err(KOMEGA_E_INVALID, "stencil edges must be >= 3");
  if (!std::isfinite(hop)) return set_err(KOMEGA_E_INVALID, "hopping must be finite");
  const int64_t M = (int64_t)Lx * Ly * Lz;
  komega_op* op = new (std::nothrow) komega_op();
  if (!op) return set_err(KOMEGA_E_NOMEM, "host allocation failed");
  double* e;
  komega_status rc = dalloc(&e, (size_t)M, op->owned);
  if (rc != KOMEGA_OK) { delete op; return rc; }
  hipError_t he = hipMemcpy(e, eps, sizeof(double) * M, hipMemcpyHostToDevice);
  if (he != hipSuccess) { delete op; return set_err(KOMEGA_E_HIP, "copy of eps failed"); }
  op->d.kind = OP_STENCIL;
  op->d.M = M;
  op->d.Lx = Lx; op->d.Ly = Ly; op->d.Lz = Lz;
  op->d.hop = hop;
  op->d.eps = e;
  *out = op;
  return KOMEGA_OK;
}

extern "C" komega_status komega_op_stencil3d_batch(komega_op** out, int32_t nsys, const int32_t* L, double hop,
                                                   const double* eps) {
  if (!out || !L || !eps) return set_err(KOMEGA_E_INVALID, "null argument");
  *out = nullptr;
  if (nsys < 1 || nsys > 65535) return set_err(KOMEGA_E_INVALID, "need 1 <= nsys <= 65535");
  if (!std::isfinite(hop)) return set_err(KOMEGA_E_INVALID, "hopping must be finite");
  std::vector<int64_t> soff((size_t)nsys + 1, 0);
  std::vector<int2> wl;
  for (int r = 0; r < nsys; ++r) {
    if (L[3 * r] < 3 || L[3 * r + 1] < 3 || L[3 * r + 2] < 3)
      return set_err(KOMEGA_E_INVALID, "cube %d: stencil edges must be >= 3", r);
    const int64_t M = (int64_t)L[3 * r] * L[3 * r + 1] * L[3 * r + 2];
    soff[r + 1] = soff[r] + M;
    for (int g = 0; g < (int)stream_blocks(M); ++g) wl.push_back(make_int2(r, g));
  }
  const int64_t M = soff[nsys];
  komega_op* op = new (std::nothrow) komega_op();
  if (!op) return set_err(KOMEGA_E_NOMEM, "host allocation failed");
  double* e;
  int32_t* Ld;
  int64_t* sd;
  int2* wd;
  komega_status rc = dalloc(&e, (size_t)M, op->owned);
  if (rc == KOMEGA_OK) rc = dalloc(&Ld, (size_t)nsys * 3, op->owned);
  if (rc == KOMEGA_OK) rc = dalloc(&sd, soff.size(), op->owned);
  if (rc == KOMEGA_OK) rc = dalloc(&wd, wl.size(), op->owned);
  if (rc != KOMEGA_OK) { delete op; return rc; }
  hipError_t he = hipMemcpy(e, eps, sizeof(double) * M, hipMemcpyHostToDevice);
  if (he == hipSuccess) he = hipMemcpy(Ld, L, sizeof(int32_t) * 3 * nsys, hipMemcpyHostToDevice);
  if (he == hipSuccess) he = hipMemcpy(sd, soff.data(), sizeof(int64_t) * soff.size(), hipMemcpyHostToDevice);
  if (he == hipSuccess) he = hipMemcpy(wd, wl.data(), sizeof(int2) * wl.size(), hipMemcpyHostToDevice);
  if (he != hipSuccess) { delete op; return set_err(KOMEGA_E_HIP, "copy of the cubes failed"); }
  op->d.kind = OP_STENCIL;
  op->d.M = M;
  op->d.hop = hop;
  op->d.eps = e;
  op->d.nsys = nsys;
  op->d.sysL = Ld;
  op->d.soff = sd;
  op->d.wl = wd;
  op->d.nwl = (int32_t)wl.size();
  op->h_soff = soff;
  *out = op;
  return KOMEGA_OK;
}

extern "C" komega_status komega_op_csr(komega_op** out, int64_t M, const int64_t* rowptr, const int32_t* col,
                                       const double* val, int32_t complex_vals) {
  if (!out || !rowptr || M < 1) return set_err(KOMEGA_E_INVALID, "bad argument");
  *out = nullptr;
  if (rowptr[0] != 0) return set_err(KOMEGA_E_INVALID, "rowptr[0] must be 0");
  for (int64_t i = 0; i < M; ++i)
    if (rowptr[i + 1] < rowptr[i]) return set_err(KOMEGA_E_INVALID, "rowptr must be non-decreasing");
  const int64_t nnz = rowptr[M];
  if (nnz > 0 && (!col || !val)) return set_err(KOMEGA_E_INVALID, "null col/val");
  for (int64_t p = 0; p < nnz; ++p)
    if (col[p] < 0 || col[p] >= M) return set_err(KOMEGA_E_INVALID, "column index out of range at %lld", (long long)p);
  komega_op* op = new (std::nothrow) komega_op();
  if (!op) return set_err(KOMEGA_E_NOMEM, "host allocation failed");
  int64_t* rp;
  int32_t* cd;
  double* vd;
  const size_t vw = complex_vals ? 2 : 1;
  komega_status rc = dalloc(&rp, (size_t)M + 1, op->owned);
  if (rc == KOMEGA_OK) rc = dalloc(&cd, (size_t)(nnz ? nnz : 1), op->owned);
  if (rc == KOMEGA_OK) rc = dalloc(&vd, (size_t)(nnz ? nnz : 1) * vw, op->owned);
  if (rc != KOMEGA_OK) { delete op; return rc; }
  hipError_t he = hipMemcpy(rp, rowptr, sizeof(int64_t) * (M + 1), hipMemcpyHostToDevice);
  if (he == hipSuccess && nnz) he = hipMemcpy(cd, col, sizeof(int32_t) * nnz, hipMemcpyHostToDevice);
  if (he == hipSuccess && nnz) he = hipMemcpy(vd, val, sizeof(double) * nnz * vw, hipMemcpyHostToDevice);
  if (he != hipSuccess) { delete op; return set_err(KOMEGA_E_HIP, "copy of CSR arrays failed"); }
  op->h_rowptr.assign(rowptr, rowptr + M + 1);
  if (nnz) op->h_col.assign(col, col + nnz);
  op->d.kind = OP_CSR;
  op->d.M = M;
  op->d.rowptr = rp;
  op->d.col = cd;
  op->d.val = vd;
  op->d.complex_vals = complex_vals ? 1 : 0;
  *out = op;
  return KOMEGA_OK;
}

static int64_t binom_host(int n, int k) {
  if (k < 0 || k > n) return 0;
  int64_t r = 1;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

extern "C" komega_status komega_op_heisenberg(komega_op** out, int32_t L, int32_t nup, int32_t nb,
                                              const int32_t* bi, const int32_t* bj, const double* J) {
  if (!out || !bi || !bj || !J) return set_err(KOMEGA_E_INVALID, "null argument");
  *out = nullptr;
  if (L < 1 || L > 32 || nup < 0 || nup > L) return set_err(KOMEGA_E_INVALID, "need 1 <= L <= 32, 0 <= nup <= L");
  if (nb < 1 || nb > 256) return set_err(KOMEGA_E_INVALID, "need 1 <= nb <= 256");
  for (int b = 0; b < nb; ++b) {
    if (bi[b] < 0 || bi[b] >= L || bj[b] < 0 || bj[b] >= L || bi[b] == bj[b])
      return set_err(KOMEGA_E_INVALID, "bond %d has bad sites (%d, %d)", b, bi[b], bj[b]);
    if (!std::isfinite(J[b])) return set_err(KOMEGA_E_INVALID, "coupling %d is not finite", b);
  }
  const int64_t M = binom_host(L, nup);
  const int h = L / 2;
  const int nlo = 1 << h, nhi = 1 << (L - h);
  komega_op* op = new (std::nothrow) komega_op();
  if (!op) return set_err(KOMEGA_E_NOMEM, "host allocation failed");
  // bond classes relative to the index split at bit h
  std::vector<uint32_t> lo_m, hb_m;
  std::vector<double> lo_J, hb_J, cr_J;
  std::vector<int32_t> cr_a, cr_c;
  for (int b = 0; b < nb; ++b) {
    const int i = bi[b], j = bj[b];
    if (i < h && j < h) {
      lo_m.push_back((1u << i) | (1u << j));
      lo_J.push_back(J[b]);
    } else if (i >= h && j >= h) {
      hb_m.push_back((1u << (i - h)) | (1u << (j - h)));
      hb_J.push_back(J[b]);
    } else {
      cr_a.push_back(i < h ? i : j);
      cr_c.push_back((i < h ? j : i) - h);
      cr_J.push_back(J[b]);
    }
  }
  int64_t segmax = 0;
  for (int p = 0; p <= L - h; ++p) {
    const int k = nup - p;
    if (k >= 0 && k <= h && binom_host(h, k) > segmax) segmax = binom_host(h, k);
  }
  // the row product's padded lists: low, high, cross, each to whole chunks
  const int pl = heis_pad((int)lo_m.size(), HEIS_CH_LO), ph = heis_pad((int)hb_m.size(), HEIS_CH_HI),
            pc = heis_pad((int)cr_a.size(), HEIS_CH_CR);
  std::vector<uint32_t> rlm((size_t)(pl + ph + pc), 0u);
  std::vector<double> rlj((size_t)(pl + ph + pc), 0.0);
  for (size_t e = 0; e < lo_m.size(); ++e) { rlm[e] = lo_m[e]; rlj[e] = 0.5 * lo_J[e]; }
  for (size_t e = 0; e < hb_m.size(); ++e) { rlm[pl + e] = hb_m[e]; rlj[pl + e] = 0.5 * hb_J[e]; }
  for (size_t e = 0; e < cr_a.size(); ++e) {
    rlm[pl + ph + e] = (1u << cr_a[e]) | (1u << (cr_c[e] + h));
    rlj[pl + ph + e] = 0.5 * cr_J[e];
  }
  // The row product takes its tiles of TPB rows ordered by the popcount of
  // their first row's high part u, then by the inversion count of u (pairs
  // of a set bit below a clear bit), then by position.  A bond on two
  // adjacent high sites swaps two bits of u and changes that count by one, so
  // the partners of a tile's rows lie in tiles taken shortly before or after
  // it, and are read through L2 rather than fetched again from memory (in
  // plain u order a swap of the top bits jumps thousands of tiles away).
  // Any order gives the same q: every row is computed the same way.
  const int64_t ntile = (M + TPB - 1) / TPB;
  std::vector<uint32_t> tord((size_t)ntile);
  {
    std::vector<uint64_t> key((size_t)ntile);
    int64_t off = 0, t = 0;
    for (int u = 0; u < nhi && t < ntile; ++u) {
      const int pu = __builtin_popcount((unsigned)u), need = nup - pu;
      const int64_t n = (need >= 0 && need <= h) ? binom_host(h, need) : 0;
      int ones = 0, inv = 0;
      for (int b = 0; b < L - h; ++b) {
        if ((u >> b) & 1) ++ones;
        else inv += ones;
      }
      for (; t < ntile && t * TPB < off + n; ++t)
        key[(size_t)t] = ((uint64_t)pu << 56) | ((uint64_t)inv << 32) | (uint64_t)t;
      off += n;
    }
    std::sort(key.begin(), key.end());
    for (int64_t e = 0; e < ntile; ++e) tord[(size_t)e] = (uint32_t)(key[(size_t)e] & 0xffffffffu);
  }
  uint32_t *states, *hi, *mask, *lom, *hbm, *koff, *rlmd, *tordd;
  uint16_t *lo, *lst;
  double *Jd, *loJ, *hbJ, *crJ, *rljd;
  int32_t *cra, *crc;
  int64_t *binom, *total;
  int32_t* bad;
  auto cnt = [](size_t n) { return n ? n : (size_t)1; };
  komega_status rc = dalloc(&states, (size_t)M, op->owned);
  if (rc == KOMEGA_OK) rc = dalloc(&hi, (size_t)nhi + 1, op->owned);
  if (rc == KOMEGA_OK) rc = dalloc(&lo, (size_t)nlo, op->owned);
  if (rc == KOMEGA_OK) rc = dalloc(&lst, (size_t)nlo, op->owned);
  if (rc == KOMEGA_OK) rc = dalloc(&koff, (size_t)h + 2, op->owned);
  if (rc == KOMEGA_OK) rc = dalloc(&mask, (size_t)nb, op->owned);
  if (rc == KOMEGA_OK) rc = dalloc(&Jd, (size_t)nb, op->owned);
  if (rc == KOMEGA_OK) rc = dalloc(&lom, cnt(lo_m.size()), op->owned);
  if (rc == KOMEGA_OK) rc = dalloc(&loJ, cnt(lo_m.size()), op->owned);
  if (rc == KOMEGA_OK) rc = dalloc(&hbm, cnt(hb_m.size()), op->owned);
  if (rc == KOMEGA_OK) rc = dalloc(&hbJ, cnt(hb_m.size()), op->owned);
  if (rc == KOMEGA_OK) rc = dalloc(&cra, cnt(cr_a.size()), op->owned);
  if (rc == KOMEGA_OK) rc = dalloc(&crc, cnt(cr_a.size()), op->owned);
  if (rc == KOMEGA_OK) rc = dalloc(&crJ, cnt(cr_a.size()), op->owned);
  if (rc == KOMEGA_OK) rc = dalloc(&rlmd, cnt(rlm.size()), op->owned);
  if (rc == KOMEGA_OK) rc = dalloc(&rljd, cnt(rlj.size()), op->owned);
  if (rc == KOMEGA_OK) rc = dalloc(&tordd, (size_t)ntile, op->owned);
  if (rc == KOMEGA_OK) rc = dalloc(&binom, 33 * 33, op->owned);
  if (rc == KOMEGA_OK) rc = dalloc(&total, 1, op->owned);
  if (rc == KOMEGA_OK) rc = dalloc(&bad, 1, op->owned);
  if (rc != KOMEGA_OK) { delete op; return rc; }
  std::vector<int64_t> bh(33 * 33);
  for (int n = 0; n <= 32; ++n)
    for (int k = 0; k <= 32; ++k) bh[n * 33 + k] = binom_host(n, k);
  // inverse rank table of the low part: the h-bit values of each popcount in
  // ascending order, classes one after another
  std::vector<uint32_t> koffh((size_t)h + 2, 0);
  for (int k = 0; k <= h; ++k) koffh[k + 1] = koffh[k] + (uint32_t)binom_host(h, k);
  std::vector<uint16_t> lsth((size_t)nlo);
  {
    std::vector<uint32_t> fill(koffh.begin(), koffh.end() - 1);
    for (int l = 0; l < nlo; ++l) lsth[fill[__builtin_popcount(l)]++] = (uint16_t)l;
  }
  std::vector<uint32_t> mh(nb);
  for (int b = 0; b < nb; ++b) mh[b] = (1u << bi[b]) | (1u << bj[b]);
  op->d.kind = OP_HEIS;
  op->d.M = M;
  op->d.L = L;
  op->d.nup = nup;
  op->d.nb = nb;
  op->d.h = h;
  op->d.states = states;
  op->d.hi_off = hi;
  op->d.lo_rank = lo;
  op->d.lo_state = lst;
  op->d.lo_koff = koff;
  op->d.bmask = mask;
  op->d.bJ = Jd;
  {
    double js = 0.0;
    for (int b = 0; b < nb; ++b) js += J[b];
    op->d.jq = 0.25 * js;
  }
  op->d.tables_in_lds = (4 * (size_t)nhi + 2 * (size_t)nlo) <= 48 * 1024;
  op->d.nlo = (int32_t)lo_m.size();
  op->d.nhb = (int32_t)hb_m.size();
  op->d.ncr = (int32_t)cr_a.size();
  op->d.lo_m = lom; op->d.lo_J = loJ;
  op->d.hb_m = hbm; op->d.hb_J = hbJ;
  op->d.cr_a = cra; op->d.cr_c = crc; op->d.cr_J = crJ;
  op->d.rl_m = rlmd; op->d.rl_j = rljd;
  op->d.tile_order = tordd;
  op->d.ngroups = nhi;
  op->d.segmax = (int32_t)segmax;
  // group kernel: LDS for the rank table and two staged segments (BiCG)
  op->d.group_kernel = 0;  // row kernel by default (faster on gfx950 for chains)
  op->d.row_groups = heis_row_groups(op->d);
  auto up = [](void* dst, const void* src, size_t bytes) {
    return bytes ? hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice) : hipSuccess;
  };
  int64_t tot = -1;
  int32_t badh = 1;
  hipError_t he = hipMemcpy(binom, bh.data(), sizeof(int64_t) * bh.size(), hipMemcpyHostToDevice);
  if (he == hipSuccess) he = hipMemcpy(mask, mh.data(), sizeof(uint32_t) * nb, hipMemcpyHostToDevice);
  if (he == hipSuccess) he = hipMemcpy(Jd, J, sizeof(double) * nb, hipMemcpyHostToDevice);
  if (he == hipSuccess) he = up(lst, lsth.data(), sizeof(uint16_t) * lsth.size());
  if (he == hipSuccess) he = up(koff, koffh.data(), sizeof(uint32_t) * koffh.size());
  if (he == hipSuccess) he = up(lom, lo_m.data(), sizeof(uint32_t) * lo_m.size());
  if (he == hipSuccess) he = up(loJ, lo_J.data(), sizeof(double) * lo_J.size());
  if (he == hipSuccess) he = up(hbm, hb_m.data(), sizeof(uint32_t) * hb_m.size());
  if (he == hipSuccess) he = up(hbJ, hb_J.data(), sizeof(double) * hb_J.size());
  if (he == hipSuccess) he = up(cra, cr_a.data(), sizeof(int32_t) * cr_a.size());
  if (he == hipSuccess) he = up(crc, cr_c.data(), sizeof(int32_t) * cr_c.size());
  if (he == hipSuccess) he = up(crJ, cr_J.data(), sizeof(double) * cr_J.size());
  if (he == hipSuccess) he = up(rlmd, rlm.data(), sizeof(uint32_t) * rlm.size());
  if (he == hipSuccess) he = up(rljd, rlj.data(), sizeof(double) * rlj.size());
  if (he == hipSuccess) he = up(tordd, tord.data(), sizeof(uint32_t) * tord.size());
  if (he == hipSuccess) he = hipMemset(bad, 0, sizeof(int32_t));
  if (he == hipSuccess) he = launch_heis_setup(op->d, binom, nullptr);
  if (he == hipSuccess) he = launch_heis_hi(op->d, binom, total, nullptr);
  if (he == hipSuccess) he = launch_heis_check(op->d, bad, nullptr);
  if (he == hipSuccess) he = hipMemcpy(&tot, total, sizeof(int64_t), hipMemcpyDeviceToHost);
  if (he == hipSuccess) he = hipMemcpy(&badh, bad, sizeof(int32_t), hipMemcpyDeviceToHost);
  if (he != hipSuccess) { delete op; return set_err(KOMEGA_E_HIP, "Heisenberg set-up failed: %s", hipGetErrorString(he)); }
  if (tot != M || badh != 0) {
    delete op;
    return set_err(KOMEGA_E_INVALID, "basis index tables are inconsistent (total %lld, expected %lld)",
                   (long long)tot, (long long)M);
  }
  *out = op;
  return KOMEGA_OK;
}

extern "C" komega_status komega_op_callback(komega_op** out, int64_t M, komega_apply_fn fn, void* user) {
  if (!out || !fn || M < 1) return set_err(KOMEGA_E_INVALID, "bad argument");
  komega_op* op = new (std::nothrow) komega_op();
  if (!op) return set_err(KOMEGA_E_NOMEM, "host allocation failed");
  op->d.kind = OP_CALLBACK;
  op->d.M = M;
  op->fn = fn;
  op->user = user;
  *out = op;
  return KOMEGA_OK;
}

extern "C" komega_status komega_op_dim(const komega_op* op, int64_t* M) {
  if (!op || !M) return set_err(KOMEGA_E_INVALID, "null argument");
  *M = op->d.M;
  return KOMEGA_OK;
}

extern "C" komega_status komega_op_apply(const komega_op* op, const void* v, void* out, int32_t nvec,
                                         int32_t is_complex, void* stream) {
  if (!op || !v || !out || nvec < 1 || nvec > 65535) return set_err(KOMEGA_E_INVALID, "bad argument");
  if (!is_complex && op->d.kind == OP_CSR && op->d.complex_vals)
    return set_err(KOMEGA_E_INVALID, "complex operator applied to real vectors");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (op->d.kind == OP_CALLBACK) {
    if (op->fn(op->user, v, out, nvec, is_complex, stream) != 0)
      return set_err(KOMEGA_E_INVALID, "operator callback failed");
    return KOMEGA_OK;
  }
  HIPCHK(launch_op_apply(op->d, v, out, nvec, is_complex, st));
  return KOMEGA_OK;
}

extern "C" komega_status komega_op_heisenberg_states(const komega_op* op, uint32_t* states, void* stream) {
  if (!op || !states) return set_err(KOMEGA_E_INVALID, "null argument");
  if (op->d.kind != OP_HEIS) return set_err(KOMEGA_E_INVALID, "not a Heisenberg operator");
  HIPCHK(hipMemcpyAsync(states, op->d.states, sizeof(uint32_t) * op->d.M, hipMemcpyDeviceToDevice,
                        reinterpret_cast<hipStream_t>(stream)));
  return KOMEGA_OK;
}

extern "C" komega_status komega_op_heisenberg_lookup(const komega_op* op, const uint32_t* states, int64_t* idx,
                                                     int64_t n, void* stream) {
  if (!op || !states || !idx || n < 0) return set_err(KOMEGA_E_INVALID, "bad argument");
  if (op->d.kind != OP_HEIS) return set_err(KOMEGA_E_INVALID, "not a Heisenberg operator");
  if (n == 0) return KOMEGA_OK;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  int32_t* bad = nullptr;
  HIPCHK(hipMalloc(&bad, sizeof(int32_t)));
  int32_t badh = 0;
  hipError_t he = hipMemsetAsync(bad, 0, sizeof(int32_t), st);
  if (he == hipSuccess) he = launch_heis_lookup(op->d, states, idx, n, bad, st);
  if (he == hipSuccess) he = hipMemcpyAsync(&badh, bad, sizeof(int32_t), hipMemcpyDeviceToHost, st);
  if (he == hipSuccess) he = hipStreamSynchronize(st);
  (void)hipFree(bad);
  if (he != hipSuccess) return set_err(KOMEGA_E_HIP, "lookup failed: %s", hipGetErrorString(he));
  if (badh) return set_err(KOMEGA_E_INVALID, "a state is outside the sector (index -1 written)");
  return KOMEGA_OK;
}

extern "C" komega_status komega_op_heisenberg_szq(const komega_op* op, const double* w, const void* v, void* out,
                                                  void* stream) {
  if (!op || !w || !v || !out) return set_err(KOMEGA_E_INVALID, "null argument");
  if (op->d.kind != OP_HEIS) return set_err(KOMEGA_E_INVALID, "not a Heisenberg operator");
  zc wh[32];
  for (int j = 0; j < 32; ++j) wh[j] = j < op->d.L ? zmk(w[2 * j], w[2 * j + 1]) : zmk(0.0, 0.0);
  HIPCHK(launch_heis_szq(op->d, wh, v, out, reinterpret_cast<hipStream_t>(stream)));
  return KOMEGA_OK;
}

extern "C" komega_status komega_op_set_variant(komega_op* op, int32_t variant) {
  if (!op) return set_err(KOMEGA_E_INVALID, "null operator");
  if (op->d.kind != OP_HEIS) return set_err(KOMEGA_E_INVALID, "not a Heisenberg operator");
  const bool fits = heis_grp_lds_bytes(op->d, true) <= 64 * 1024;
  switch (variant) {
    case 0:
    case 1: op->d.group_kernel = 0; op->version++; break;
    case 2:
      if (!fits) return set_err(KOMEGA_E_INVALID, "group kernel does not fit in LDS for L = %d", op->d.L);
      op->d.group_kernel = 1;
      op->version++;
      break;
    default: return set_err(KOMEGA_E_INVALID, "unknown variant %d", variant);
  }
  return KOMEGA_OK;
}

// Scratch for partial sums, allocated on the caller's stream with the
// stream-ordered allocator and released after use.
static int grad_groups(int64_t M) {
  int64_t g = (M + TPB - 1) / TPB;
  return (int)(g < 64 ? (g < 1 ? 1 : g) : 64);
}

extern "C" komega_status komega_op_heisenberg_bond_grad(const komega_op* op, const void* w, int64_t ldw,
                                                        const void* x, int64_t ldx, int32_t n, void* out,
                                                        void* stream) {
  if (!op || !w || !x || !out || n < 1 || n > 65535) return set_err(KOMEGA_E_INVALID, "bad argument");
  if (op->d.kind != OP_HEIS) return set_err(KOMEGA_E_INVALID, "not a Heisenberg operator");
  if (ldw < op->d.M || ldx < op->d.M) return set_err(KOMEGA_E_INVALID, "leading dimension smaller than M");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int G = grad_groups(op->d.M);
  double* part = nullptr;
  HIPCHK(hipMallocAsync((void**)&part, sizeof(double) * 2 * (size_t)n * G * op->d.nb, st));
  hipError_t e = launch_bond_grad(op->d, w, ldw, x, ldx, n, part, G, out, st);
  hipError_t e2 = hipFreeAsync(part, st);
  if (e != hipSuccess) return set_err(KOMEGA_E_HIP, "bond contraction failed: %s", hipGetErrorString(e));
  if (e2 != hipSuccess) return set_err(KOMEGA_E_HIP, "free failed: %s", hipGetErrorString(e2));
  return KOMEGA_OK;
}

static komega_status dotc_impl(const void* a, int64_t lda, const void* x, int64_t ldx, int64_t M, int32_t n,
                               void* out, int x32, void* stream) {
  if (!a || !x || !out || M < 1 || n < 1 || n > 65535 || lda < 0 || ldx < M)
    return set_err(KOMEGA_E_INVALID, "bad argument");
  if (lda != 0 && lda < M) return set_err(KOMEGA_E_INVALID, "lda must be 0 or >= M");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int G = grad_groups(M);
  double* part = nullptr;
  HIPCHK(hipMallocAsync((void**)&part, sizeof(double) * 2 * (size_t)n * G, st));
  hipError_t e = launch_dotc(a, lda, x, ldx, M, n, part, G, out, x32, st);
  hipError_t e2 = hipFreeAsync(part, st);
  if (e != hipSuccess) return set_err(KOMEGA_E_HIP, "inner product failed: %s", hipGetErrorString(e));
  if (e2 != hipSuccess) return set_err(KOMEGA_E_HIP, "free failed: %s", hipGetErrorString(e2));
  return KOMEGA_OK;
}

extern "C" komega_status komega_dotc(const void* a, int64_t lda, const void* x, int64_t ldx, int64_t M, int32_t n,
                                     void* out, void* stream) {
  return dotc_impl(a, lda, x, ldx, M, n, out, 0, stream);
}

// ------------------------------------------------- allocation-free projection
// komega_dotc_noalloc keeps the partial sums of k_dotc in this file-scope
// array instead of stream-ordered scratch.  In host code `scratch` names a
// host-side stand-in, never the device copy: the device address is looked up
// once per device (hipGetSymbolAddress, with that device current) and only
// that address is handed to kernels.
constexpr int NOALLOC_GROUPS = 64;  // grad_groups(M) never exceeds this
static __device__ __align__(256) double scratch[2 * (size_t)NOALLOC_GROUPS * KOMEGA_NOALLOC_MAX_VECTORS];
constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_dev[NOALLOC_MAX_DEVICES];

static komega_status scratch_address(double** out) {
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return set_err(KOMEGA_E_INVALID, "device %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return set_err(KOMEGA_E_HIP, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                     hipGetErrorString(e));
    g_scratch_dev[dev] = reinterpret_cast<double*>(p);
  }
  *out = g_scratch_dev[dev];
  return KOMEGA_OK;
}

extern "C" komega_status komega_dotc_noalloc(const void* a, int64_t lda, const void* x, int64_t ldx, int64_t M,
                                             int32_t n, void* out, void* stream) {
  if (!a || !x || !out || M < 1 || n < 1 || lda < 0 || ldx < M)
    return set_err(KOMEGA_E_INVALID, "bad argument");
  if (lda != 0 && lda < M) return set_err(KOMEGA_E_INVALID, "lda must be 0 or >= M");
  if (n > KOMEGA_NOALLOC_MAX_VECTORS)
    return set_err(KOMEGA_E_INVALID, "n = %d exceeds the static scratch limit of %d vectors", n,
                   KOMEGA_NOALLOC_MAX_VECTORS);
  const int G = grad_groups(M);
  if (G > NOALLOC_GROUPS) return set_err(KOMEGA_E_INVALID, "internal: %d groups exceed the scratch layout", G);
  double* part = nullptr;
  TRY(scratch_address(&part));
  // every slot that k_sum_groups reads is written by k_dotc first, so the
  // previous call's contents need no clearing
  hipError_t e = launch_dotc(a, lda, x, ldx, M, n, part, G, out, 0, reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return set_err(KOMEGA_E_HIP, "inner product failed: %s", hipGetErrorString(e));
  return KOMEGA_OK;
}

extern "C" komega_status komega_dotc_c64(const void* a, int64_t lda, const void* x, int64_t ldx, int64_t M,
                                         int32_t n, void* out, void* stream) {
  return dotc_impl(a, lda, x, ldx, M, n, out, 1, stream);
}

extern "C" komega_status komega_onsite_grad(const void* g, const void* w, int64_t ldw, const void* x, int64_t ldx,
                                            int64_t M, int32_t n, void* out, void* stream) {
  if (!g || !w || !x || !out || M < 1 || n < 1 || ldw < M || ldx < M)
    return set_err(KOMEGA_E_INVALID, "bad argument (need M >= 1, n >= 1, ldw, ldx >= M)");
  if ((M + TPB - 1) / TPB > 0x7fffffff) return set_err(KOMEGA_E_INVALID, "M too large");
  HIPCHK(launch_onsite_grad(g, w, ldw, x, ldx, M, n, out, reinterpret_cast<hipStream_t>(stream)));
  return KOMEGA_OK;
}

extern "C" komega_status komega_stream_probe(const void* src, void* dst, int64_t bytes, int32_t kind, void* stream) {
  if (!src || !dst || bytes < 16 || bytes % 16 != 0 || (kind != 0 && kind != 1))
    return set_err(KOMEGA_E_INVALID, "need src, dst, bytes >= 16 a multiple of 16, kind 0 (copy) or 1 (read)");
  HIPCHK(launch_stream_probe(src, dst, bytes / 16, kind, reinterpret_cast<hipStream_t>(stream)));
  return KOMEGA_OK;
}

extern "C" int32_t komega_stream_probe_groups(void) { return stream_probe_groups(); }

extern "C" komega_status komega_contour_moments(const void* x, int32_t nz, int64_t M, int32_t nrhs,
                                                int32_t nk, const double* w, void* s, void* stream) {
  if (!x || !w || !s || nz < 1 || M < 1 || nrhs < 1 || nrhs > 65535 || nk < 1 || nk > 16)
    return set_err(KOMEGA_E_INVALID, "bad argument (need 1 <= nk <= 16)");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  void* wd = nullptr;
  const size_t wb = sizeof(double) * 2 * (size_t)nk * nz;
  HIPCHK(hipMallocAsync(&wd, wb, st));
  hipError_t e = hipMemcpyAsync(wd, w, wb, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = launch_moments(x, nz, M, nrhs, nk, wd, s, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFreeAsync(wd, st);
  if (e != hipSuccess) return set_err(KOMEGA_E_HIP, "moments failed: %s", hipGetErrorString(e));
  return KOMEGA_OK;
}

extern "C" komega_status komega_op_destroy(komega_op* op) {
  if (!op) return KOMEGA_OK;
  (void)hipDeviceSynchronize();
  delete op;
  return KOMEGA_OK;
}

// ---------------------------------------------------------------- strings
extern "C" const char* komega_strerror(komega_status code) {
  switch (code) {
    case KOMEGA_OK: return "ok";
    case KOMEGA_CONVERGED: return "converged";
    case KOMEGA_E_INVALID: return "invalid argument";
    case KOMEGA_E_BREAKDOWN: return "seed breakdown (rho or alpha denominator vanished)";
    case KOMEGA_E_SHIFT_BREAKDOWN: return "shift breakdown (pi vanished)";
    case KOMEGA_E_MAXITER: return "iteration limit reached";
    case KOMEGA_E_HIP: return "HIP runtime error";
    case KOMEGA_E_STATE: return "call out of order";
    case KOMEGA_E_NONFINITE: return "non-finite scalar";
    case KOMEGA_E_NOMEM: return "out of device memory";
    default: return "unknown status";
  }
}

extern "C" const char* komega_last_error(void) { return g_err.c_str(); }
