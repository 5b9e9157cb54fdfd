// Host side of libf3r: the C ABI of include/f3r.h, set-up, the level
// engine of the nested solver and hipGraph capture of the inner levels.
//
// The outermost FGMRES level runs on the host-visible stream and reads one
// pinned word per iteration (the Givens residual estimate), the only
// device-to-host synchronisation of an iteration (Sec. 5.2: everything but
// the convergence check runs on the GPU).  One call of the second level
// (F2 with everything below it) is a fixed kernel sequence: the data-
// dependent decisions (breakdown, non-finite fallback) are taken on the
// device through flags, and the Richardson update schedule of Alg. 1 is a
// function of the call counter, which the host knows.  So each F2 call is
// recorded once per update pattern as a hipGraph and replayed.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "f3r.h"
#include "host.h"
#include "kernels.h"
#include "krylov.h"
#include "setup.h"

using namespace f3r;

namespace {

struct LevelRT {
  f3r_level cfg{};
  int pv = T64, pa = T64, q = T64, zt = T64;
  bool alias0 = false;  // V_0 is the parent's basis vector (same storage type)
  void* V = nullptr;    // m+1 basis vectors (type pv)
  void* Z = nullptr;    // m directions (type zt)
  void* tmp = nullptr;  // one vector (type pv), M application of a last FGMRES level
  LevelLayout L;
  double* S = nullptr;
  int* I = nullptr;
  HistOut hist;         // inner FGMRES level: residual estimates of every call
  // Richardson
  void* rt = nullptr;
  void* ry = nullptr;
  void* rr = nullptr;
  void* rz[2] = {nullptr, nullptr};
  void* rv = nullptr;   // the level's input rounded to its precision (a Richardson
                        // level whose preconditioner is the next level)
  double* omega = nullptr;
  double* wcur = nullptr;
  int64_t* cntr_dev = nullptr;
};

// Richardson schedule of one enqueue: update flag and poison flag per call
struct RSched {
  std::vector<char> upd, poison;
  size_t pos = 0;
};
// the schedules of every Richardson level of one enqueue (indexed by level)
struct RScheds {
  RSched lev[F3R_MAX_LEVELS];
};

}  // namespace

struct f3r_handle {
  int device = 0;
  hipStream_t st = nullptr;
  hipStream_t cap = nullptr;
  f3r_params p{};
  int64_t n = 0, nnz = 0;
  // device matrix
  SellDesc A;
  uint32_t* off = nullptr;
  void* idx = nullptr;
  uint16_t* kd = nullptr;
  uint16_t* kd_true = nullptr;  // diagonal-aligned format: true diagonal positions
  int32_t* ci = nullptr;        // slice-offset format: CSR columns (read-back)
  IluDesc ilu;                  // block-Jacobi ILU(0) schedule when M is ILU
  int ilu_used = 0;             // ILU sweep forms launched since set-up
  uint32_t* kdr = nullptr;
  int32_t* rp = nullptr;  // CSR row pointers, kept for debug read-back
  double* a64 = nullptr;
  void* ah[4] = {};
  void* mv[4] = {};
  bool m_shared = true;
  double gd[4] = {1, 1, 1, 1};
  double* s = nullptr;
  int64_t padded = 0;
  // levels
  std::vector<LevelRT> lev;
  int rich = -1;  // the innermost level when it is a Richardson level (it applies M), else -1
  std::vector<int> rlevs;  // every Richardson level (each keeps its own weights, Sec. 4.3)
  int64_t rcnt[F3R_MAX_LEVELS] = {1, 1, 1, 1, 1, 1, 1, 1};  // host copies of each level's c_ntr
  void* partials = nullptr;
  double* one = nullptr;   // device constant 1.0
  double* tmp64 = nullptr;  // n doubles
  double* tmp64b = nullptr;
  double* hpin = nullptr;  // pinned host words
  std::map<std::string, hipGraphExec_t> graphs;
  std::vector<hipGraph_t> graph_objs;
  // several independent systems as the diagonal blocks of one matrix (see
  // SysLayout): rows of system s start at sys_row0[s] (a multiple of 1024)
  // and its first sys_n[s] rows are its own (the rest are identity rows)
  int nsys = 1;
  std::vector<int64_t> sys_row0, sys_n;
  double* Sall = nullptr;  // per-system level scalars, nsys x dS
  int* Iall = nullptr;     // per-system level flags and counters, nsys x dI
  int64_t dS = 0, dI = 0;
  double* ibn = nullptr;   // device: 1 / ||b_s|| per system
  int* mask = nullptr;     // device: nsys ints (systems to hold)
  // stacked systems: row ranges on the device, the caller's vector pointers
  // and the stacked right-hand side and solution
  int64_t* row0_dev = nullptr;
  int64_t* nrows_dev = nullptr;
  double** ptrs_dev = nullptr;
  double* bcat = nullptr;
  double* xcat = nullptr;
  int base_prec = T64;  // storage of M in the comparison FGMRES
  // comparison solvers: ten work vectors and the scalar slots
  double* kv = nullptr;
  double* ks = nullptr;
  std::vector<std::vector<double>> history;  // per system
  // stats of the last solve
  int64_t graph_launches = 0;
  // kernel probe: event pairs around every launch of one kernel
  int probe = 0;
  std::vector<hipEvent_t> ev;
  size_t ev_used = 0;
  double probe_ms = 0;
  int64_t probe_n = 0;
  double setup_ms = 0;
  // shapes (10 x rows per lane + entry chunk) of the W sweep, the G sweep
  // and the Richardson residual
  int kr[3] = {44, 44, 44};
  double tune_ms = 0;
  DevAllocs al;

  void* dalloc(size_t bytes) { return al.get(bytes); }
};

// format in use and bits of its per-entry index (0: none, offsets per slice)
static int32_t layout_of(const SellDesc& A) {
  if (A.idx16 == 2) return F3R_LAYOUT_SLICE;
  return A.dell_w ? F3R_LAYOUT_DIAG : F3R_LAYOUT_SELL;
}
static int32_t idx_bits_of(const SellDesc& A) { return A.idx16 == 2 ? 0 : (A.idx16 ? 16 : 32); }
static const int32_t* soff_of(const f3r_handle* h) {
  return h->A.idx16 == 2 ? (const int32_t*)h->A.idx : nullptr;
}


// address of this device's copy of the fixed scratch (defined with it below)
static hipError_t scratch_address(int device, void** out);

namespace {

void destroy_graphs(f3r_handle* h);

double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

size_t tsz(int t) { return type_size(t); }
void* vec_at(void* base, int t, int64_t j, int64_t n) {
  return (char*)base + (size_t)j * (size_t)n * tsz(t);
}

bool prec_ok(int p) { return p >= F3R_FP64 && p <= F3R_BF16; }

// the inner levels are recorded and replayed as hipGraphs only on request
bool use_graphs(const f3r_params& p) { return (p.flags & F3R_USE_GRAPH) && !(p.flags & F3R_NO_GRAPH); }

f3r_status check_params(const f3r_params* p) {
  if (!p || p->nlev < 1 || p->nlev > F3R_MAX_LEVELS) return F3R_ERR_ARG;
  if (p->lev[0].kind != F3R_FGMRES || p->lev[0].prec_a != F3R_FP64 || p->lev[0].prec_v != F3R_FP64)
    return F3R_ERR_ARG;
  if (p->lev[0].m < 1 || p->lev[0].m > 1000) return F3R_ERR_ARG;
  for (int d = 1; d < p->nlev; d++) {
    const f3r_level& l = p->lev[d];
    if (l.m < 1 || l.m > 64 || !prec_ok(l.prec_a) || !prec_ok(l.prec_v)) return F3R_ERR_ARG;
    // a Richardson level below the second; one that is not innermost hands
    // its vectors to the next level, whose vectors have its precision
    if (l.kind == F3R_RICHARDSON && d < 2) return F3R_ERR_ARG;
    if (l.kind == F3R_RICHARDSON && d + 1 < p->nlev && p->lev[d + 1].prec_v != l.prec_v) return F3R_ERR_ARG;
    if (l.kind != F3R_FGMRES && l.kind != F3R_RICHARDSON) return F3R_ERR_ARG;
    // matrix no wider than the vectors, narrow vectors only with equal matrix
    if (l.prec_v == F3R_FP64 && l.prec_a != F3R_FP64) return F3R_ERR_ARG;
    if (l.prec_v == F3R_FP32 && l.prec_a == F3R_FP64) return F3R_ERR_ARG;
    if ((l.prec_v == F3R_FP16 || l.prec_v == F3R_BF16) && l.prec_a != l.prec_v) return F3R_ERR_ARG;
    // a level's vectors are no wider than its parent's
    const int pp = p->lev[d - 1].prec_v;
    auto width = [](int t) { return t == F3R_FP64 ? 3 : t == F3R_FP32 ? 2 : 1; };
    if (width(l.prec_v) > width(pp)) return F3R_ERR_ARG;
    if (d >= 2 && l.prec_v != pp && width(l.prec_v) == width(pp)) return F3R_ERR_ARG;
  }
  if (!prec_ok(p->prec_m)) return F3R_ERR_ARG;
  const int plast = p->lev[p->nlev - 1].prec_v;
  auto width = [](int t) { return t == F3R_FP64 ? 3 : t == F3R_FP32 ? 2 : 1; };
  if (width(p->prec_m) > width(plast)) return F3R_ERR_ARG;
  if (width(plast) == 1 && p->prec_m != plast) return F3R_ERR_ARG;
  if (!(p->alpha > 0.0) || !std::isfinite(p->alpha)) return F3R_ERR_ARG;
  if (p->c < 0 || p->max_outer < 1) return F3R_ERR_ARG;
  if (p->m_identity != 0) return F3R_ERR_ARG;  // M = I is not provided
  int nrich = 0;
  for (int d = 1; d < p->nlev; d++) nrich += p->lev[d].kind == F3R_RICHARDSON;
  if (nrich > 1 && p->poison_call > 0) return F3R_ERR_ARG;  // the test hook needs one Richardson level
  if (p->layout < F3R_LAYOUT_AUTO || p->layout > F3R_LAYOUT_SLICE) return F3R_ERR_ARG;
  if (p->m_kind != F3R_M_SGS && p->m_kind != F3R_M_ILU) return F3R_ERR_ARG;
  if (p->m_kind == F3R_M_ILU && p->ilu_blocks < 1) return F3R_ERR_ARG;
  if (p->rows_per_lane != -1 && p->rows_per_lane != 0 && p->rows_per_lane != 1 &&
      p->rows_per_lane != 2 && p->rows_per_lane != 4)
    return F3R_ERR_ARG;
  if (p->entry_chunk != 0 && p->rows_per_lane <= 0) return F3R_ERR_ARG;
  if (p->entry_chunk != 0) {
    const int code = 10 * p->rows_per_lane + p->entry_chunk;
    const int plast = p->lev[p->nlev - 1].prec_v;
    const bool narrow_v = plast == F3R_FP16 || plast == F3R_BF16;
    const bool any3 = narrow_v || p->layout == F3R_LAYOUT_SLICE;
    if (!(code == 18 || code == 24 || code == 44 || ((code == 23 || code == 43) && any3)))
      return F3R_ERR_ARG;
  }
  return F3R_OK;
}

// output type of level d's preconditioner call (type of its Z vectors)
int z_type(const f3r_params& p, int d) {
  if (d == 0) return T64;
  if (d + 1 < p.nlev) return p.lev[d + 1].prec_v;
  return p.lev[d].prec_v;  // M applied in the level's own vector precision
}

void alloc_levels(f3r_handle* h) {
  const f3r_params& p = h->p;
  const int64_t n = h->n;
  h->lev.assign(p.nlev, LevelRT{});
  h->rich = -1;
  h->rlevs.clear();
  h->dS = 0;
  h->dI = 0;
  std::vector<int64_t> soff((size_t)p.nlev, 0), ioff((size_t)p.nlev, 0);
  for (int d = 0; d < p.nlev; d++) {
    LevelRT& L = h->lev[d];
    L.cfg = p.lev[d];
    L.pv = p.lev[d].prec_v;
    L.pa = p.lev[d].prec_a;
    L.q = q_of(L.pv);
    L.zt = z_type(p, d);
    const int m = L.cfg.m;
    if (L.cfg.kind == F3R_FGMRES) {
      L.alias0 = d >= 2 && p.lev[d - 1].prec_v == L.pv;
      L.V = h->dalloc((size_t)(m + 1) * n * tsz(L.pv));
      L.Z = h->dalloc((size_t)m * n * tsz(L.zt));
      if (d + 1 == p.nlev) L.tmp = h->dalloc((size_t)n * tsz(L.pv));
      L.L.init(m);
      if (d >= 1 && h->nsys == 1) {
        // room for 1,000 outermost iterations of calls of this level
        int64_t per = 1;
        for (int e = 1; e <= d; e++) per *= p.lev[e].m;
        L.hist.cap = std::min<int64_t>(1000 * per, (int64_t)1 << 22);
        L.hist.p = (double*)h->dalloc((size_t)L.hist.cap * sizeof(double));
      }
      soff[d] = h->dS;
      ioff[d] = h->dI;
      h->dS += L.L.total;
      h->dI += level_ints(m);
    } else {
      if (d + 1 == p.nlev) h->rich = d;
      else L.rv = h->dalloc((size_t)n * tsz(L.pv));
      h->rlevs.push_back(d);
      L.rt = h->dalloc((size_t)n * tsz(L.pv));
      L.ry = h->dalloc((size_t)n * tsz(L.pv));
      L.rr = h->dalloc((size_t)n * tsz(L.pv));
      L.rz[0] = h->dalloc((size_t)n * tsz(L.pv));
      L.rz[1] = h->dalloc((size_t)n * tsz(L.pv));
      soff[d] = h->dS;  // omega_1..64, then w_cur
      h->dS += 65;
      L.cntr_dev = (int64_t*)h->dalloc(sizeof(int64_t));
    }
  }
  // the scalars and flags of every level of every system in two arrays, so
  // that system s's state is at a fixed distance from system 0's
  const size_t ns = (size_t)h->nsys;
  h->Sall = (double*)h->dalloc(ns * (size_t)h->dS * sizeof(double));
  h->Iall = (int*)h->dalloc(ns * (size_t)std::max<int64_t>(h->dI, 1) * sizeof(int));
  HIPCHK(hipMemsetAsync(h->Sall, 0, ns * (size_t)h->dS * sizeof(double), h->st));
  HIPCHK(hipMemsetAsync(h->Iall, 0, ns * (size_t)std::max<int64_t>(h->dI, 1) * sizeof(int), h->st));
  for (int d = 0; d < p.nlev; d++) {
    LevelRT& L = h->lev[d];
    if (L.cfg.kind == F3R_FGMRES) {
      L.S = h->Sall + soff[d];
      L.I = h->Iall + ioff[d];
    } else {
      L.omega = h->Sall + soff[d];
      L.wcur = L.omega + 64;
    }
  }
  h->A.sys.dS = h->dS;
  h->A.sys.dI = h->dI;
  h->ibn = (double*)h->dalloc(ns * sizeof(double));
  h->mask = (int*)h->dalloc(ns * sizeof(int));
  for (int d : h->rlevs) {
    const LevelRT& R = h->lev[d];
    HIPCHK(set_omega(h->st, h->A.sys, R.omega, R.cfg.m,
                     R.q == T32 ? (double)(float)p.omega_init : p.omega_init));
  }
}

// ---------------------------------------------------------------------------
// level engine
// ---------------------------------------------------------------------------
struct Ctx {
  f3r_handle* h;
  hipStream_t st;
  RScheds* rs;
};

// HIP events around the launches of the probed kernel (direct launches on
// the solve's stream only)
// Probe: each launch of the probed kernel is made kProbeReps times in a row
// (every probed kernel rewrites the same output from the same inputs) between
// one pair of events, so the cost of the event pair is spread over the
// repeats; probe_ms / probe_launches is the time of one launch.
constexpr int kProbeReps = 4;

void probe_drain(f3r_handle* h) {
  for (size_t i = 0; i + 1 < h->ev_used; i += 2) {
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, h->ev[i], h->ev[i + 1]));
    h->probe_ms += ms;
    h->probe_n += kProbeReps;
  }
  h->ev_used = 0;
}
// returns how many times the caller makes the launch
int probe_begin(Ctx& c, int id) {
  f3r_handle* h = c.h;
  if (h->probe != id || c.st != h->st) return 1;
  if (h->ev_used + 2 > h->ev.size()) {
    HIPCHK(hipStreamSynchronize(h->st));
    probe_drain(h);
    while (h->ev.size() < 512) {
      hipEvent_t e;
      HIPCHK(hipEventCreate(&e));
      h->ev.push_back(e);
    }
  }
  HIPCHK(hipEventRecord(h->ev[h->ev_used], h->st));
  return kProbeReps;
}
void probe_end(Ctx& c, int id) {
  f3r_handle* h = c.h;
  if (h->probe != id || c.st != h->st) return;
  HIPCHK(hipEventRecord(h->ev[h->ev_used + 1], h->st));
  h->ev_used += 2;
}
void probe_collect(f3r_handle* h) {
  if (!h->probe || h->ev_used == 0) return;
  HIPCHK(hipStreamSynchronize(h->st));
  probe_drain(h);
}

struct OutSpec {
  void* ptr = nullptr;   // output vector (or base when cur is set)
  const double* s = nullptr;
  const int* cur = nullptr;
  int* fb = nullptr;     // non-finite flag of the parent's column (base when cur is set)
};

// Gram-Schmidt step with nv dots whose finalisation runs inside the update
// kernel: one system (the batched layout sums per system), fp32 arithmetic
// (measured: with fp64 levels the fused kernel made fp64-F3R 15% slower)
bool fuse_dots(const f3r_handle* h, int nv, int q) { return !h->A.sys.blk && nv <= 16 && q == T32; }

void enqueue_rich(Ctx& c, int d, const Basis& vin, const int* stop, void* out, int* fb);
void enqueue_fgmres(Ctx& c, int d, const Basis& vin, const void* alias_raw, const int* pstop,
                    const OutSpec& out, bool force_entry);

const void* m_values(f3r_handle* h, int& tm, int& neg) {
  tm = h->p.prec_m;
  if (h->m_shared) {
    neg = 1;
    return h->ah[tm];
  }
  neg = 0;
  return h->mv[tm];
}

void enqueue_rich(Ctx& c, int d, const Basis& vin, const int* stop, void* out, int* fb) {
  f3r_handle* h = c.h;
  LevelRT& R = h->lev[d];
  const int tr = R.pv;
  const int m = R.cfg.m;
  RSched& rs = c.rs->lev[d];
  const bool upd = rs.upd[rs.pos] != 0;
  const bool poison = rs.poison[rs.pos] != 0;
  rs.pos++;
  const bool inner = d + 1 == h->p.nlev;  // the innermost level applies M
  int tm = T64, neg = 0;
  const void* mv = inner ? m_values(h, tm, neg) : nullptr;
  const double gd = inner ? h->gd[tm] : 1.0;
  const void* av = h->ah[R.pa];
  const void* zprev = nullptr;
  const int64_t nb = n_blocks(h->n);
  if (!inner) {
    // v = the input rounded to the level's precision, which the next level
    // receives as its right-hand side in the first step
    HIPCHK(entry_cast(c.st, h->A.sys, h->n, vin, R.rv, tr, h->partials, stop));
  }
  for (int k = 0; k < m; k++) {
    const bool last = k == m - 1;
    void* zk = last ? out : R.rz[k & 1];
    int* zfb = last ? fb : nullptr;
    Basis rsrc;
    if (k == 0) {
      rsrc = vin;
    } else {
      const int nr = inner ? probe_begin(c, F3R_PROBE_R_RESIDUAL) : 1;
      for (int r = 0; r < nr; r++)
        HIPCHK(rich_residual(c.st, h->A, av, R.pa, vin, zprev, R.rr, tr, stop, h->kr[2]));
      if (inner) probe_end(c, F3R_PROBE_R_RESIDUAL);
      rsrc.raw = R.rr;
      rsrc.type = tr;
    }
    if (!inner) {
      // y = the next level applied to r (Sec. 4.3: Richardson at several
      // levels, each with its own weights), then the update of z
      Basis cin;
      cin.raw = k == 0 ? R.rv : R.rr;
      cin.type = tr;
      if (k == 0) HIPCHK(cntr_advance(c.st, R.cntr_dev));
      const LevelRT& C = h->lev[d + 1];
      if (C.cfg.kind == F3R_FGMRES) {
        OutSpec o;
        o.ptr = R.ry;
        enqueue_fgmres(c, d + 1, cin, nullptr, stop, o, true);
      } else {
        enqueue_rich(c, d + 1, cin, stop, R.ry, nullptr);
      }
      if (!upd) {
        HIPCHK(rich_zupdate(c.st, h->A.sys, h->n, k == 0 ? nullptr : zprev, R.ry, tr, R.omega + k, zk,
                            zfb, stop));
      } else {
        HIPCHK(rich_tdots(c.st, h->A, av, R.pa, R.ry, tr, rsrc, h->partials, stop));
        HIPCHK(rich_omega(c.st, h->A.sys, q_of(tr), h->partials, nb, R.omega + k, R.wcur, R.cntr_dev,
                          h->p.c, stop));
        HIPCHK(rich_zupdate(c.st, h->A.sys, h->n, k == 0 ? nullptr : zprev, R.ry, tr, R.wcur, zk, zfb,
                            stop));
      }
      zprev = zk;
      continue;
    }
    const int nw = probe_begin(c, F3R_PROBE_M_LOWER);
    for (int r = 0; r < nw; r++)  // the call counter advances once
      HIPCHK(m_apply_w(c.st, h->A, mv, tm, neg, rsrc, R.rt, tr, stop,
                       k == 0 && r == 0 ? R.cntr_dev : nullptr, h->kr[0]));
    probe_end(c, F3R_PROBE_M_LOWER);
    if (!upd) {
      const int ng = probe_begin(c, F3R_PROBE_M_UPPER);
      for (int r = 0; r < ng; r++)
        HIPCHK(m_apply_g(c.st, h->A, mv, tm, neg, gd, R.rt, tr, k == 0 ? 1 : 2, R.omega + k, zprev, zk,
                         tr, nullptr, zfb, stop, nullptr, h->kr[1]));
      probe_end(c, F3R_PROBE_M_UPPER);
    } else {
      HIPCHK(m_apply_g(c.st, h->A, mv, tm, neg, gd, R.rt, tr, 0, nullptr, nullptr, R.ry, tr, nullptr,
                       nullptr, stop, nullptr, h->kr[1]));
      HIPCHK(rich_tdots(c.st, h->A, av, R.pa, R.ry, tr, rsrc, h->partials, stop));
      HIPCHK(rich_omega(c.st, h->A.sys, q_of(tr), h->partials, nb, R.omega + k, R.wcur, R.cntr_dev,
                        h->p.c, stop));
      HIPCHK(rich_zupdate(c.st, h->A.sys, h->n, k == 0 ? nullptr : zprev, R.ry, tr, R.wcur, zk, zfb,
                          stop));
    }
    zprev = zk;
  }
  if (poison) HIPCHK(fill_nan(c.st, out, tr, 1, fb));
}

// z = M v for a last FGMRES level (vectors in the level's precision)
void enqueue_m(Ctx& c, int d, const Basis& vin, const int* stop, void* out, int* fb) {
  f3r_handle* h = c.h;
  LevelRT& L = h->lev[d];
  int tm, neg;
  const void* mv = m_values(h, tm, neg);
  HIPCHK(m_apply_w(c.st, h->A, mv, tm, neg, vin, L.tmp, L.pv, stop, nullptr));
  HIPCHK(m_apply_g(c.st, h->A, mv, tm, neg, h->gd[tm], L.tmp, L.pv, 0, nullptr, nullptr, out, L.pv,
                   nullptr, fb, stop));
}

void enqueue_fgmres(Ctx& c, int d, const Basis& vin, const void* alias_raw, const int* pstop,
                    const OutSpec& out, bool force_entry) {
  f3r_handle* h = c.h;
  const f3r_params& p = h->p;
  LevelRT& L = h->lev[d];
  const int64_t n = h->n;
  const int64_t nb = n_blocks(n);
  const int m = L.cfg.m;
  const bool aliased = L.alias0 && !force_entry;
  const bool has_child = d + 1 < p.nlev;
  LevelRT* C = has_child ? &h->lev[d + 1] : nullptr;
  const bool child_alias = C && C->cfg.kind == F3R_FGMRES && C->alias0;
  ChildInit ci_child;
  if (child_alias) {
    ci_child.S = C->S;
    ci_child.I = C->I;
    ci_child.m = C->cfg.m;
    ci_child.g = C->L.g;
    ci_child.scale = C->L.scale;
    ci_child.beta = C->L.beta;
  }
  const void* v0 = aliased ? alias_raw : L.V;
  if (!aliased) {
    ChildInit self{L.S, L.I, m, L.L.g, L.L.scale, L.L.beta};
    HIPCHK(entry_cast(c.st, h->A.sys, n, vin, L.V, L.pv, h->partials, pstop));
    HIPCHK(entry_finalize(c.st, h->A.sys, L.q, h->partials, nb, self,
                          child_alias ? &ci_child : nullptr, pstop));
  } else if (child_alias) {
    HIPCHK(child_init0(c.st, h->A.sys, L.S, L.I, L.L, ci_child));
  }
  const void* vb = vec_at(L.V, L.pv, 1, n);
  const int* stop = L.I + I_STOP;
  for (int j = 0; j < m; j++) {
    const void* vj = j == 0 ? v0 : vec_at(L.V, L.pv, j, n);
    void* zj = vec_at(L.Z, L.zt, j, n);
    Basis bj;
    bj.raw = vj;
    bj.type = L.pv;
    bj.scale = L.S + L.L.scale + j;
    int* fbj = L.I + I_FB + j;
    if (has_child) {
      if (C->cfg.kind == F3R_FGMRES) {
        OutSpec o;
        o.ptr = zj;
        o.fb = fbj;
        enqueue_fgmres(c, d + 1, bj, vj, stop, o, false);
      } else {
        enqueue_rich(c, d + 1, bj, stop, zj, fbj);
      }
    } else {
      enqueue_m(c, d, bj, stop, zj, fbj);
    }
    const int pid = d == 1 ? F3R_PROBE_SPMV_L1 : d == 2 ? F3R_PROBE_SPMV_L2 : -1;
    double* hcol = L.S + L.L.H + (int64_t)j * (m + 1);
    const int ns_ = probe_begin(c, pid);
    for (int r = 0; r < ns_; r++)
      HIPCHK(spmv_dots(c.st, h->A, h->ah[L.pa], L.pa, zj, L.zt, &bj, fbj, vec_at(L.V, L.pv, j + 1, n),
                       L.pv, v0, vb, j + 1, h->partials, stop));
    probe_end(c, pid);
    if (fuse_dots(h, j + 1, L.q)) {
      // dots finalised inside the update; its norm partials follow the dots
      void* npart = (char*)h->partials + (size_t)(j + 1) * (size_t)nb * tsz(L.q);
      int64_t nnb = 0;
      HIPCHK(axpy_norm_fin(c.st, n, vec_at(L.V, L.pv, j + 1, n), L.pv, v0, vb, j + 1, h->partials, nb,
                           L.S + L.L.scale, hcol, npart, &nnb, stop));
      HIPCHK(givens(c.st, h->A.sys, L.q, npart, nnb, L.S, L.I, L.L, j, j == m - 1, nullptr, nullptr,
                    child_alias ? &ci_child : nullptr, 0.0, L.hist));
    } else {
      HIPCHK(finalize_sums(c.st, h->A.sys, L.q, h->partials, nb, j + 1, L.S + L.L.scale, hcol, stop));
      HIPCHK(axpy_norm(c.st, h->A.sys, n, vec_at(L.V, L.pv, j + 1, n), L.pv, v0, vb, j + 1, hcol,
                       L.S + L.L.scale, h->partials, stop));
      HIPCHK(givens(c.st, h->A.sys, L.q, h->partials, nb, L.S, L.I, L.L, j, j == m - 1, nullptr,
                    nullptr, child_alias ? &ci_child : nullptr, 0.0, L.hist));
    }
  }
  LevelBasis lb;
  lb.v0 = v0;
  lb.vb = vb;
  lb.type = L.pv;
  lb.scales = L.S + L.L.scale;
  HIPCHK(combine(c.st, h->A.sys, n, L.Z, L.zt, L.pv, L.S + L.L.y, L.I + I_MEFF, m, out.ptr, out.s,
                 out.cur, 0, &lb, L.I + I_FB, out.fb, pstop));
}

// Set-up autotuner: times the candidate shapes (rows per lane and entry
// chunk) of the three sweeps of the Richardson level on this matrix and
// keeps the fastest of each.  The sweeps have no reductions, so the shape
// changes only the time, never a result.
void autotune(f3r_handle* h) {
  const int fixed = h->p.rows_per_lane;
  if (fixed > 0) {
    const int code = h->p.entry_chunk ? 10 * fixed + h->p.entry_chunk : fixed == 1 ? 18 : fixed == 2 ? 24 : 44;
    h->kr[0] = h->kr[1] = h->kr[2] = code;
    return;
  }
  if (h->rich < 0) return;
  if (h->ilu.blocks > 0) {
    // block-Jacobi ILU(0): M runs its own sweeps; only the residual's shape
    // matters, the row-length rule below picks it
    h->kr[0] = h->kr[1] = 24;
    h->kr[2] = 18;
    return;
  }
  if (fixed == 0) {
    // Rule from measurements of whole solves (stencils with 3-13 entries
    // per half row, elasticity with 41): rows with at most four entries on
    // a side of the diagonal take two rows per lane and one chunk for the
    // side (three entries with narrow vectors), longer rows one row per
    // lane and chunks of eight; the residual sweeps whole rows, one per
    // lane, chunks of eight.  Timing the candidates at set-up (-1) measures
    // them on warm caches, which the solve does not see.
    const LevelRT& R = h->lev[h->rich];
    const bool narrow = tsz(R.pv) == 2;
    int lower, upper;
    if (h->A.dell_w) {
      lower = h->A.dell_kd;
      upper = h->A.dell_w - 1 - h->A.dell_kd;
    } else {
      lower = upper = (int)((h->padded / std::max<int64_t>(h->n, 1) - 1) / 2);
    }
    // (the slice-offset format reads every position of a chunk: a chunk
    // longer than the side reads values it does not sum, so chunks of three
    // serve three entries in every precision there; with its short per-entry
    // code, narrow vectors there take four rows per lane, one round of waves
    // over the chip, and the residual chunks of four, or one chunk of seven
    // over rows of seven entries: measured on the 128^3 Poisson matrix, 12.8
    // against 13.2 ms a solve, then 12.15 against 12.3 ms for the chunk of
    // seven)
    const bool slice = h->A.idx16 == 2;
    const bool four = slice && narrow;
    auto pick = [&](int side) {
      if (side <= 3 && (narrow || slice)) return four ? 43 : 23;
      return side <= 4 ? (four ? 44 : 24) : 18;
    };
    h->kr[0] = pick(lower);
    h->kr[1] = pick(upper);
    h->kr[2] = !four ? 18 : h->A.dell_w == 7 ? 47 : h->A.dell_w <= 8 ? 44 : 18;
    return;
  }
  const double t0 = now_ms();
  LevelRT& R = h->lev[h->rich];
  const int tr = R.pv;
  int tm, neg;
  const void* mv = m_values(h, tm, neg);
  const double gd = h->gd[tm];
  const int64_t n = h->n;
  // The candidates run on the matrix without its system layout: the
  // pointers passed here (a constant 1.0 as scale and weight, scratch
  // vectors) are not per-system state, so no kernel may shift them.
  SellDesc At = h->A;
  At.sys = SysLayout{};
  // inputs with ordinary finite values (byte pattern 0x3C in every format)
  HIPCHK(hipMemsetAsync(R.rr, 0x3C, (size_t)n * tsz(tr), h->st));
  HIPCHK(hipMemsetAsync(R.rz[0], 0x3C, (size_t)n * tsz(tr), h->st));
  const int tin = h->p.lev[h->rich - 1].prec_v;
  HIPCHK(hipMemsetAsync(h->tmp64, 0x3C, (size_t)n * tsz(tin), h->st));
  Basis vec;
  vec.raw = R.rr;
  vec.type = tr;
  Basis basis;
  basis.raw = h->tmp64;
  basis.type = tin;
  basis.scale = h->one;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  const int cand[5] = {18, 24, 44, 23, 43};
  const int ncand = tsz(tr) == 2 || h->A.idx16 == 2 ? 5 : 3;
  for (int f = 0; f < 3; f++) {
    auto launch = [&](int kr) {
      if (f == 0) {
        // the two W sweeps of a Richardson call: from the level's input
        // basis (wider, scaled) and from the residual
        HIPCHK(m_apply_w(h->st, At, mv, tm, neg, basis, R.rt, tr, nullptr, nullptr, kr));
        HIPCHK(m_apply_w(h->st, At, mv, tm, neg, vec, R.rt, tr, nullptr, nullptr, kr));
      } else if (f == 1)
        HIPCHK(m_apply_g(h->st, At, mv, tm, neg, gd, R.rr, tr, 2, h->one, R.rz[0], R.rt, tr,
                         nullptr, nullptr, nullptr, nullptr, kr));
      else
        HIPCHK(rich_residual(h->st, At, h->ah[R.pa], R.pa, basis, R.rz[0], R.rt, tr, nullptr, kr));
    };
    // the residual also tries one chunk over rows of seven entries (narrow
    // vectors in the slice-offset format)
    int cf[6], nf = 0;
    for (int c = 0; c < ncand; c++) cf[nf++] = cand[c];
    if (f == 2 && tsz(tr) == 2 && h->A.idx16 == 2 && h->A.dell_w == 7) cf[nf++] = 47;
    // three interleaved rounds; each candidate keeps its best round
    float best[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int c = 0; c < nf; c++) launch(cf[c]);
    for (int round = 0; round < 3; round++) {
      for (int c = 0; c < nf; c++) {
        HIPCHK(hipEventRecord(e0, h->st));
        for (int i = 0; i < 4; i++) launch(cf[c]);
        HIPCHK(hipEventRecord(e1, h->st));
        HIPCHK(hipEventSynchronize(e1));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        if (round == 0 || ms < best[c]) best[c] = ms;
      }
    }
    int bc = 0;
    for (int c = 1; c < nf; c++)
      if (best[c] < best[bc]) bc = c;
    h->kr[f] = cf[bc];
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  h->tune_ms = now_ms() - t0;
}

// initial weight in the arithmetic of Richardson level d
double omega_init_q(const f3r_handle* h, int d) {
  const double w = h->p.omega_init;
  return h->lev[d].q == T32 ? (double)(float)w : w;
}

// calls of level d made by one call of level `from` (from <= d)
int64_t calls_between(const f3r_params& p, int from, int d) {
  int64_t c = 1;
  for (int e = from; e < d; e++) c *= p.lev[e].m;
  return c;
}

// Update and poison flags of every call, in order, of each Richardson level
// at or below `from` during one call of level `from` (Alg. 1: an update when
// the level's c_ntr is a multiple of c).  executed_inner: calls of the
// innermost Richardson level made before (the poison test hook counts them).
RScheds make_scheds(const f3r_handle* h, int from, int64_t executed_inner) {
  RScheds rs;
  for (int d : h->rlevs) {
    if (d < from) continue;
    const int64_t ncalls = calls_between(h->p, from, d);
    RSched& r = rs.lev[d];
    r.upd.assign((size_t)ncalls, 0);
    r.poison.assign((size_t)ncalls, 0);
    for (int64_t i = 0; i < ncalls; i++) {
      const int64_t cn = h->rcnt[d] + i;
      r.upd[(size_t)i] = h->p.c > 0 && cn % h->p.c == 0;
      r.poison[(size_t)i] = d == h->rich && h->p.poison_call > 0 && executed_inner + i + 1 == h->p.poison_call;
    }
  }
  return rs;
}

std::string sched_key(const RScheds& rs) {
  std::string k;
  for (int d = 0; d < F3R_MAX_LEVELS; d++) {
    const RSched& r = rs.lev[d];
    if (r.upd.empty()) continue;
    k += 'L';
    k += (char)('0' + d);
    for (size_t i = 0; i < r.upd.size(); i++) {
      k += r.upd[i] ? '1' : '0';
      k += r.poison[i] ? '1' : '0';
    }
  }
  return k;
}

// sets the weights of every Richardson level at or below `from` whose next
// call is its first (Alg. 1: omega_k = 1 at the first call), and after the
// enqueue advances the host counters by the calls it made
void scheds_begin(f3r_handle* h, hipStream_t st, int from) {
  for (int d : h->rlevs)
    if (d >= from && h->rcnt[d] == 1)
      HIPCHK(set_omega(st, h->A.sys, h->lev[d].omega, h->lev[d].cfg.m, omega_init_q(h, d)));
}
void scheds_end(f3r_handle* h, const RScheds& rs, int from, int64_t* upd) {
  for (int d : h->rlevs) {
    if (d < from) continue;
    const RSched& r = rs.lev[d];
    int64_t u = 0;
    for (char f : r.upd) u += f;
    if (upd) upd[d] = u;
    h->rcnt[d] += (int64_t)r.upd.size();
  }
}

// ---------------------------------------------------------------------------
// the outermost level
// ---------------------------------------------------------------------------
struct SolveStats {
  int outer = 0, restarts = 0;
  int64_t m_calls = 0;
  int64_t rc[F3R_MAX_LEVELS] = {}, ru[F3R_MAX_LEVELS] = {};  // Richardson calls and updates per level
  double est = 0, relres = 0;
};

// one call of the second level for every system; upd[d]: the Richardson
// calls of level d in it that update the weights
void f2_call(f3r_handle* h, SolveStats& ss, bool use_graph, int64_t* upd) {
  LevelRT& L0 = h->lev[0];
  RScheds rs = make_scheds(h, 1, h->rich >= 0 ? ss.rc[h->rich] : 0);
  scheds_begin(h, h->st, 1);
  Basis in;
  in.raw = L0.V;
  in.type = T64;
  in.scale = L0.S + L0.L.scale;
  in.s = h->s;
  in.cur = L0.I + I_CUR;
  in.stride = h->n;
  OutSpec out;
  out.ptr = L0.Z;
  out.s = h->s;
  out.cur = L0.I + I_CUR;
  out.fb = L0.I + I_FB;
  if (use_graph) {
    const std::string key = sched_key(rs);
    auto it = h->graphs.find(key);
    hipGraphExec_t ex = nullptr;
    if (it == h->graphs.end()) {
      HIPCHK(hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal));
      Ctx c{h, h->cap, &rs};
      try {
        enqueue_fgmres(c, 1, in, nullptr, L0.I + I_STOP, out, false);
      } catch (...) {
        hipGraph_t g;
        (void)hipStreamEndCapture(h->cap, &g);
        throw;
      }
      hipGraph_t g;
      HIPCHK(hipStreamEndCapture(h->cap, &g));
      HIPCHK(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0));
      h->graph_objs.push_back(g);
      h->graphs[key] = ex;
    } else {
      ex = it->second;
    }
    HIPCHK(hipGraphLaunch(ex, h->st));
    h->graph_launches++;
  } else {
    Ctx c{h, h->st, &rs};
    enqueue_fgmres(c, 1, in, nullptr, L0.I + I_STOP, out, false);
  }
  scheds_end(h, rs, 1, upd);
  for (int d : h->rlevs) {
    ss.rc[d] += calls_between(h->p, 1, d);
    ss.ru[d] += upd[d];
  }
}

void baseline_prec(f3r_handle* h) {
  // P(v) = S M64 (S v), every value fp64 (the comparison solver of Sec. 5)
  LevelRT& L0 = h->lev[0];
  Basis in;
  in.raw = L0.V;
  in.type = T64;
  in.scale = L0.S + L0.L.scale;
  in.s = h->s;
  in.cur = L0.I + I_CUR;
  in.stride = h->n;
  // M's values in the storage the call asked for (fp64 arithmetic)
  const int tm = h->base_prec;
  const void* mv = h->m_shared ? h->ah[tm] : h->mv[tm];
  const int neg = h->m_shared ? 1 : 0;
  HIPCHK(m_apply_w(h->st, h->A, mv, tm, neg, in, h->tmp64, T64, L0.I + I_STOP, nullptr));
  HIPCHK(m_apply_g(h->st, h->A, mv, tm, neg, h->gd[tm], h->tmp64, T64, 3, nullptr, nullptr, L0.Z,
                   T64, h->s, L0.I + I_FB, L0.I + I_STOP, L0.I + I_CUR));
}

// Per-system record of one solve.
struct SysStat {
  f3r_status status = F3R_NOT_CONVERGED;
  int outer = 0, restarts = 0;
  int64_t m_calls = 0;
  int64_t rc[F3R_MAX_LEVELS] = {}, ru[F3R_MAX_LEVELS] = {};  // Richardson calls and updates per level
  double est = 0, relres = 0;
  bool hold = false;   // finished (or failed): its rows are skipped by every kernel
  bool run = false;    // iterating in the current cycle
};

// Marks on the device the systems held since the last call (held[] is the
// host's copy of what the device already knows).  Nothing is enqueued when
// no system changed.
void upload_holds(f3r_handle* h, const std::vector<SysStat>& ss, std::vector<int>& held) {
  bool changed = false;
  std::vector<int> m((size_t)h->nsys, 0);
  for (int s = 0; s < h->nsys; s++) {
    if (ss[(size_t)s].hold && !held[(size_t)s]) {
      m[(size_t)s] = 1;
      held[(size_t)s] = 1;
      changed = true;
    }
  }
  if (!changed) return;
  // ordered after the stream's earlier work, complete before m goes away
  HIPCHK(hipStreamSynchronize(h->st));
  HIPCHK(hipMemcpy(h->mask, m.data(), m.size() * sizeof(int), hipMemcpyHostToDevice));
  HIPCHK(sys_hold(h->st, h->A.sys, h->lev[0].I, h->mask));
}

// The outermost FGMRES(m1) of every system in lockstep: one F2 call and one
// outermost step per iteration for all systems that are still iterating;
// a system whose estimate reaches tol (or breaks down) stops its rows on
// the device and waits for the end of the cycle, where x += Z y and the true
// residual are formed for every system at once.  With one system this is
// exactly the restarted FGMRES of Sec. 4.2 with the host check of Sec. 5.2.
f3r_status outer_solve(f3r_handle* h, const double* b, double* x, double tol, int m1, int max_outer,
                       bool baseline, bool use_graph, f3r_info* infos) {
  const int64_t n = h->n;
  const int64_t nb = n_blocks(n);
  const int ns = h->nsys;
  const SysLayout& sl = h->A.sys;
  LevelRT& L0 = h->lev[0];
  if (m1 > L0.cfg.m) return F3R_ERR_ARG;
  const double t0 = now_ms();
  SolveStats gs;
  std::vector<SysStat> ss((size_t)ns);
  std::vector<int> held((size_t)ns, 0);  // holds the device knows of
  h->history.assign((size_t)ns, std::vector<double>());
  h->graph_launches = 0;
  h->probe = h->p.probe_kernel;
  h->probe_ms = 0;
  h->probe_n = 0;
  h->ev_used = 0;
  if (h->probe) use_graph = false;
  int64_t m_per_outer = 1;
  if (!baseline)
    for (int d = 1; d < h->p.nlev; d++) m_per_outer *= h->p.lev[d].m;
  if (!(h->p.flags & F3R_USE_X0)) HIPCHK(hipMemsetAsync(x, 0, (size_t)n * sizeof(double), h->st));
  if (!h->rlevs.empty() && !(h->p.flags & F3R_PERSIST_WEIGHTS)) {
    // synchronous: the host copies of the counters change as calls are enqueued
    HIPCHK(hipStreamSynchronize(h->st));
    for (int d : h->rlevs) {
      h->rcnt[d] = 1;
      HIPCHK(hipMemcpy(h->lev[d].cntr_dev, &h->rcnt[d], sizeof(int64_t), hipMemcpyHostToDevice));
    }
  }
  // every level's flags and counters of every system start clear
  HIPCHK(hipMemsetAsync(h->Iall, 0, (size_t)ns * (size_t)h->dI * sizeof(int), h->st));
  HIPCHK(dot64_to_host(h->st, sl, n, b, b, h->partials, h->hpin));
  HIPCHK(hipStreamSynchronize(h->st));
  std::vector<double> ibn((size_t)ns, 0.0);
  for (int s = 0; s < ns; s++) {
    SysStat& q = ss[(size_t)s];
    const double bnorm = std::sqrt(h->hpin[4 * s]);
    if (bnorm == 0.0) {
      const int64_t r0 = h->sys_row0[(size_t)s];
      HIPCHK(hipMemsetAsync(x + r0, 0, (size_t)h->sys_n[(size_t)s] * sizeof(double), h->st));
      q.status = F3R_OK;
      q.hold = true;
    } else if (!std::isfinite(bnorm)) {
      q.status = F3R_ERR_ARG;
      q.hold = true;
    } else {
      ibn[(size_t)s] = 1.0 / bnorm;
    }
  }
  HIPCHK(hipMemcpy(h->ibn, ibn.data(), ibn.size() * sizeof(double), hipMemcpyHostToDevice));
  upload_holds(h, ss, held);
  auto any_open = [&]() {
    for (const SysStat& q : ss)
      if (!q.hold) return true;
    return false;
  };
  if (any_open()) {
    HIPCHK(residual64(h->st, h->A, h->a64, x, b, (double*)L0.V, h->partials));
    HIPCHK(residual_finalize(h->st, sl, h->partials, nb, L0.S, L0.I, L0.L, h->ibn, h->hpin));
    HIPCHK(hipStreamSynchronize(h->st));
    for (int s = 0; s < ns; s++) {
      SysStat& q = ss[(size_t)s];
      if (q.hold) continue;
      q.relres = h->hpin[4 * s];
      if (q.relres < tol) {
        q.status = F3R_OK;
        q.hold = true;
      }
    }
    upload_holds(h, ss, held);
  }
  while (any_open()) {
    int omax = 0;
    for (SysStat& q : ss) {
      q.run = !q.hold;
      if (q.run) omax = std::max(omax, q.outer);
    }
    const int len = std::min(m1, max_outer - omax);
    int it = 0;
    for (int j = 0; j < len; j++) {
      int64_t upd[F3R_MAX_LEVELS] = {};
      if (baseline)
        baseline_prec(h);
      else
        f2_call(h, gs, use_graph, upd);
      void* zj = vec_at(L0.Z, T64, j, n);
      Basis bj;
      bj.raw = vec_at(L0.V, T64, j, n);
      bj.type = T64;
      bj.scale = L0.S + L0.L.scale + j;
      Ctx c0{h, h->st, nullptr};
      const int n0 = probe_begin(c0, F3R_PROBE_SPMV_L0);
      for (int r = 0; r < n0; r++)
        HIPCHK(spmv_dots(h->st, h->A, h->a64, T64, zj, T64, &bj, L0.I + I_FB + j,
                         vec_at(L0.V, T64, j + 1, n), T64, L0.V, vec_at(L0.V, T64, 1, n), j + 1,
                         h->partials, L0.I + I_STOP));
      probe_end(c0, F3R_PROBE_SPMV_L0);
      double* hcol = L0.S + L0.L.H + (int64_t)j * (L0.cfg.m + 1);
      if (fuse_dots(h, j + 1, T64)) {
        void* npart = (double*)h->partials + (size_t)(j + 1) * (size_t)nb;
        int64_t nnb = 0;
        HIPCHK(axpy_norm_fin(h->st, n, vec_at(L0.V, T64, j + 1, n), T64, L0.V, vec_at(L0.V, T64, 1, n),
                             j + 1, h->partials, nb, L0.S + L0.L.scale, hcol, npart, &nnb,
                             L0.I + I_STOP));
        HIPCHK(givens(h->st, sl, T64, npart, nnb, L0.S, L0.I, L0.L, j, 0, h->ibn, h->hpin, nullptr,
                      tol));
      } else {
        HIPCHK(finalize_sums(h->st, sl, T64, h->partials, nb, j + 1, L0.S + L0.L.scale, hcol,
                             L0.I + I_STOP));
        HIPCHK(axpy_norm(h->st, sl, n, vec_at(L0.V, T64, j + 1, n), T64, L0.V, vec_at(L0.V, T64, 1, n),
                         j + 1, hcol, L0.S + L0.L.scale, h->partials, L0.I + I_STOP));
        HIPCHK(givens(h->st, sl, T64, h->partials, nb, L0.S, L0.I, L0.L, j, 0, h->ibn, h->hpin, nullptr,
                      tol));
      }
      HIPCHK(hipStreamSynchronize(h->st));
      probe_collect(h);
      it++;
      bool more = false;
      for (int s = 0; s < ns; s++) {
        SysStat& q = ss[(size_t)s];
        if (!q.run) continue;
        q.outer++;
        if (!baseline)
          for (int d : h->rlevs) {
            q.rc[d] += calls_between(h->p, 1, d);
            q.ru[d] += upd[d];
          }
        q.m_calls += baseline ? 1 : m_per_outer;
        q.est = h->hpin[4 * s];
        h->history[(size_t)s].push_back(q.est);
        const int flags = (int)h->hpin[4 * s + 1];
        if (flags & 2) {
          q.status = F3R_ERR_BREAKDOWN;
          q.run = false;
          q.hold = true;  // x is left as it is (no update from a broken cycle)
        } else if (q.est < tol || (flags & 1)) {
          q.run = false;
        }
        more = more || q.run;
      }
      if (!more) break;
    }
    upload_holds(h, ss, held);
    HIPCHK(backsolve(h->st, sl, T64, L0.S, L0.I, L0.L));
    LevelBasis lb;
    lb.v0 = L0.V;
    lb.vb = vec_at(L0.V, T64, 1, n);
    lb.type = T64;
    lb.scales = L0.S + L0.L.scale;
    HIPCHK(combine(h->st, sl, n, L0.Z, T64, T64, L0.S + L0.L.y, L0.I + I_MEFF, L0.cfg.m, x, nullptr,
                   nullptr, 1, &lb, L0.I + I_FB, nullptr, L0.I + I_HOLD));
    HIPCHK(residual64(h->st, h->A, h->a64, x, b, (double*)L0.V, h->partials));
    HIPCHK(residual_finalize(h->st, sl, h->partials, nb, L0.S, L0.I, L0.L, h->ibn, h->hpin));
    HIPCHK(hipStreamSynchronize(h->st));
    for (int s = 0; s < ns; s++) {
      SysStat& q = ss[(size_t)s];
      if (q.hold) continue;
      q.relres = h->hpin[4 * s];
      if (!std::isfinite(q.relres)) {
        q.status = F3R_ERR_BREAKDOWN;
        q.hold = true;
      } else if (q.relres < tol) {
        q.status = F3R_OK;
        q.hold = true;
      } else {
        q.restarts++;
        if (q.outer >= max_outer || it == 0) q.hold = true;  // not converged
      }
    }
    if (any_open()) upload_holds(h, ss, held);
  }
  const double t1 = now_ms();
  probe_collect(h);
  f3r_status worst = F3R_OK;
  auto severity = [](f3r_status st) { return st == F3R_OK ? 0 : st == F3R_NOT_CONVERGED ? 1 : 2 - st; };
  for (const SysStat& q : ss)
    if (severity(q.status) > severity(worst)) worst = q.status;
  if (infos) {
    // per-system counters of every level
    std::vector<int> iall((size_t)ns * (size_t)h->dI);
    HIPCHK(hipMemcpy(iall.data(), h->Iall, iall.size() * sizeof(int), hipMemcpyDeviceToHost));
    const f3r_params& p = h->p;
    for (int s = 0; s < ns; s++) {
      const SysStat& q = ss[(size_t)s];
      f3r_info* info = infos + s;
      std::memset(info, 0, sizeof(*info));
      info->status = q.status;
      info->outer_iters = q.outer;
      info->restarts = q.restarts;
      info->m_calls = q.m_calls;
      info->spmv[0] = q.outer;
      if (!baseline) {
        int64_t per = 1;  // calls of level d per outermost iteration
        for (int d = 1; d < p.nlev; d++) {
          if (p.lev[d].kind == F3R_FGMRES)
            info->spmv[d] = (int64_t)q.outer * per * p.lev[d].m;
          else
            info->spmv[d] = q.rc[d] * (p.lev[d].m - 1) + q.ru[d] * p.lev[d].m;
          per *= p.lev[d].m;
        }
        for (int d : h->rlevs) info->r_calls += q.rc[d];
      }
      int64_t fbk = 0, brk = 0;
      for (size_t d = 0; d < h->lev.size(); d++) {
        if (!h->lev[d].I) continue;
        const int* I = iall.data() + (size_t)s * (size_t)h->dI + (size_t)(h->lev[d].I - h->Iall);
        fbk += I[I_FALLBACKS];
        brk += I[I_BREAKDOWNS];
      }
      info->fallbacks = fbk;
      info->breakdowns = brk;
      info->relres_est = q.est;
      info->relres_true = q.relres;
      info->setup_ms = h->setup_ms;
      info->solve_ms = t1 - t0;
      info->graph_launches = h->graph_launches;
      info->idx_bits = idx_bits_of(h->A);
      info->sell_c = 64;
      info->probe_ms = h->probe_ms;
      info->probe_launches = h->probe_n;
      info->padded_nnz = h->padded;
      info->layout = layout_of(h->A);
      info->ilu_sweep = h->ilu_used;
      for (int f = 0; f < 3; f++) {
        info->rows_per_lane[f] = h->kr[f] / 10;
        info->entry_chunk[f] = h->kr[f] % 10;
      }
      info->tune_ms = h->tune_ms;
    }
  }
  return worst;
}

template <class F> f3r_status guarded(f3r_handle* h, f3r_info* info, F&& f) {
  try {
    return f();
  } catch (const StatusErr& e) {
    if (info) info->status = e.s;
    return e.s;
  } catch (const DevErr& e) {
    if (info) {
      info->status = F3R_ERR_DEVICE;
      info->hip_error = (int32_t)e.e;
    }
    (void)h;
    return F3R_ERR_DEVICE;
  } catch (...) {
    return F3R_ERR_DEVICE;
  }
}

void destroy_graphs(f3r_handle* h) {
  for (auto& kv : h->graphs) (void)hipGraphExecDestroy(kv.second);
  for (auto g : h->graph_objs) (void)hipGraphDestroy(g);
  h->graphs.clear();
  h->graph_objs.clear();
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

void f3r_params_default(f3r_params* p, int32_t variant) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->prec_m = F3R_FP16;
  p->c = 64;
  p->alpha = 1.0;
  p->omega_init = 1.0;
  p->max_outer = 300;
  p->ilu_blocks = 112;  // Sec. 5.1 (block-Jacobi ILU(0), when selected)
  p->nlev = 4;
  const int ms[4] = {100, 8, 4, 2};
  int pa[4] = {F3R_FP64, F3R_FP32, F3R_FP16, F3R_FP16};
  int pv[4] = {F3R_FP64, F3R_FP32, F3R_FP32, F3R_FP16};
  if (variant == F3R_VARIANT_FP32) {
    for (int d = 1; d < 4; d++) pa[d] = pv[d] = F3R_FP32;
    p->prec_m = F3R_FP32;
  } else if (variant == F3R_VARIANT_FP64) {
    for (int d = 0; d < 4; d++) pa[d] = pv[d] = F3R_FP64;
    p->prec_m = F3R_FP64;
  } else if (variant == F3R_VARIANT_BF16) {
    pa[2] = pa[3] = F3R_BF16;
    pv[3] = F3R_BF16;
    p->prec_m = F3R_BF16;
  }
  for (int d = 0; d < 4; d++) {
    p->lev[d].kind = d == 3 ? F3R_RICHARDSON : F3R_FGMRES;
    p->lev[d].m = ms[d];
    p->lev[d].prec_a = pa[d];
    p->lev[d].prec_v = pv[d];
  }
  if (variant == F3R_VARIANT_FGMRES64) {
    p->nlev = 1;
    p->lev[0].m = 64;
    p->prec_m = F3R_FP64;
    p->max_outer = 19200;
  }
}

const char* f3r_status_str(f3r_status s) {
  switch (s) {
    case F3R_OK: return "ok";
    case F3R_NOT_CONVERGED: return "not converged";
    case F3R_ERR_ARG: return "invalid argument";
    case F3R_ERR_MATRIX: return "invalid matrix";
    case F3R_ERR_RANGE: return "value out of range of a narrow format";
    case F3R_ERR_NOMEM: return "out of memory";
    case F3R_ERR_DEVICE: return "HIP device error";
    case F3R_ERR_BREAKDOWN: return "non-finite value in the outermost level";
  }
  return "unknown status";
}

void f3r_destroy(f3r_handle* h) {
  if (!h) return;
  (void)hipSetDevice(h->device);
  if (h->st) (void)hipStreamSynchronize(h->st);
  destroy_graphs(h);
  for (hipEvent_t e : h->ev) (void)hipEventDestroy(e);
  h->al.release_all();
  if (h->hpin) (void)hipHostFree(h->hpin);
  if (h->cap) (void)hipStreamDestroy(h->cap);
  delete h;
}

}  // extern "C"

namespace {
// Set-up of one matrix holding nsys >= 1 systems on its diagonal; row0 (nsys
// + 1 entries) and nrows describe the systems (see SysLayout).
f3r_status setup_impl(const f3r_csr* A, const f3r_params* p, void* hip_stream, int nsys,
                      const std::vector<int64_t>& row0, const std::vector<int64_t>& nrows,
                      bool stacked, f3r_handle** out) {
  if (!out) return F3R_ERR_ARG;
  *out = nullptr;
  if (!A || !A->row_ptr || !A->col_idx || !A->val || A->n <= 0 || A->nnz < A->n) return F3R_ERR_ARG;
  f3r_status ps = check_params(p);
  if (ps != F3R_OK) return ps;
  f3r_handle* h = new f3r_handle();
  h->p = *p;
  h->n = A->n;
  h->nnz = A->nnz;
  h->st = (hipStream_t)hip_stream;
  const double t0 = now_ms();
  f3r_status st = guarded(h, nullptr, [&]() -> f3r_status {
    HIPCHK(hipGetDevice(&h->device));
    {
      // the device's copy of the fixed scratch of f3r_apply_m_static
      void* sp = nullptr;
      HIPCHK(scratch_address(h->device, &sp));
    }
    HIPCHK(hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking));
    // fp64 copy: fp64 levels and the comparison solver
    const bool need[4] = {true, false, false, false};
    MatrixDev m;
    const f3r_status bs = build_matrix(h->st, A, p, need, h->al, m);
    if (bs != F3R_OK) return bs;
    const int64_t n = A->n;
    h->A = m.A;
    h->off = (uint32_t*)m.A.off;
    h->idx = (void*)m.A.idx;
    h->kd = (uint16_t*)m.A.kd;
    h->kd_true = m.kd_true;
    h->ci = m.ci;
    h->ilu = m.ilu;
    if (h->ilu.blocks > 0) {
      h->ilu.used = &h->ilu_used;
      h->A.ilu = &h->ilu;
    }
    h->kdr = (uint32_t*)m.A.kdr;
    h->rp = m.rp;
    h->a64 = m.a64;
    for (int t = 0; t < 4; t++) {
      h->ah[t] = m.ah[t];
      h->mv[t] = m.mv[t];
      h->gd[t] = m.gd[t];
    }
    h->m_shared = m.m_shared;
    h->s = m.s;
    h->padded = m.padded;
    h->nsys = nsys;
    h->sys_row0 = row0;
    h->sys_n = nrows;
    if (stacked) {
      // 1024-row block -> system, and each system's first block
      const int64_t nblk = n / kSysAlign;
      std::vector<int> blk((size_t)nblk), b0((size_t)nsys + 1);
      for (int sy = 0; sy < nsys; sy++) {
        b0[(size_t)sy] = (int)(row0[(size_t)sy] / kSysAlign);
        for (int64_t k = row0[(size_t)sy] / kSysAlign; k < row0[(size_t)sy + 1] / kSysAlign; k++)
          blk[(size_t)k] = sy;
      }
      b0[(size_t)nsys] = (int)nblk;
      int* dblk = (int*)h->dalloc(blk.size() * sizeof(int));
      int* db0 = (int*)h->dalloc(b0.size() * sizeof(int));
      // synchronous: the host vectors end with this block
      HIPCHK(hipStreamSynchronize(h->st));
      HIPCHK(hipMemcpy(dblk, blk.data(), blk.size() * sizeof(int), hipMemcpyHostToDevice));
      HIPCHK(hipMemcpy(db0, b0.data(), b0.size() * sizeof(int), hipMemcpyHostToDevice));
      h->A.sys.blk = dblk;
      h->A.sys.b0 = db0;
      h->A.sys.nsys = nsys;
      h->row0_dev = (int64_t*)h->dalloc(row0.size() * sizeof(int64_t));
      h->nrows_dev = (int64_t*)h->dalloc(nrows.size() * sizeof(int64_t));
      h->ptrs_dev = (double**)h->dalloc((size_t)nsys * sizeof(double*));
      h->bcat = (double*)h->dalloc((size_t)n * sizeof(double));
      h->xcat = (double*)h->dalloc((size_t)n * sizeof(double));
      HIPCHK(hipMemcpy(h->row0_dev, row0.data(), row0.size() * sizeof(int64_t), hipMemcpyHostToDevice));
      HIPCHK(hipMemcpy(h->nrows_dev, nrows.data(), nrows.size() * sizeof(int64_t),
                       hipMemcpyHostToDevice));
    }
    // workspaces
    int maxdots = p->lev[0].m + 2;
    maxdots = std::max(maxdots, 66);
    h->partials = h->dalloc((size_t)maxdots * (size_t)n_blocks(n) * sizeof(double));
    h->tmp64 = (double*)h->dalloc((size_t)n * 8);
    h->tmp64b = (double*)h->dalloc((size_t)n * 8);
    h->one = (double*)h->dalloc(sizeof(double));
    const double one = 1.0;
    HIPCHK(hipMemcpyAsync(h->one, &one, sizeof(double), hipMemcpyHostToDevice, h->st));
    HIPCHK(hipHostMalloc((void**)&h->hpin, (4 * (size_t)h->nsys + 16) * sizeof(double),
                         hipHostMallocDefault));
    std::memset(h->hpin, 0, (4 * (size_t)h->nsys + 16) * sizeof(double));
    alloc_levels(h);
    autotune(h);
    HIPCHK(hipStreamSynchronize(h->st));
    return F3R_OK;
  });
  h->setup_ms = now_ms() - t0;
  if (st != F3R_OK) {
    f3r_destroy(h);
    return st;
  }
  *out = h;
  return F3R_OK;
}

}  // namespace

extern "C" {

f3r_status f3r_setup(const f3r_csr* A, const f3r_params* p, void* hip_stream, f3r_handle** out) {
  if (!out) return F3R_ERR_ARG;
  *out = nullptr;
  if (!A || A->n <= 0) return F3R_ERR_ARG;
  return setup_impl(A, p, hip_stream, 1, {0, A->n}, {A->n}, false, out);
}

f3r_status f3r_solve(f3r_handle* h, const double* b, double* x, double tol,
                     const f3r_params* lo, f3r_info* info) {
  if (!h || !b || !x || !(tol > 0.0)) return F3R_ERR_ARG;
  if (h->p.nlev < 2) {
    // a one-level nest is FGMRES(m1) + M on the fp64 values
    return guarded(h, info, [&]() {
      HIPCHK(hipSetDevice(h->device));
      return outer_solve(h, b, x, tol, h->p.lev[0].m, h->p.max_outer, true, false, info);
    });
  }
  f3r_params saved = h->p;
  if (lo) {
    if (lo->nlev != h->p.nlev) return F3R_ERR_ARG;
    for (int d = 0; d < lo->nlev; d++)
      if (lo->lev[d].m != h->p.lev[d].m || lo->lev[d].prec_a != h->p.lev[d].prec_a ||
          lo->lev[d].prec_v != h->p.lev[d].prec_v || lo->lev[d].kind != h->p.lev[d].kind)
        return F3R_ERR_ARG;
    if (lo->c < 0 || lo->max_outer < 1) return F3R_ERR_ARG;
    h->p.c = lo->c;
    h->p.omega_init = lo->omega_init;
    h->p.max_outer = lo->max_outer;
    h->p.flags = lo->flags;
    h->p.poison_call = lo->poison_call;
    h->p.probe_kernel = lo->probe_kernel;
    // the ILU backward sweep overwrites its input, so it cannot be repeated
    if (h->ilu.blocks > 0 && h->p.probe_kernel == F3R_PROBE_M_UPPER) {
      h->p = saved;
      return F3R_ERR_ARG;
    }
    if (h->p.c != saved.c || h->p.poison_call != saved.poison_call) destroy_graphs(h);
  }
  f3r_status s = guarded(h, info, [&]() {
    HIPCHK(hipSetDevice(h->device));
    return outer_solve(h, b, x, tol, h->p.lev[0].m, h->p.max_outer, false,
                       use_graphs(h->p), info);
  });
  if (lo) {
    if (h->p.c != saved.c || h->p.poison_call != saved.poison_call) destroy_graphs(h);
    h->p = saved;
  }
  return s;
}

f3r_status f3r_fgmres_solve(f3r_handle* h, const double* b, double* x, double tol, int32_t m,
                            int32_t max_iter, int32_t prec_m, f3r_info* info) {
  if (!h || !b || !x || !(tol > 0.0) || m < 1 || max_iter < 1 || !prec_ok(prec_m))
    return F3R_ERR_ARG;
  if (m > h->p.lev[0].m) return F3R_ERR_ARG;
  if (!(h->m_shared ? h->ah[prec_m] : h->mv[prec_m])) return F3R_ERR_ARG;
  h->base_prec = prec_m;
  return guarded(h, info, [&]() {
    HIPCHK(hipSetDevice(h->device));
    return outer_solve(h, b, x, tol, m, max_iter, true, false, info);
  });
}

f3r_status f3r_get_history(const f3r_handle* h, int32_t level, double* buf, int64_t cap,
                           int64_t* len) {
  if (!h || level < 0 || level >= h->p.nlev || cap < 0 || (cap > 0 && !buf)) return F3R_ERR_ARG;
  if (level > 0) {
    // an inner FGMRES level: the device record of the last solve
    const LevelRT& L = h->lev[(size_t)level];
    if (L.cfg.kind != F3R_FGMRES) return F3R_ERR_ARG;
    int cnt = 0;
    if (L.hist.p) {
      if (hipMemcpyAsync(&cnt, L.I + I_HLEN, sizeof(int), hipMemcpyDeviceToHost, h->st) != hipSuccess ||
          hipStreamSynchronize(h->st) != hipSuccess)
        return F3R_ERR_DEVICE;
    }
    const int64_t k = std::min<int64_t>(cap, cnt);
    if (k > 0 && (hipMemcpyAsync(buf, L.hist.p, (size_t)k * sizeof(double), hipMemcpyDeviceToHost,
                                 h->st) != hipSuccess ||
                  hipStreamSynchronize(h->st) != hipSuccess))
      return F3R_ERR_DEVICE;
    if (len) *len = cnt;
    return F3R_OK;
  }
  const std::vector<double> none;
  const std::vector<double>& hs = h->history.empty() ? none : h->history[0];
  const int64_t k = std::min<int64_t>(cap, (int64_t)hs.size());
  for (int64_t i = 0; i < k; i++) buf[i] = hs[(size_t)i];
  if (len) *len = (int64_t)hs.size();
  return F3R_OK;
}

static bool is_rich(const f3r_handle* h, int32_t level) {
  return level >= 1 && level < h->p.nlev && h->lev[(size_t)level].cfg.kind == F3R_RICHARDSON;
}

f3r_status f3r_get_weights(f3r_handle* h, int32_t level, double* omega, int64_t* c_ntr) {
  if (!h || !is_rich(h, level) || !omega) return F3R_ERR_ARG;
  return guarded(h, nullptr, [&]() {
    HIPCHK(hipStreamSynchronize(h->st));
    HIPCHK(hipMemcpy(omega, h->lev[level].omega, (size_t)h->lev[level].cfg.m * sizeof(double),
                     hipMemcpyDeviceToHost));
    if (c_ntr) *c_ntr = h->rcnt[level];
    return F3R_OK;
  });
}

f3r_status f3r_set_weights(f3r_handle* h, int32_t level, const double* omega, int64_t c_ntr) {
  if (!h || !is_rich(h, level) || !omega || c_ntr < 1) return F3R_ERR_ARG;
  return guarded(h, nullptr, [&]() {
    // weights are quantities of the level arithmetic (fp32 for narrow levels)
    std::vector<double> w(omega, omega + h->lev[level].cfg.m);
    if (h->lev[level].q == T32)
      for (double& v : w) v = (double)(float)v;
    HIPCHK(hipMemcpy(h->lev[level].omega, w.data(), w.size() * sizeof(double),
                     hipMemcpyHostToDevice));
    h->rcnt[level] = c_ntr;
    HIPCHK(hipMemcpy(h->lev[level].cntr_dev, &h->rcnt[level], sizeof(int64_t), hipMemcpyHostToDevice));
    return F3R_OK;
  });
}

f3r_status f3r_debug_spmv(f3r_handle* h, int32_t level, const double* x, double* y) {
  if (!h || !x || !y || level < 0 || level >= h->p.nlev) return F3R_ERR_ARG;
  return guarded(h, nullptr, [&]() {
    LevelRT& L = h->lev[level];
    const int64_t n = h->n;
    if (level == 0) {
      HIPCHK(spmv_dots(h->st, h->A, h->a64, T64, x, T64, nullptr, nullptr, y, T64, nullptr, nullptr, 0,
                       h->partials, nullptr));
    } else {
      const int tx = L.cfg.kind == F3R_FGMRES ? L.zt : L.pv;
      const int ty = L.cfg.kind == F3R_FGMRES ? L.pv : q_of(L.pv);
      HIPCHK(convert(h->st, n, x, T64, h->tmp64, tx));
      HIPCHK(spmv_dots(h->st, h->A, h->ah[L.pa], L.pa, h->tmp64, tx, nullptr, nullptr, h->tmp64b, ty,
                       nullptr, nullptr, 0, h->partials, nullptr));
      HIPCHK(convert(h->st, n, h->tmp64b, ty, y, T64));
    }
    HIPCHK(hipStreamSynchronize(h->st));
    return F3R_OK;
  });
}

// Reads a buffer once with 16-byte loads (one pass, grid-stride) and writes
// nothing unless the XOR of everything read equals a value a zero-filled
// buffer cannot give: evicts the caches without leaving dirty lines behind.
__global__ void k_scrub_read(const uint4* __restrict__ p, int64_t count, uint32_t* sink) {
  uint32_t acc = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + 3 * stride < count; i += 4 * stride) {
    const uint4 a = p[i], b = p[i + stride], c = p[i + 2 * stride], d = p[i + 3 * stride];
    acc ^= a.x ^ a.y ^ a.z ^ a.w ^ b.x ^ b.y ^ b.z ^ b.w ^ c.x ^ c.y ^ c.z ^ c.w ^ d.x ^ d.y ^ d.z ^ d.w;
  }
  for (; i < count; i += stride) {
    const uint4 a = p[i];
    acc ^= a.x ^ a.y ^ a.z ^ a.w;
  }
  if (acc == 0x9e3779b9u) sink[0] = acc;
}

f3r_status f3r_time_spmv(f3r_handle* h, int32_t level, int32_t reps, void* scrub,
                         int64_t scrub_bytes, double* avg_ms) {
  if (!h || !avg_ms || level < 0 || level >= h->p.nlev || reps < 1 || reps > 10000 ||
      scrub_bytes < 0 || (scrub_bytes > 0 && !scrub))
    return F3R_ERR_ARG;
  if (h->lev[level].cfg.kind != F3R_FGMRES) return F3R_ERR_ARG;
  return guarded(h, nullptr, [&]() -> f3r_status {
    HIPCHK(hipSetDevice(h->device));
    LevelRT& L = h->lev[level];
    const int64_t n = h->n;
    // the level's own operands: x = its first Z slot (zeroed), y = V_1
    const int tx = level == 0 ? T64 : L.zt;
    const int ty = level == 0 ? T64 : L.pv;
    const void* av = level == 0 ? (const void*)h->a64 : h->ah[L.pa];
    const int ta = level == 0 ? T64 : L.pa;
    void* x = vec_at(L.Z, tx, 0, n);
    void* y = vec_at(L.V, ty, 1, n);
    HIPCHK(hipMemsetAsync(x, 0, (size_t)n * tsz(tx), h->st));
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    double total = 0.0;
    hipError_t err = hipSuccess;
    for (int r = 0; r < reps && err == hipSuccess; r++) {
      // evict the matrix from the caches before each timed launch (a read,
      // so the eviction writes nothing back during the timed launch)
      if (scrub_bytes >= 16) {
        hipLaunchKernelGGL(k_scrub_read, dim3(4096), dim3(256), 0, h->st, (const uint4*)scrub,
                           scrub_bytes / 16, (uint32_t*)h->partials);
        err = hipGetLastError();
      }
      if (err == hipSuccess) err = hipEventRecord(e0, h->st);
      if (err == hipSuccess)
        err = spmv_dots(h->st, h->A, av, ta, x, tx, nullptr, nullptr, y, ty, nullptr, nullptr, 0,
                        h->partials, nullptr);
      if (err == hipSuccess) err = hipEventRecord(e1, h->st);
      if (err == hipSuccess) err = hipEventSynchronize(e1);
      float ms = 0.f;
      if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
      total += ms;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    HIPCHK(err);
    *avg_ms = total / reps;
    return F3R_OK;
  });
}

// The read-bandwidth reference: workgroup b reads the b-th of gridDim.x
// contiguous ranges of the buffer with 16-byte non-temporal loads, eight in
// flight per thread, and writes nothing unless the XOR of everything it read
// equals a value a zero-filled buffer cannot give.  (Contiguous ranges per
// workgroup and non-temporal loads read faster than a grid-stride loop: 6.5
// against 5.3 TB/s on 1 GiB of an MI355X.)
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
constexpr int kReadBlock = 512;
constexpr int kReadGrid = 2048;
constexpr int kReadUnroll = 8;
__global__ __launch_bounds__(kReadBlock) void k_read_ref(const u32x4* __restrict__ p, int64_t count,
                                                         uint32_t* sink) {
  const int64_t per = (count + gridDim.x - 1) / gridDim.x;
  const int64_t b0 = (int64_t)blockIdx.x * per;
  const int64_t b1 = b0 + per < count ? b0 + per : count;
  uint32_t acc = 0;
  int64_t i = b0 + threadIdx.x;
  for (; i + (kReadUnroll - 1) * kReadBlock < b1; i += kReadUnroll * kReadBlock) {
    u32x4 a[kReadUnroll];
#pragma unroll
    for (int u = 0; u < kReadUnroll; u++) a[u] = __builtin_nontemporal_load(p + i + u * kReadBlock);
#pragma unroll
    for (int u = 0; u < kReadUnroll; u++) acc ^= a[u].x ^ a[u].y ^ a[u].z ^ a[u].w;
  }
  for (; i < b1; i += kReadBlock) {
    const u32x4 a = p[i];
    acc ^= a.x ^ a.y ^ a.z ^ a.w;
  }
  if (acc == 0x9e3779b9u) sink[0] = acc;
}

f3r_status f3r_time_read(f3r_handle* h, const void* buf, int64_t bytes, int32_t reps, double* avg_ms) {
  if (!h || !buf || !avg_ms || bytes < 16 || reps < 1 || reps > 10000 ||
      (reinterpret_cast<uintptr_t>(buf) & 15) != 0)
    return F3R_ERR_ARG;
  return guarded(h, nullptr, [&]() -> f3r_status {
    HIPCHK(hipSetDevice(h->device));
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    double total = 0.0;
    hipError_t err = hipSuccess;
    for (int r = 0; r < reps && err == hipSuccess; r++) {
      err = hipEventRecord(e0, h->st);
      if (err == hipSuccess) {
        hipLaunchKernelGGL(k_read_ref, dim3(kReadGrid), dim3(kReadBlock), 0, h->st,
                           (const u32x4*)buf, bytes / 16, (uint32_t*)h->partials);
        err = hipGetLastError();
      }
      if (err == hipSuccess) err = hipEventRecord(e1, h->st);
      if (err == hipSuccess) err = hipEventSynchronize(e1);
      float ms = 0.f;
      if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
      total += ms;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    HIPCHK(err);
    *avg_ms = total / reps;
    return F3R_OK;
  });
}

f3r_status f3r_debug_apply_m(f3r_handle* h, int32_t prec, const double* r, double* y) {
  if (!h || !r || !y || !prec_ok(prec)) return F3R_ERR_ARG;
  return guarded(h, nullptr, [&]() -> f3r_status {
    int tm, neg;
    const void* mv = m_values(h, tm, neg);
    double gd = h->gd[tm];
    if (prec == T64 && tm != T64) {  // the comparison solver's fp64 factors
      mv = h->m_shared ? h->ah[T64] : h->mv[T64];
      tm = T64;
      gd = h->gd[T64];
    }
    const int64_t n = h->n;
    Basis in;
    in.raw = h->tmp64;
    in.type = prec;
    HIPCHK(convert(h->st, n, r, T64, h->tmp64, prec));
    void* t = h->tmp64b;
    double* outb = (double*)h->partials;  // n values fit: partials hold >= 66 n / 256 doubles
    (void)outb;
    // the sweep shapes of the solve (picked at set-up); chunks of three exist
    // for narrow vectors only
    auto shape = [&](int code) { return code % 10 == 3 && tsz(prec) != 2 ? code + 1 : code; };
    hipError_t e = m_apply_w(h->st, h->A, mv, tm, neg, in, t, prec, nullptr, nullptr, shape(h->kr[0]));
    if (e == hipErrorInvalidValue) return F3R_ERR_ARG;
    HIPCHK(e);
    // y (type prec) into tmp64 (the input is dead now)
    HIPCHK(m_apply_g(h->st, h->A, mv, tm, neg, gd, t, prec, 0, nullptr, nullptr, h->tmp64, prec,
                     nullptr, nullptr, nullptr, nullptr, shape(h->kr[1])));
    HIPCHK(convert(h->st, n, h->tmp64, prec, y, T64));
    HIPCHK(hipStreamSynchronize(h->st));
    return F3R_OK;
  });
}

// ---------------------------------------------------------------------------
// M applied without allocating: the two intermediate vectors of
// f3r_debug_apply_m live in a fixed device array of this file instead of the
// handle's workspace.  Each device holds its own copy of the array; its
// address on a device is looked up once (hipGetSymbolAddress), with that
// device current, when a handle is set up there.
// ---------------------------------------------------------------------------
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
constexpr int kMaxDevices = 64;
static void* g_scratch[kMaxDevices] = {};
static std::once_flag g_scratch_once[kMaxDevices];
static hipError_t g_scratch_err[kMaxDevices] = {};

// address of this device's scratch (the caller has made `device` current)
static hipError_t scratch_address(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::call_once(g_scratch_once[device], [device]() {
    void* p = nullptr;
    g_scratch_err[device] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (g_scratch_err[device] == hipSuccess) g_scratch[device] = p;
  });
  *out = g_scratch[device];
  return g_scratch_err[device];
}

f3r_status f3r_apply_m_static(f3r_handle* h, int32_t prec, const double* r, double* y) {
  if (!h || !r || !y || !prec_ok(prec)) return F3R_ERR_ARG;
  const int64_t n = h->n;
  // the input cast to prec and t = W r, each n values of prec, 256-aligned
  const size_t vec = ((size_t)n * tsz(prec) + 255) & ~(size_t)255;
  if (2 * vec > kStaticScratchBytes) return F3R_ERR_ARG;
  return guarded(h, nullptr, [&]() -> f3r_status {
    HIPCHK(hipSetDevice(h->device));
    void* base = nullptr;
    HIPCHK(scratch_address(h->device, &base));
    if (!base) return F3R_ERR_DEVICE;
    int tm, neg;
    const void* mv = m_values(h, tm, neg);
    double gd = h->gd[tm];
    if (prec == T64 && tm != T64) {  // the comparison solver's fp64 factors
      mv = h->m_shared ? h->ah[T64] : h->mv[T64];
      tm = T64;
      gd = h->gd[T64];
    }
    void* rin = base;
    void* t = (unsigned char*)base + vec;
    Basis in;
    in.raw = rin;
    in.type = prec;
    HIPCHK(convert(h->st, n, r, T64, rin, prec));
    auto shape = [&](int code) { return code % 10 == 3 && tsz(prec) != 2 ? code + 1 : code; };
    hipError_t e = m_apply_w(h->st, h->A, mv, tm, neg, in, t, prec, nullptr, nullptr, shape(h->kr[0]));
    if (e == hipErrorInvalidValue) return F3R_ERR_ARG;
    HIPCHK(e);
    // y (type prec) over the input, which is dead now
    HIPCHK(m_apply_g(h->st, h->A, mv, tm, neg, gd, t, prec, 0, nullptr, nullptr, rin, prec, nullptr,
                     nullptr, nullptr, nullptr, shape(h->kr[1])));
    HIPCHK(convert(h->st, n, rin, prec, y, T64));
    HIPCHK(hipStreamSynchronize(h->st));
    return F3R_OK;
  });
}

f3r_status f3r_debug_apply_level(f3r_handle* h, int32_t level, const double* v, double* z) {
  if (!h || !v || !z || level < 1 || level >= h->p.nlev) return F3R_ERR_ARG;
  return guarded(h, nullptr, [&]() {
    LevelRT& L = h->lev[level];
    const int64_t n = h->n;
    // every inner-level state flag starts clear
    for (size_t d = 1; d < h->lev.size(); d++)
      if (h->lev[d].I) HIPCHK(hipMemsetAsync(h->lev[d].I, 0, level_ints(h->lev[d].cfg.m) * sizeof(int), h->st));
    RScheds rs = make_scheds(h, level, 0);
    scheds_begin(h, h->st, level);
    Ctx c{h, h->st, &rs};
    // the level receives its input in the parent's vector precision
    const int tin = h->p.lev[level - 1].prec_v;
    HIPCHK(convert(h->st, n, v, T64, h->tmp64, tin));
    Basis in;
    in.raw = h->tmp64;
    in.type = tin;
    in.scale = h->one;
    int* zero_flag = h->lev[0].I + I_FB;  // scratch flag, cleared below
    if (L.cfg.kind == F3R_RICHARDSON) {
      enqueue_rich(c, level, in, nullptr, h->tmp64b, zero_flag);
      HIPCHK(convert(h->st, n, h->tmp64b, L.pv, z, T64));
    } else {
      OutSpec o;
      o.ptr = h->tmp64b;
      o.fb = zero_flag;
      enqueue_fgmres(c, level, in, nullptr, nullptr, o, true);
      HIPCHK(convert(h->st, n, h->tmp64b, L.pv, z, T64));
    }
    scheds_end(h, rs, level, nullptr);
    HIPCHK(hipMemsetAsync(zero_flag, 0, sizeof(int), h->st));
    HIPCHK(hipStreamSynchronize(h->st));
    return F3R_OK;
  });
}

f3r_status f3r_debug_round(int32_t prec, const double* in, double* out, int64_t n, void* hip_stream) {
  if (!prec_ok(prec) || !in || !out || n < 0) return F3R_ERR_ARG;
  if (n == 0) return F3R_OK;
  hipStream_t st = (hipStream_t)hip_stream;
  void* tmp = nullptr;
  if (hipMalloc(&tmp, (size_t)n * tsz(prec)) != hipSuccess) return F3R_ERR_NOMEM;
  f3r_status r = F3R_OK;
  if (convert(st, n, in, T64, tmp, prec) != hipSuccess || convert(st, n, tmp, prec, out, T64) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    r = F3R_ERR_DEVICE;
  (void)hipFree(tmp);
  return r;
}

f3r_status f3r_debug_scaling(f3r_handle* h, double* s_host) {
  if (!h || !s_host) return F3R_ERR_ARG;
  return guarded(h, nullptr, [&]() {
    HIPCHK(hipMemcpy(s_host, h->s, (size_t)h->n * 8, hipMemcpyDeviceToHost));
    return F3R_OK;
  });
}

f3r_status f3r_debug_m_values(f3r_handle* h, int32_t prec, double* vals_host) {
  if (!h || !vals_host || !prec_ok(prec) || h->m_shared || !h->mv[prec]) return F3R_ERR_ARG;
  return guarded(h, nullptr, [&]() {
    double* d = (double*)h->dalloc((size_t)h->nnz * 8);
    HIPCHK(sell_to_csr_values(h->st, h->n, h->rp, h->off, h->kd_true, h->A.dell_kd, h->ci, soff_of(h), h->mv[prec], prec,
                              d));
    HIPCHK(hipMemcpyAsync(vals_host, d, (size_t)h->nnz * 8, hipMemcpyDeviceToHost, h->st));
    HIPCHK(hipStreamSynchronize(h->st));
    h->al.release(d);
    return F3R_OK;
  });
}

f3r_status f3r_debug_level_values(f3r_handle* h, int32_t prec, double* vals_host) {
  if (!h || !vals_host || !prec_ok(prec) || !h->ah[prec]) return F3R_ERR_ARG;
  return guarded(h, nullptr, [&]() {
    double* d = (double*)h->dalloc((size_t)h->nnz * 8);
    HIPCHK(sell_to_csr_values(h->st, h->n, h->rp, h->off, h->kd_true, h->A.dell_kd, h->ci, soff_of(h), h->ah[prec], prec,
                              d));
    HIPCHK(hipMemcpyAsync(vals_host, d, (size_t)h->nnz * 8, hipMemcpyDeviceToHost, h->st));
    HIPCHK(hipStreamSynchronize(h->st));
    h->al.release(d);
    return F3R_OK;
  });
}

}  // extern "C"

// ===========================================================================
// stacked systems (the lockstep mode of the batched entry points)
// ===========================================================================
namespace f3r {

f3r_status stacked_setup(int32_t count, const f3r_csr* A, const f3r_params* p, void* hip_stream,
                         f3r_handle** out) {
  if (!out || count < 1 || !A) return F3R_ERR_ARG;
  *out = nullptr;
  std::vector<int64_t> row0((size_t)count + 1), nrows((size_t)count);
  int64_t rows = 0, nnz = 0;
  for (int s = 0; s < count; s++) {
    const f3r_csr& a = A[s];
    if (!a.row_ptr || !a.col_idx || !a.val || a.n <= 0 || a.nnz < a.n) return F3R_ERR_ARG;
    if (a.row_ptr[0] != 0 || a.row_ptr[a.n] != a.nnz) return F3R_ERR_MATRIX;
    row0[(size_t)s] = rows;
    nrows[(size_t)s] = a.n;
    const int64_t padded = (a.n + kSysAlign - 1) / kSysAlign * kSysAlign;
    rows += padded;
    nnz += a.nnz + (padded - a.n);
  }
  row0[(size_t)count] = rows;
  if (rows >= ((int64_t)1 << 31) - 64 || nnz >= ((int64_t)1 << 31)) return F3R_ERR_ARG;
  // one CSR matrix with the systems on its diagonal; each system is padded
  // with identity rows to a multiple of 1024 rows (b = 0 there, so those
  // rows stay zero in every vector and add nothing to any sum)
  std::vector<int32_t> rp((size_t)rows + 1), ci((size_t)nnz);
  std::vector<double> va((size_t)nnz);
  int64_t k = 0;
  for (int s = 0; s < count; s++) {
    const f3r_csr& a = A[s];
    const int64_t r0 = row0[(size_t)s];
    for (int64_t i = 0; i < a.n; i++) {
      rp[(size_t)(r0 + i)] = (int32_t)k;
      if (a.row_ptr[i + 1] < a.row_ptr[i]) return F3R_ERR_MATRIX;
      for (int64_t e = a.row_ptr[i]; e < a.row_ptr[i + 1]; e++) {
        const int64_t c = a.col_idx[e];
        if (c < 0 || c >= a.n) return F3R_ERR_MATRIX;
        ci[(size_t)k] = (int32_t)(r0 + c);
        va[(size_t)k] = a.val[e];
        k++;
      }
    }
    for (int64_t i = a.n; i < row0[(size_t)s + 1] - r0; i++) {
      rp[(size_t)(r0 + i)] = (int32_t)k;
      ci[(size_t)k] = (int32_t)(r0 + i);
      va[(size_t)k] = 1.0;
      k++;
    }
  }
  rp[(size_t)rows] = (int32_t)k;
  const f3r_csr cat{rows, nnz, rp.data(), ci.data(), va.data()};
  return setup_impl(&cat, p, hip_stream, count, row0, nrows, true, out);
}

f3r_status stacked_solve(f3r_handle* h, const double* const* b, double* const* x, double tol,
                         f3r_info* infos) {
  if (!h || !b || !x || !(tol > 0.0) || !h->ptrs_dev) return F3R_ERR_ARG;
  for (int s = 0; s < h->nsys; s++)
    if (!b[s] || !x[s]) return F3R_ERR_ARG;
  f3r_status st = guarded(h, nullptr, [&]() -> f3r_status {
    HIPCHK(hipSetDevice(h->device));
    const StackIo io{h->A.sys, h->row0_dev, h->nrows_dev, h->ptrs_dev, h->n};
    HIPCHK(hipMemcpyAsync(h->ptrs_dev, b, (size_t)h->nsys * sizeof(double*), hipMemcpyHostToDevice,
                          h->st));
    HIPCHK(stack_gather(h->st, io, h->bcat));
    HIPCHK(hipMemcpyAsync(h->ptrs_dev, x, (size_t)h->nsys * sizeof(double*), hipMemcpyHostToDevice,
                          h->st));
    if (h->p.flags & F3R_USE_X0) HIPCHK(stack_gather(h->st, io, h->xcat));
    const f3r_status r = outer_solve(h, h->bcat, h->xcat, tol, h->p.lev[0].m, h->p.max_outer,
                                     h->p.nlev < 2, use_graphs(h->p), infos);
    HIPCHK(stack_scatter(h->st, io, h->xcat));
    HIPCHK(hipStreamSynchronize(h->st));
    return r;
  });
  return st;
}

f3r_status stacked_history(const f3r_handle* h, int32_t sys, double* buf, int64_t cap, int64_t* len) {
  if (!h || sys < 0 || sys >= h->nsys || cap < 0 || (cap > 0 && !buf)) return F3R_ERR_ARG;
  const std::vector<double> none;
  const std::vector<double>& hs = (size_t)sys < h->history.size() ? h->history[(size_t)sys] : none;
  const int64_t k = std::min<int64_t>(cap, (int64_t)hs.size());
  for (int64_t i = 0; i < k; i++) buf[i] = hs[(size_t)i];
  if (len) *len = (int64_t)hs.size();
  return F3R_OK;
}

}  // namespace f3r

// ===========================================================================
// comparison solvers of Sec. 5: preconditioned CG and BiCGStab in fp64
// ===========================================================================
namespace {

enum { KS_RZ0 = 0, KS_RZ1 = 1, KS_PQ = 2, KS_RHO0 = 3, KS_RHO1 = 4, KS_ALPHA = 5, KS_OMEGA = 6,
       KS_RV = 7, KS_TS = 8, KS_TT = 9, KS_NORM = 10, KS_ONE = 11, KS_COUNT = 16 };

f3r_status krylov_impl(f3r_handle* h, int method, int prec, const double* b, double* x, double tol,
                       int max_iter, f3r_info* info) {
  const int64_t n = h->n;
  const int64_t nb = n_blocks(n);
  const SysLayout one_sys{};
  // M's values in the requested storage
  const void* mv = nullptr;
  int neg = 0;
  if (h->m_shared) {
    mv = h->ah[prec];
    neg = 1;
  } else {
    mv = h->mv[prec];
  }
  if (!mv) return F3R_ERR_ARG;
  const double gd = h->gd[prec];
  if (!h->kv) {
    h->kv = (double*)h->dalloc((size_t)10 * (size_t)n * sizeof(double));
    h->ks = (double*)h->dalloc(KS_COUNT * sizeof(double));
  }
  double* V[10];
  for (int k = 0; k < 10; k++) V[k] = h->kv + (size_t)k * (size_t)n;
  double *r = V[0], *z = V[1], *p = V[2], *q = V[3], *tmp = V[4], *rh = V[5], *v = V[6], *t = V[7],
         *ps = V[8], *sv = V[9];
  double* ks = h->ks;
  const double t0 = now_ms();
  int64_t m_calls = 0;
  auto prec_apply = [&](const double* in_v, double* out_v) {  // out = S M (S in)
    Basis in;
    in.raw = in_v;
    in.type = T64;
    in.scale = h->one;
    in.s = h->s;
    HIPCHK(m_apply_w(h->st, h->A, mv, prec, neg, in, tmp, T64, nullptr, nullptr));
    HIPCHK(m_apply_g(h->st, h->A, mv, prec, neg, gd, tmp, T64, 3, nullptr, nullptr, out_v, T64, h->s,
                     nullptr, nullptr, nullptr));
    m_calls++;
  };
  auto sum_to = [&](int slot) {  // partials -> device slot
    HIPCHK(finalize_sums(h->st, one_sys, T64, h->partials, nb, 1, nullptr, ks + slot, nullptr));
  };
  auto dot_to = [&](const double* a, const double* c, int slot) {
    HIPCHK(dot64_partials(h->st, n, a, c, h->partials));
    sum_to(slot);
  };
  auto host_norm = [&]() {  // sqrt of slot KS_NORM on the host
    HIPCHK(hipMemcpyAsync(h->hpin, ks + KS_NORM, sizeof(double), hipMemcpyDeviceToHost, h->st));
    HIPCHK(hipStreamSynchronize(h->st));
    return std::sqrt(h->hpin[0]);
  };
  auto true_residual = [&]() {  // r = b - A x, its norm on the host
    HIPCHK(residual64(h->st, h->A, h->a64, x, b, r, h->partials));
    sum_to(KS_NORM);
    return host_norm();
  };
  h->history.assign(1, std::vector<double>());
  std::vector<double>& hist = h->history[0];
  if (!(h->p.flags & F3R_USE_X0)) HIPCHK(hipMemsetAsync(x, 0, (size_t)n * sizeof(double), h->st));
  dot_to(b, b, KS_NORM);
  const double bn = host_norm();
  f3r_status status = F3R_NOT_CONVERGED;
  int it = 0;
  double rel = 0.0, est = 0.0;
  if (bn == 0.0) {
    HIPCHK(hipMemsetAsync(x, 0, (size_t)n * sizeof(double), h->st));
    status = F3R_OK;
  } else if (!std::isfinite(bn)) {
    status = F3R_ERR_ARG;
  } else if (method == F3R_CG) {
    rel = true_residual() / bn;
    prec_apply(r, z);
    HIPCHK(hipMemcpyAsync(p, z, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, h->st));
    int cur = KS_RZ0, nxt = KS_RZ1;
    dot_to(r, z, cur);
    while (rel >= tol && it < max_iter) {
      // q = A p and (p, q)
      HIPCHK(spmv_dots(h->st, h->A, h->a64, T64, p, T64, nullptr, nullptr, q, T64, p, nullptr, 1,
                       h->partials, nullptr));
      sum_to(KS_PQ);
      HIPCHK(cg_update_xr(h->st, n, x, r, p, q, ks + cur, ks + KS_PQ, h->partials));
      sum_to(KS_NORM);
      it++;
      est = rel = host_norm() / bn;
      hist.push_back(rel);
      if (!std::isfinite(rel)) break;
      if (rel < tol) {
        rel = true_residual() / bn;  // confirmed, or continue from the true residual
        if (rel < tol) break;
      }
      prec_apply(r, z);
      dot_to(r, z, nxt);
      HIPCHK(cg_update_p(h->st, n, p, z, ks + nxt, ks + cur));
      std::swap(cur, nxt);
    }
  } else {
    rel = true_residual() / bn;
    HIPCHK(hipMemcpyAsync(rh, r, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, h->st));
    HIPCHK(hipMemsetAsync(p, 0, (size_t)n * sizeof(double), h->st));
    HIPCHK(hipMemsetAsync(v, 0, (size_t)n * sizeof(double), h->st));
    const double ones[3] = {1.0, 1.0, 1.0};  // rho, alpha, omega start at 1
    HIPCHK(hipMemcpy(ks + KS_RHO0, ones, sizeof(double), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(ks + KS_ALPHA, ones + 1, 2 * sizeof(double), hipMemcpyHostToDevice));
    int cur = KS_RHO0, nxt = KS_RHO1;
    while (rel >= tol && it < max_iter) {
      dot_to(rh, r, nxt);
      HIPCHK(bicg_update_p(h->st, n, p, r, v, ks + nxt, ks + cur, ks + KS_ALPHA, ks + KS_OMEGA));
      std::swap(cur, nxt);  // rho = rho_new
      prec_apply(p, z);
      // v = A z and (rh, v)
      HIPCHK(spmv_dots(h->st, h->A, h->a64, T64, z, T64, nullptr, nullptr, v, T64, rh, nullptr, 1,
                       h->partials, nullptr));
      sum_to(KS_RV);
      HIPCHK(bicg_update_s(h->st, n, sv, r, v, ks + cur, ks + KS_RV, ks + KS_ALPHA, h->partials));
      sum_to(KS_NORM);
      it++;
      const double srel = host_norm() / bn;
      if (srel < tol) {  // the half step meets the tolerance
        HIPCHK(axpy_dev(h->st, n, x, z, ks + KS_ALPHA));
        est = rel = true_residual() / bn;
        hist.push_back(rel);
        if (rel < tol || !std::isfinite(rel)) break;
        continue;
      }
      prec_apply(sv, ps);
      // t = A ps and (t, s); then (t, t)
      HIPCHK(spmv_dots(h->st, h->A, h->a64, T64, ps, T64, nullptr, nullptr, t, T64, sv, nullptr, 1,
                       h->partials, nullptr));
      sum_to(KS_TS);
      dot_to(t, t, KS_TT);
      HIPCHK(bicg_update_xr(h->st, n, x, r, sv, t, z, ps, ks + KS_ALPHA, ks + KS_TS, ks + KS_TT,
                            ks + KS_OMEGA, h->partials));
      sum_to(KS_NORM);
      est = rel = host_norm() / bn;
      hist.push_back(rel);
      if (!std::isfinite(rel)) break;
      if (rel < tol) {
        rel = true_residual() / bn;
        if (rel < tol) break;
      }
    }
  }
  if (bn != 0.0 && std::isfinite(bn)) {
    rel = true_residual() / bn;
    if (!std::isfinite(rel))
      status = F3R_ERR_BREAKDOWN;
    else if (rel < tol)
      status = F3R_OK;
  }
  const double t1 = now_ms();
  if (info) {
    std::memset(info, 0, sizeof(*info));
    info->status = status;
    info->outer_iters = it;
    info->m_calls = m_calls;
    info->spmv[0] = method == F3R_CG ? it : 2 * (int64_t)it;
    info->relres_est = est;
    info->relres_true = rel;
    info->setup_ms = h->setup_ms;
    info->solve_ms = t1 - t0;
    info->idx_bits = idx_bits_of(h->A);
    info->sell_c = 64;
    info->padded_nnz = h->padded;
    info->layout = layout_of(h->A);
  }
  return status;
}

}  // namespace

extern "C" f3r_status f3r_krylov_solve(f3r_handle* h, int32_t method, int32_t prec_m,
                                       const double* b, double* x, double tol, int32_t max_iter,
                                       f3r_info* info) {
  if (!h || !b || !x || !(tol > 0.0) || max_iter < 1 || !prec_ok(prec_m)) return F3R_ERR_ARG;
  if (method != F3R_CG && method != F3R_BICGSTAB) return F3R_ERR_ARG;
  if (h->nsys != 1) return F3R_ERR_ARG;
  return guarded(h, info, [&]() {
    HIPCHK(hipSetDevice(h->device));
    return krylov_impl(h, method, prec_m, b, x, tol, max_iter, info);
  });
}
