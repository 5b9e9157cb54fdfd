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
#include <string>
#include <vector>

#include "f3r.h"
#include "host.h"
#include "kernels.h"
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
  // Richardson
  void* rt = nullptr;
  void* ry = nullptr;
  void* rr = nullptr;
  void* rz[2] = {nullptr, nullptr};
  double* omega = nullptr;
  double* wcur = nullptr;
  int64_t* cntr_dev = nullptr;
};

// Richardson schedule of one enqueue: update flag and poison flag per call
struct RSched {
  std::vector<char> upd, poison;
  size_t pos = 0;
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
  int rich = -1;  // index of the Richardson level, -1 when none
  int64_t cntr = 1;  // host copy of c_ntr of the Richardson level
  void* partials = nullptr;
  double* one = nullptr;   // device constant 1.0
  double* tmp64 = nullptr;  // n doubles
  double* tmp64b = nullptr;
  double* hpin = nullptr;  // pinned host words
  std::map<std::string, hipGraphExec_t> graphs;
  std::vector<hipGraph_t> graph_objs;
  std::vector<double> history;
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

f3r_status check_params(const f3r_params* p) {
  if (!p || p->nlev < 1 || p->nlev > F3R_MAX_LEVELS) return F3R_ERR_ARG;
  if (p->lev[0].kind != F3R_FGMRES || p->lev[0].prec_a != F3R_FP64 || p->lev[0].prec_v != F3R_FP64)
    return F3R_ERR_ARG;
  if (p->lev[0].m < 1 || p->lev[0].m > 1000) return F3R_ERR_ARG;
  for (int d = 1; d < p->nlev; d++) {
    const f3r_level& l = p->lev[d];
    if (l.m < 1 || l.m > 64 || !prec_ok(l.prec_a) || !prec_ok(l.prec_v)) return F3R_ERR_ARG;
    if (l.kind == F3R_RICHARDSON && d != p->nlev - 1) return F3R_ERR_ARG;
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
  if (p->rows_per_lane != 0 && p->rows_per_lane != 1 && p->rows_per_lane != 2 && p->rows_per_lane != 4)
    return F3R_ERR_ARG;
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
      L.S = (double*)h->dalloc((size_t)L.L.total * sizeof(double));
      L.I = (int*)h->dalloc((size_t)level_ints(m) * sizeof(int));
      HIPCHK(hipMemsetAsync(L.S, 0, (size_t)L.L.total * sizeof(double), h->st));
      HIPCHK(hipMemsetAsync(L.I, 0, (size_t)level_ints(m) * sizeof(int), h->st));
    } else {
      h->rich = d;
      L.rt = h->dalloc((size_t)n * tsz(L.pv));
      L.ry = h->dalloc((size_t)n * tsz(L.pv));
      L.rr = h->dalloc((size_t)n * tsz(L.pv));
      L.rz[0] = h->dalloc((size_t)n * tsz(L.pv));
      L.rz[1] = h->dalloc((size_t)n * tsz(L.pv));
      L.omega = (double*)h->dalloc(64 * sizeof(double));
      L.wcur = (double*)h->dalloc(sizeof(double));
      L.cntr_dev = (int64_t*)h->dalloc(sizeof(int64_t));
      HIPCHK(set_omega(h->st, L.omega, m, L.q == T32 ? (double)(float)p.omega_init : p.omega_init));
    }
  }
}

// ---------------------------------------------------------------------------
// level engine
// ---------------------------------------------------------------------------
struct Ctx {
  f3r_handle* h;
  hipStream_t st;
  RSched* rs;
};

// HIP events around the launches of the probed kernel (direct launches on
// the solve's stream only)
void probe_begin(Ctx& c, int id) {
  f3r_handle* h = c.h;
  if (h->probe != id || c.st != h->st) return;
  if (h->ev_used + 2 > h->ev.size()) {
    HIPCHK(hipStreamSynchronize(h->st));
    for (size_t i = 0; i + 1 < h->ev_used; i += 2) {
      float ms = 0;
      HIPCHK(hipEventElapsedTime(&ms, h->ev[i], h->ev[i + 1]));
      h->probe_ms += ms;
      h->probe_n++;
    }
    h->ev_used = 0;
    while (h->ev.size() < 512) {
      hipEvent_t e;
      HIPCHK(hipEventCreate(&e));
      h->ev.push_back(e);
    }
  }
  HIPCHK(hipEventRecord(h->ev[h->ev_used], h->st));
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
  for (size_t i = 0; i + 1 < h->ev_used; i += 2) {
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, h->ev[i], h->ev[i + 1]));
    h->probe_ms += ms;
    h->probe_n++;
  }
  h->ev_used = 0;
}

struct OutSpec {
  void* ptr = nullptr;   // output vector (or base when cur is set)
  const double* s = nullptr;
  const int* cur = nullptr;
  int* fb = nullptr;     // non-finite flag of the parent's column (base when cur is set)
};

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
  const bool upd = c.rs->upd[c.rs->pos] != 0;
  const bool poison = c.rs->poison[c.rs->pos] != 0;
  c.rs->pos++;
  int tm, neg;
  const void* mv = m_values(h, tm, neg);
  const double gd = h->gd[tm];
  const void* av = h->ah[R.pa];
  const void* zprev = nullptr;
  const int64_t nb = n_blocks(h->n);
  for (int k = 0; k < m; k++) {
    const bool last = k == m - 1;
    void* zk = last ? out : R.rz[k & 1];
    int* zfb = last ? fb : nullptr;
    Basis rsrc;
    if (k == 0) {
      rsrc = vin;
    } else {
      probe_begin(c, F3R_PROBE_R_RESIDUAL);
      HIPCHK(rich_residual(c.st, h->A, av, R.pa, vin, zprev, R.rr, tr, stop, h->kr[2]));
      probe_end(c, F3R_PROBE_R_RESIDUAL);
      rsrc.raw = R.rr;
      rsrc.type = tr;
    }
    probe_begin(c, F3R_PROBE_M_LOWER);
    HIPCHK(m_apply_w(c.st, h->A, mv, tm, neg, rsrc, R.rt, tr, stop, k == 0 ? R.cntr_dev : nullptr,
                     h->kr[0]));
    probe_end(c, F3R_PROBE_M_LOWER);
    if (!upd) {
      probe_begin(c, F3R_PROBE_M_UPPER);
      HIPCHK(m_apply_g(c.st, h->A, mv, tm, neg, gd, R.rt, tr, k == 0 ? 1 : 2, R.omega + k, zprev, zk,
                       tr, nullptr, zfb, stop, nullptr, h->kr[1]));
      probe_end(c, F3R_PROBE_M_UPPER);
    } else {
      HIPCHK(m_apply_g(c.st, h->A, mv, tm, neg, gd, R.rt, tr, 0, nullptr, nullptr, R.ry, tr, nullptr,
                       nullptr, stop, nullptr, h->kr[1]));
      HIPCHK(rich_tdots(c.st, h->A, av, R.pa, R.ry, tr, rsrc, h->partials, stop));
      HIPCHK(rich_omega(c.st, q_of(tr), h->partials, nb, R.omega + k, R.wcur, R.cntr_dev, h->p.c,
                        stop));
      HIPCHK(rich_zupdate(c.st, h->n, k == 0 ? nullptr : zprev, R.ry, tr, R.wcur, zk, zfb, stop));
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
  }
  const void* v0 = aliased ? alias_raw : L.V;
  if (!aliased) {
    ChildInit self{L.S, L.I, m, L.L.g, L.L.scale};
    HIPCHK(entry_cast(c.st, n, vin, L.V, L.pv, h->partials, pstop));
    HIPCHK(entry_finalize(c.st, L.q, h->partials, nb, self, child_alias ? &ci_child : nullptr, pstop));
  } else if (child_alias) {
    HIPCHK(child_init0(c.st, L.S, L.I, L.L, ci_child));
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
    probe_begin(c, pid);
    HIPCHK(spmv_dots(c.st, h->A, h->ah[L.pa], L.pa, zj, L.zt, &bj, fbj, vec_at(L.V, L.pv, j + 1, n),
                     L.pv, v0, vb, j + 1, h->partials, stop));
    probe_end(c, pid);
    HIPCHK(finalize_sums(c.st, L.q, h->partials, nb, j + 1, L.S + L.L.scale, hcol, stop));
    HIPCHK(axpy_norm(c.st, n, vec_at(L.V, L.pv, j + 1, n), L.pv, v0, vb, j + 1, hcol, L.S + L.L.scale,
                     h->partials, stop));
    HIPCHK(givens(c.st, L.q, h->partials, nb, L.S, L.I, L.L, j, j == m - 1, 1.0, nullptr,
                  child_alias ? &ci_child : nullptr));
  }
  LevelBasis lb;
  lb.v0 = v0;
  lb.vb = vb;
  lb.type = L.pv;
  lb.scales = L.S + L.L.scale;
  HIPCHK(combine(c.st, n, L.Z, L.zt, L.pv, L.S + L.L.y, L.I + I_MEFF, out.ptr, out.s, out.cur, 0, &lb,
                 L.I + I_FB, out.fb));
}

// Set-up autotuner: times the candidate shapes (rows per lane and entry
// chunk) of the three sweeps of the Richardson level on this matrix and
// keeps the fastest of each.  The sweeps have no reductions, so the shape
// changes only the time, never a result.
void autotune(f3r_handle* h) {
  const int fixed = h->p.rows_per_lane;
  if (fixed) {
    const int code = fixed == 1 ? 18 : fixed == 2 ? 24 : 44;
    h->kr[0] = h->kr[1] = h->kr[2] = code;
    return;
  }
  if (h->rich < 0) return;
  const double t0 = now_ms();
  LevelRT& R = h->lev[h->rich];
  const int tr = R.pv;
  int tm, neg;
  const void* mv = m_values(h, tm, neg);
  const double gd = h->gd[tm];
  const int64_t n = h->n;
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
  const int ncand = tsz(tr) == 2 ? 5 : 3;
  for (int f = 0; f < 3; f++) {
    float best = 0.f;
    for (int c = 0; c < ncand; c++) {
      const int kr = cand[c];
      auto launch = [&]() {
        if (f == 0)
          HIPCHK(m_apply_w(h->st, h->A, mv, tm, neg, vec, R.rt, tr, nullptr, nullptr, kr));
        else if (f == 1)
          HIPCHK(m_apply_g(h->st, h->A, mv, tm, neg, gd, R.rr, tr, 2, h->one, R.rz[0], R.rt, tr,
                           nullptr, nullptr, nullptr, nullptr, kr));
        else
          HIPCHK(rich_residual(h->st, h->A, h->ah[R.pa], R.pa, basis, R.rz[0], R.rt, tr, nullptr, kr));
      };
      launch();
      HIPCHK(hipEventRecord(e0, h->st));
      for (int i = 0; i < 5; i++) launch();
      HIPCHK(hipEventRecord(e1, h->st));
      HIPCHK(hipEventSynchronize(e1));
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, e0, e1));
      if (c == 0 || ms < best) {
        best = ms;
        h->kr[f] = kr;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  h->tune_ms = now_ms() - t0;
}

// initial weight in the Richardson level's arithmetic
double omega_init_q(const f3r_handle* h) {
  const double w = h->p.omega_init;
  return h->lev[h->rich].q == T32 ? (double)(float)w : w;
}

// Richardson calls made by one invocation of level 1
int64_t r_calls_per_f2(const f3r_params& p) {
  if (p.nlev < 2 || p.lev[p.nlev - 1].kind != F3R_RICHARDSON) return 0;
  int64_t c = 1;
  for (int d = 1; d < p.nlev - 1; d++) c *= p.lev[d].m;
  return c;
}

RSched make_sched(f3r_handle* h, int64_t ncalls, int64_t executed_before) {
  RSched rs;
  rs.upd.resize((size_t)std::max<int64_t>(ncalls, 1), 0);
  rs.poison.resize((size_t)std::max<int64_t>(ncalls, 1), 0);
  for (int64_t i = 0; i < ncalls; i++) {
    const int64_t cn = h->cntr + i;
    rs.upd[(size_t)i] = h->p.c > 0 && cn % h->p.c == 0;
    rs.poison[(size_t)i] = h->p.poison_call > 0 && executed_before + i + 1 == h->p.poison_call;
  }
  return rs;
}

std::string sched_key(const RSched& rs) {
  std::string k(rs.upd.size() * 2, '0');
  for (size_t i = 0; i < rs.upd.size(); i++) {
    k[2 * i] = rs.upd[i] ? '1' : '0';
    k[2 * i + 1] = rs.poison[i] ? '1' : '0';
  }
  return k;
}

// ---------------------------------------------------------------------------
// the outermost level
// ---------------------------------------------------------------------------
struct SolveStats {
  int outer = 0, restarts = 0;
  int64_t r_calls = 0, m_calls = 0, upd_calls = 0;
  double est = 0, relres = 0;
};

void f2_call(f3r_handle* h, SolveStats& ss, bool use_graph) {
  LevelRT& L0 = h->lev[0];
  const int64_t ncalls = r_calls_per_f2(h->p);
  RSched rs = make_sched(h, ncalls, ss.r_calls);
  if (h->rich >= 0 && h->cntr == 1)  // Alg. 1: the first call sets every weight to omega_init
    HIPCHK(set_omega(h->st, h->lev[h->rich].omega, h->lev[h->rich].cfg.m, omega_init_q(h)));
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
      rs.pos = 0;
    } else {
      ex = it->second;
    }
    HIPCHK(hipGraphLaunch(ex, h->st));
    h->graph_launches++;
  } else {
    Ctx c{h, h->st, &rs};
    enqueue_fgmres(c, 1, in, nullptr, L0.I + I_STOP, out, false);
  }
  for (int64_t i = 0; i < ncalls; i++) ss.upd_calls += rs.upd[(size_t)i];
  h->cntr += ncalls;
  ss.r_calls += ncalls;
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
  const void* mv = h->m_shared ? h->ah[T64] : h->mv[T64];
  const int neg = h->m_shared ? 1 : 0;
  HIPCHK(m_apply_w(h->st, h->A, mv, T64, neg, in, h->tmp64, T64, L0.I + I_STOP, nullptr));
  HIPCHK(m_apply_g(h->st, h->A, mv, T64, neg, h->gd[T64], h->tmp64, T64, 3, nullptr, nullptr, L0.Z,
                   T64, h->s, L0.I + I_FB, L0.I + I_STOP, L0.I + I_CUR));
}

f3r_status outer_solve(f3r_handle* h, const double* b, double* x, double tol, int m1, int max_outer,
                       bool baseline, bool use_graph, f3r_info* info) {
  const int64_t n = h->n;
  const int64_t nb = n_blocks(n);
  LevelRT& L0 = h->lev[0];
  if (m1 > L0.cfg.m) return F3R_ERR_ARG;
  const double t0 = now_ms();
  SolveStats ss;
  h->history.clear();
  h->graph_launches = 0;
  h->probe = h->p.probe_kernel;
  h->probe_ms = 0;
  h->probe_n = 0;
  h->ev_used = 0;
  if (h->probe) use_graph = false;
  if (!(h->p.flags & F3R_USE_X0)) HIPCHK(hipMemsetAsync(x, 0, (size_t)n * sizeof(double), h->st));
  if (h->rich >= 0 && !(h->p.flags & F3R_PERSIST_WEIGHTS)) {
    h->cntr = 1;
    HIPCHK(hipMemcpyAsync(h->lev[h->rich].cntr_dev, &h->cntr, sizeof(int64_t), hipMemcpyHostToDevice,
                          h->st));
  }
  HIPCHK(hipMemsetAsync(L0.I, 0, (size_t)level_ints(L0.cfg.m) * sizeof(int), h->st));
  for (size_t d = 1; d < h->lev.size(); d++)
    if (h->lev[d].I)
      HIPCHK(hipMemsetAsync(h->lev[d].I + I_FALLBACKS, 0, 2 * sizeof(int), h->st));
  HIPCHK(dot64_to_host(h->st, n, b, b, h->partials, h->hpin + 4));
  HIPCHK(hipStreamSynchronize(h->st));
  const double bnorm = std::sqrt(h->hpin[4]);
  f3r_status status = F3R_NOT_CONVERGED;
  if (bnorm == 0.0) {
    HIPCHK(hipMemsetAsync(x, 0, (size_t)n * sizeof(double), h->st));
    HIPCHK(hipStreamSynchronize(h->st));
    ss.relres = 0.0;
    status = F3R_OK;
  } else if (!std::isfinite(bnorm)) {
    status = F3R_ERR_ARG;
  } else {
    const double inv_bnorm = 1.0 / bnorm;
    HIPCHK(residual64(h->st, h->A, h->a64, x, b, (double*)L0.V, h->partials));
    HIPCHK(residual_finalize(h->st, h->partials, nb, L0.S, L0.I, L0.L, inv_bnorm, h->hpin));
    HIPCHK(hipStreamSynchronize(h->st));
    ss.relres = h->hpin[0];
    if (ss.relres < tol) status = F3R_OK;
    while (status == F3R_NOT_CONVERGED && ss.outer < max_outer) {
      const int len = std::min(m1, max_outer - ss.outer);
      int it = 0;
      bool bad = false;
      for (int j = 0; j < len; j++) {
        if (baseline) {
          baseline_prec(h);
          ss.m_calls += 1;
        } else {
          f2_call(h, ss, use_graph);
        }
        void* zj = vec_at(L0.Z, T64, j, n);
        Basis bj;
        bj.raw = vec_at(L0.V, T64, j, n);
        bj.type = T64;
        bj.scale = L0.S + L0.L.scale + j;
        Ctx c0{h, h->st, nullptr};
        probe_begin(c0, F3R_PROBE_SPMV_L0);
        HIPCHK(spmv_dots(h->st, h->A, h->a64, T64, zj, T64, &bj, L0.I + I_FB + j,
                         vec_at(L0.V, T64, j + 1, n), T64, L0.V, vec_at(L0.V, T64, 1, n), j + 1,
                         h->partials, L0.I + I_STOP));
        probe_end(c0, F3R_PROBE_SPMV_L0);
        double* hcol = L0.S + L0.L.H + (int64_t)j * (L0.cfg.m + 1);
        HIPCHK(finalize_sums(h->st, T64, h->partials, nb, j + 1, L0.S + L0.L.scale, hcol,
                             L0.I + I_STOP));
        HIPCHK(axpy_norm(h->st, n, vec_at(L0.V, T64, j + 1, n), T64, L0.V, vec_at(L0.V, T64, 1, n),
                         j + 1, hcol, L0.S + L0.L.scale, h->partials, L0.I + I_STOP));
        HIPCHK(givens(h->st, T64, h->partials, nb, L0.S, L0.I, L0.L, j, 0, inv_bnorm, h->hpin,
                      nullptr));
        HIPCHK(hipStreamSynchronize(h->st));
        probe_collect(h);
        it++;
        ss.outer++;
        ss.est = h->hpin[0];
        h->history.push_back(ss.est);
        const int flags = (int)h->hpin[1];
        if (flags & 2) {
          bad = true;
          break;
        }
        if (ss.est < tol || (flags & 1)) break;
      }
      if (bad) {
        status = F3R_ERR_BREAKDOWN;
        break;
      }
      HIPCHK(backsolve(h->st, T64, L0.S, L0.I, L0.L));
      LevelBasis lb;
      lb.v0 = L0.V;
      lb.vb = vec_at(L0.V, T64, 1, n);
      lb.type = T64;
      lb.scales = L0.S + L0.L.scale;
      HIPCHK(combine(h->st, n, L0.Z, T64, T64, L0.S + L0.L.y, L0.I + I_MEFF, x, nullptr, nullptr, 1,
                     &lb, L0.I + I_FB, nullptr));
      HIPCHK(residual64(h->st, h->A, h->a64, x, b, (double*)L0.V, h->partials));
      HIPCHK(residual_finalize(h->st, h->partials, nb, L0.S, L0.I, L0.L, inv_bnorm, h->hpin));
      HIPCHK(hipStreamSynchronize(h->st));
      ss.relres = h->hpin[0];
      if (!std::isfinite(ss.relres)) {
        status = F3R_ERR_BREAKDOWN;
        break;
      }
      if (ss.relres < tol) {
        status = F3R_OK;
        break;
      }
      ss.restarts++;
      if (it == 0) break;
    }
  }
  const double t1 = now_ms();
  if (info) {
    std::memset(info, 0, sizeof(*info));
    info->status = status;
    info->outer_iters = ss.outer;
    info->restarts = ss.restarts;
    const f3r_params& p = h->p;
    if (baseline) {
      info->m_calls = ss.m_calls;
      info->spmv[0] = ss.outer;
    } else {
      int64_t per = 1;  // calls of level d per outermost iteration
      info->spmv[0] = ss.outer;
      for (int d = 1; d < p.nlev; d++) {
        if (p.lev[d].kind == F3R_FGMRES) {
          info->spmv[d] = (int64_t)ss.outer * per * p.lev[d].m;
        } else {
          info->spmv[d] = ss.r_calls * (p.lev[d].m - 1) + ss.upd_calls * p.lev[d].m;
        }
        per *= p.lev[d].m;
      }
      info->m_calls = (int64_t)ss.outer * per;
      info->r_calls = ss.r_calls;
    }
    // device counters
    int64_t fbk = 0, brk = 0;
    for (size_t d = 0; d < h->lev.size(); d++) {
      if (!h->lev[d].I) continue;
      int v[2];
      HIPCHK(hipMemcpy(v, h->lev[d].I + I_FALLBACKS, 2 * sizeof(int), hipMemcpyDeviceToHost));
      fbk += v[0];
      brk += v[1];
    }
    info->fallbacks = fbk;
    info->breakdowns = brk;
    info->relres_est = ss.est;
    info->relres_true = ss.relres;
    info->setup_ms = h->setup_ms;
    info->solve_ms = t1 - t0;
    info->graph_launches = h->graph_launches;
    info->idx_bits = h->A.idx16 ? 16 : 32;
    info->sell_c = 64;
    probe_collect(h);
    info->probe_ms = h->probe_ms;
    info->probe_launches = h->probe_n;
    info->padded_nnz = h->padded;
    for (int f = 0; f < 3; f++) {
      info->rows_per_lane[f] = h->kr[f] / 10;
      info->entry_chunk[f] = h->kr[f] % 10;
    }
    info->tune_ms = h->tune_ms;
  }
  return status;
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

f3r_status f3r_setup(const f3r_csr* A, const f3r_params* p, void* hip_stream, f3r_handle** out) {
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
    // workspaces
    int maxdots = p->lev[0].m + 2;
    maxdots = std::max(maxdots, 66);
    h->partials = h->dalloc((size_t)maxdots * (size_t)n_blocks(n) * sizeof(double));
    h->tmp64 = (double*)h->dalloc((size_t)n * 8);
    h->tmp64b = (double*)h->dalloc((size_t)n * 8);
    h->one = (double*)h->dalloc(sizeof(double));
    const double one = 1.0;
    HIPCHK(hipMemcpyAsync(h->one, &one, sizeof(double), hipMemcpyHostToDevice, h->st));
    HIPCHK(hipHostMalloc((void**)&h->hpin, 64 * sizeof(double), hipHostMallocDefault));
    std::memset(h->hpin, 0, 64 * sizeof(double));
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
    if (h->p.c != saved.c || h->p.poison_call != saved.poison_call) destroy_graphs(h);
  }
  f3r_status s = guarded(h, info, [&]() {
    HIPCHK(hipSetDevice(h->device));
    return outer_solve(h, b, x, tol, h->p.lev[0].m, h->p.max_outer, false,
                       !(h->p.flags & F3R_NO_GRAPH), info);
  });
  if (lo) {
    if (h->p.c != saved.c || h->p.poison_call != saved.poison_call) destroy_graphs(h);
    h->p = saved;
  }
  return s;
}

f3r_status f3r_fgmres_solve(f3r_handle* h, const double* b, double* x, double tol, int32_t m,
                            int32_t max_iter, f3r_info* info) {
  if (!h || !b || !x || !(tol > 0.0) || m < 1 || max_iter < 1) return F3R_ERR_ARG;
  if (m > h->p.lev[0].m) return F3R_ERR_ARG;
  return guarded(h, info, [&]() {
    HIPCHK(hipSetDevice(h->device));
    return outer_solve(h, b, x, tol, m, max_iter, true, false, info);
  });
}

f3r_status f3r_get_history(const f3r_handle* h, int32_t level, double* buf, int64_t cap,
                           int64_t* len) {
  if (!h || level != 0 || cap < 0 || (cap > 0 && !buf)) return F3R_ERR_ARG;
  const int64_t k = std::min<int64_t>(cap, (int64_t)h->history.size());
  for (int64_t i = 0; i < k; i++) buf[i] = h->history[(size_t)i];
  if (len) *len = (int64_t)h->history.size();
  return F3R_OK;
}

f3r_status f3r_get_weights(f3r_handle* h, int32_t level, double* omega, int64_t* c_ntr) {
  if (!h || level != h->rich || h->rich < 0 || !omega) return F3R_ERR_ARG;
  return guarded(h, nullptr, [&]() {
    HIPCHK(hipStreamSynchronize(h->st));
    HIPCHK(hipMemcpy(omega, h->lev[level].omega, (size_t)h->lev[level].cfg.m * sizeof(double),
                     hipMemcpyDeviceToHost));
    if (c_ntr) *c_ntr = h->cntr;
    return F3R_OK;
  });
}

f3r_status f3r_set_weights(f3r_handle* h, int32_t level, const double* omega, int64_t c_ntr) {
  if (!h || level != h->rich || h->rich < 0 || !omega || c_ntr < 1) return F3R_ERR_ARG;
  return guarded(h, nullptr, [&]() {
    // weights are quantities of the level arithmetic (fp32 for narrow levels)
    std::vector<double> w(omega, omega + h->lev[level].cfg.m);
    if (h->lev[level].q == T32)
      for (double& v : w) v = (double)(float)v;
    HIPCHK(hipMemcpy(h->lev[level].omega, w.data(), w.size() * sizeof(double),
                     hipMemcpyHostToDevice));
    h->cntr = c_ntr;
    HIPCHK(hipMemcpy(h->lev[level].cntr_dev, &h->cntr, sizeof(int64_t), hipMemcpyHostToDevice));
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
    // the sweep shapes of the solve (picked at set-up)
    hipError_t e = m_apply_w(h->st, h->A, mv, tm, neg, in, t, prec, nullptr, nullptr, h->kr[0]);
    if (e == hipErrorInvalidValue) return F3R_ERR_ARG;
    HIPCHK(e);
    // y (type prec) into tmp64 (the input is dead now)
    HIPCHK(m_apply_g(h->st, h->A, mv, tm, neg, gd, t, prec, 0, nullptr, nullptr, h->tmp64, prec,
                     nullptr, nullptr, nullptr, nullptr, h->kr[1]));
    HIPCHK(convert(h->st, n, h->tmp64, prec, y, T64));
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
    int64_t ncalls = 0;
    if (h->rich >= 0) {
      ncalls = 1;
      for (int d = level; d < h->rich; d++) ncalls *= h->p.lev[d].m;
    }
    RSched rs = make_sched(h, ncalls, 0);
    if (h->rich >= 0 && h->cntr == 1)
      HIPCHK(set_omega(h->st, h->lev[h->rich].omega, h->lev[h->rich].cfg.m, omega_init_q(h)));
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
    h->cntr += ncalls;
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

f3r_status f3r_debug_level_values(f3r_handle* h, int32_t prec, double* vals_host) {
  if (!h || !vals_host || !prec_ok(prec) || !h->ah[prec]) return F3R_ERR_ARG;
  return guarded(h, nullptr, [&]() {
    double* d = (double*)h->dalloc((size_t)h->nnz * 8);
    HIPCHK(sell_to_csr_values(h->st, h->n, h->rp, h->off, h->ah[prec], prec, d));
    HIPCHK(hipMemcpyAsync(vals_host, d, (size_t)h->nnz * 8, hipMemcpyDeviceToHost, h->st));
    HIPCHK(hipStreamSynchronize(h->st));
    h->al.release(d);
    return F3R_OK;
  });
}

}  // extern "C"
