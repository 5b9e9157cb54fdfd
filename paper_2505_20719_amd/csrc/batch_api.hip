// Host side of the batched entry points of include/f3r.h: per-system set-up
// (the same set-up kernels as f3r_setup), workspace allocation, the
// processing order (largest system first, so the longest solves start
// first), and one persistent launch per column-index width.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "batch.h"
#include "f3r.h"
#include "host.h"
#include "kernels.h"

using namespace f3r;

struct f3r_batch {
  int device = 0;
  hipStream_t st = nullptr;
  f3r_params p{};
  int count = 0;
  std::vector<MatrixDev> mats;
  std::vector<char*> ws;
  DevAllocs al;
  BatchSys* dsys = nullptr;
  std::vector<BatchSys> hsys;
  int* dorder = nullptr;     // two groups: 16-bit then 32-bit column indices
  int* dqueue = nullptr;     // one counter per group
  BatchOut* dout = nullptr;
  double* dhist = nullptr;   // count x max_outer
  int n16 = 0;               // systems in the 16-bit group
  int grid_cap = 1;
  bool narrow_bf16 = false;
  float gd = 1.f;
  int neg = 1;
  double setup_ms = 0;
  std::vector<BatchOut> hout;
  std::vector<double> hist;
  f3r_handle* ls = nullptr;  // lockstep mode: the stacked systems
};

namespace {

double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

bool narrow(int t) { return t == F3R_FP16 || t == F3R_BF16; }

f3r_status check_batch_params(const f3r_params* p) {
  if (!p || p->nlev != 4) return F3R_ERR_ARG;
  const f3r_level* L = p->lev;
  if (L[0].kind != F3R_FGMRES || L[1].kind != F3R_FGMRES || L[2].kind != F3R_FGMRES ||
      L[3].kind != F3R_RICHARDSON)
    return F3R_ERR_ARG;
  const int t = L[3].prec_v;
  if (!narrow(t)) return F3R_ERR_ARG;
  if (L[0].prec_a != F3R_FP64 || L[0].prec_v != F3R_FP64) return F3R_ERR_ARG;
  if (L[1].prec_a != F3R_FP32 || L[1].prec_v != F3R_FP32) return F3R_ERR_ARG;
  if (L[2].prec_a != t || L[2].prec_v != F3R_FP32) return F3R_ERR_ARG;
  if (L[3].prec_a != t || p->prec_m != t) return F3R_ERR_ARG;
  if (L[0].m < 1 || L[0].m > kBatchMaxM1) return F3R_ERR_ARG;
  for (int d = 1; d < 4; d++)
    if (L[d].m < 1 || L[d].m > kBatchMaxInner) return F3R_ERR_ARG;
  if (p->m_identity != 0 || p->c < 0 || p->max_outer < 1) return F3R_ERR_ARG;
  if (!(p->alpha > 0.0) || !std::isfinite(p->alpha) || !std::isfinite(p->omega_init)) return F3R_ERR_ARG;
  if ((p->flags & ~F3R_USE_X0) != 0 || p->poison_call != 0 || p->probe_kernel != 0) return F3R_ERR_ARG;
  return F3R_OK;
}

template <class F> f3r_status guarded_b(F&& f, int32_t* hip_error) {
  try {
    return f();
  } catch (const StatusErr& e) {
    return e.s;
  } catch (const DevErr& e) {
    if (hip_error) *hip_error = (int32_t)e.e;
    return F3R_ERR_DEVICE;
  } catch (...) {
    return F3R_ERR_DEVICE;
  }
}

// severity order for the combined status of a batch
int severity(f3r_status s) {
  if (s == F3R_OK) return 0;
  if (s == F3R_NOT_CONVERGED) return 1;
  return 2 - s;  // every error is worse than not converging
}

}  // namespace

extern "C" {

void f3r_batch_destroy(f3r_batch* bt) {
  if (!bt) return;
  if (bt->ls) f3r_destroy(bt->ls);
  (void)hipSetDevice(bt->device);
  if (bt->st) (void)hipStreamSynchronize(bt->st);
  bt->al.release_all();
  delete bt;
}

f3r_status f3r_setup_batched(int32_t count, const f3r_csr* A, const f3r_params* p, void* hip_stream,
                             f3r_batch** out) {
  if (!out) return F3R_ERR_ARG;
  *out = nullptr;
  if (count < 1 || !A || !p) return F3R_ERR_ARG;
  if (p->m_kind != F3R_M_SGS) return F3R_ERR_ARG;  // batches use the two-sweep M
  if (p->flags & F3R_BATCH_LOCKSTEP) {
    f3r_params q = *p;
    q.flags &= ~F3R_BATCH_LOCKSTEP;
    if (q.poison_call != 0 || q.probe_kernel != 0 || (q.flags & F3R_PERSIST_WEIGHTS)) return F3R_ERR_ARG;
    f3r_batch* bt = new f3r_batch();
    bt->p = *p;
    bt->count = count;
    bt->st = (hipStream_t)hip_stream;
    const double t0 = now_ms();
    const f3r_status st = stacked_setup(count, A, &q, hip_stream, &bt->ls);
    bt->setup_ms = now_ms() - t0;
    if (st != F3R_OK) {
      f3r_batch_destroy(bt);
      return st;
    }
    *out = bt;
    return F3R_OK;
  }
  const f3r_status ps = check_batch_params(p);
  if (ps != F3R_OK) return ps;
  f3r_batch* bt = new f3r_batch();
  bt->p = *p;
  bt->count = count;
  bt->st = (hipStream_t)hip_stream;
  const double t0 = now_ms();
  const f3r_status st = guarded_b(
      [&]() -> f3r_status {
        HIPCHK(hipGetDevice(&bt->device));
        int cus = 0;
        HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, bt->device));
        bt->grid_cap = std::max(cus, 1);
        const int t = p->prec_m;
        bt->narrow_bf16 = t == F3R_BF16;
        const bool need[4] = {false, false, false, false};
        bt->mats.resize((size_t)count);
        bt->ws.resize((size_t)count);
        for (int i = 0; i < count; i++) {
          const f3r_status bs = build_matrix(bt->st, &A[i], p, need, bt->al, bt->mats[(size_t)i], false);
          if (bs != F3R_OK) return bs;
          const MatrixDev& m = bt->mats[(size_t)i];
          bt->ws[(size_t)i] = (char*)bt->al.get(batch_ws_bytes(m.n, p->lev[0].m, p->lev[1].m, p->lev[2].m));
        }
        const MatrixDev& m0 = bt->mats[0];
        bt->neg = m0.m_shared ? 1 : 0;
        bt->gd = (float)m0.gd[t];
        // order: 16-bit index systems first, each group by decreasing padded size
        std::vector<int> ord((size_t)count);
        std::iota(ord.begin(), ord.end(), 0);
        std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) {
          const MatrixDev& ma = bt->mats[(size_t)a];
          const MatrixDev& mb = bt->mats[(size_t)b];
          if (ma.A.idx16 != mb.A.idx16) return ma.A.idx16 > mb.A.idx16;
          return ma.padded + 8 * ma.n > mb.padded + 8 * mb.n;
        });
        bt->n16 = 0;
        for (int i = 0; i < count; i++) bt->n16 += bt->mats[(size_t)i].A.idx16 ? 1 : 0;
        bt->hsys.resize((size_t)count);
        bt->dsys = (BatchSys*)bt->al.get(sizeof(BatchSys) * (size_t)count);
        bt->dorder = (int*)bt->al.get(sizeof(int) * (size_t)count);
        bt->dqueue = (int*)bt->al.get(2 * sizeof(int));
        bt->dout = (BatchOut*)bt->al.get(sizeof(BatchOut) * (size_t)count);
        bt->dhist = (double*)bt->al.get(sizeof(double) * (size_t)count * (size_t)p->max_outer);
        HIPCHK(hipMemcpyAsync(bt->dorder, ord.data(), sizeof(int) * (size_t)count, hipMemcpyHostToDevice,
                              bt->st));
        for (int i = 0; i < count; i++) {
          const MatrixDev& m = bt->mats[(size_t)i];
          BatchSys& s = bt->hsys[(size_t)i];
          std::memset(&s, 0, sizeof(s));
          s.A = m.A;
          s.a64 = m.a64;
          s.a32 = (const float*)m.ah[T32];
          s.a16 = m.ah[t];
          s.m16 = m.m_shared ? m.ah[t] : m.mv[t];
          s.s = m.s;
          s.ws = bt->ws[(size_t)i];
          s.hist = bt->dhist + (size_t)i * (size_t)p->max_outer;
          s.out = bt->dout + i;
        }
        bt->hout.resize((size_t)count);
        bt->hist.assign((size_t)count * (size_t)p->max_outer, 0.0);
        HIPCHK(hipStreamSynchronize(bt->st));
        return F3R_OK;
      },
      nullptr);
  bt->setup_ms = now_ms() - t0;
  if (st != F3R_OK) {
    f3r_batch_destroy(bt);
    return st;
  }
  *out = bt;
  return F3R_OK;
}

f3r_status f3r_solve_batched(f3r_batch* bt, const double* const* b, double* const* x, double tol,
                             f3r_info* infos) {
  if (!bt || !b || !x || !(tol > 0.0)) return F3R_ERR_ARG;
  for (int i = 0; i < bt->count; i++)
    if (!b[i] || !x[i]) return F3R_ERR_ARG;
  if (bt->ls) {
    const f3r_status st = stacked_solve(bt->ls, b, x, tol, infos);
    if (infos)
      for (int i = 0; i < bt->count; i++) infos[i].setup_ms = bt->setup_ms;
    return st;
  }
  int32_t herr = 0;
  const double t0 = now_ms();
  f3r_status st = guarded_b(
      [&]() -> f3r_status {
        HIPCHK(hipSetDevice(bt->device));
        for (int i = 0; i < bt->count; i++) {
          bt->hsys[(size_t)i].b = b[i];
          bt->hsys[(size_t)i].x = x[i];
        }
        HIPCHK(hipMemcpyAsync(bt->dsys, bt->hsys.data(), sizeof(BatchSys) * (size_t)bt->count,
                              hipMemcpyHostToDevice, bt->st));
        HIPCHK(hipMemsetAsync(bt->dqueue, 0, 2 * sizeof(int), bt->st));
        const f3r_params& p = bt->p;
        BatchArgs a{};
        a.sys = bt->dsys;
        a.m1 = p.lev[0].m;
        a.m2 = p.lev[1].m;
        a.m3 = p.lev[2].m;
        a.m4 = p.lev[3].m;
        a.c = p.c;
        a.max_outer = p.max_outer;
        a.use_x0 = (p.flags & F3R_USE_X0) ? 1 : 0;
        a.neg = bt->neg;
        a.bf16 = bt->narrow_bf16 ? 1 : 0;
        a.omega_init = (float)p.omega_init;
        a.gd = bt->gd;
        a.tol = tol;
        const int groups[2][2] = {{0, bt->n16}, {bt->n16, bt->count - bt->n16}};
        for (int g = 0; g < 2; g++) {
          const int cnt = groups[g][1];
          if (cnt == 0) continue;
          a.order = bt->dorder + groups[g][0];
          a.count = cnt;
          a.queue = bt->dqueue + g;
          a.idx16 = g == 0 ? 1 : 0;
          HIPCHK(batch_launch(bt->st, a, std::min(cnt, bt->grid_cap)));
        }
        HIPCHK(hipMemcpyAsync(bt->hout.data(), bt->dout, sizeof(BatchOut) * (size_t)bt->count,
                              hipMemcpyDeviceToHost, bt->st));
        HIPCHK(hipMemcpyAsync(bt->hist.data(), bt->dhist, sizeof(double) * bt->hist.size(),
                              hipMemcpyDeviceToHost, bt->st));
        HIPCHK(hipStreamSynchronize(bt->st));
        return F3R_OK;
      },
      &herr);
  const double t1 = now_ms();
  f3r_status worst = F3R_OK;
  for (int i = 0; i < bt->count; i++) {
    const BatchOut o = st == F3R_OK ? bt->hout[(size_t)i] : BatchOut{};
    const f3r_status si = st == F3R_OK ? (f3r_status)o.status : st;
    if (severity(si) > severity(worst)) worst = si;
    if (!infos) continue;
    f3r_info& in = infos[i];
    std::memset(&in, 0, sizeof(in));
    in.status = si;
    in.hip_error = herr;
    in.outer_iters = o.outer;
    in.restarts = o.restarts;
    const f3r_params& p = bt->p;
    int64_t per = 1;
    in.spmv[0] = o.outer;
    for (int d = 1; d < 3; d++) {
      in.spmv[d] = (int64_t)o.outer * per * p.lev[d].m;
      per *= p.lev[d].m;
    }
    in.spmv[3] = o.r_calls * (p.lev[3].m - 1) + o.upd_calls * p.lev[3].m;
    in.m_calls = (int64_t)o.outer * per * p.lev[3].m;
    in.r_calls = o.r_calls;
    in.fallbacks = o.fallbacks;
    in.breakdowns = o.breakdowns;
    in.relres_est = o.relres_est;
    in.relres_true = o.relres_true;
    in.setup_ms = bt->setup_ms;
    in.solve_ms = t1 - t0;
    in.idx_bits = bt->mats[(size_t)i].A.idx16 ? 16 : 32;
    in.sell_c = 64;
    in.padded_nnz = bt->mats[(size_t)i].padded;
    in.layout = bt->mats[(size_t)i].A.dell_w ? F3R_LAYOUT_DIAG : F3R_LAYOUT_SELL;
  }
  return worst;
}

f3r_status f3r_batch_get_history(const f3r_batch* bt, int32_t sys, double* buf, int64_t cap,
                                 int64_t* len) {
  if (!bt || sys < 0 || sys >= bt->count || cap < 0 || (cap > 0 && !buf)) return F3R_ERR_ARG;
  if (bt->ls) return stacked_history(bt->ls, sys, buf, cap, len);
  const int64_t avail = bt->hout[(size_t)sys].outer;
  const int64_t k = std::min(cap, avail);
  const double* h = bt->hist.data() + (size_t)sys * (size_t)bt->p.max_outer;
  for (int64_t i = 0; i < k; i++) buf[i] = h[i];
  if (len) *len = avail;
  return F3R_OK;
}

}  // extern "C"
