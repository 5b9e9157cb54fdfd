// Batched F3R in one persistent launch.
//
// Every workgroup (512 threads) takes a system from a queue ordered by
// decreasing size and runs the whole nest on it: the fp64 outermost FGMRES
// with its restarts and stopping test (Sec. 4.2, Sec. 5), the fp32 second
// level, the fp16/bf16-matrix third level and the narrow Richardson level
// with the adaptive weights of Alg. 1 and Eq. (5), and M (Sec. 5.2).  A level
// step is the same sequence of sweeps as in the per-kernel path, separated
// by workgroup barriers instead of kernel boundaries, and the arithmetic of
// every stored value is the one of Table 1: each sweep rounds exactly like
// the kernel it replaces.  Only the order of the terms of the dot products
// and norms differs (one workgroup sums everything), and the per-iteration
// stopping test is taken on the device instead of the host.
//
// Sparse sweeps use the SELL-64 slices of the system (wave w takes slice
// groups w, w + 8, ...); vector sweeps give thread t the rows t, t + 512, ...
// Workgroup sums go through a wave shuffle and a fixed-order sum of the 8
// wave results in LDS, so every thread gets the same value and a run is
// bitwise repeatable.
#include "batch.h"
#include "common.h"
#include "f3r.h"
#include "kernels.h"
#include "sell.h"

namespace f3r {

namespace {

constexpr int kBT = kBatchThreads;
constexpr int kBW = kBT / kWave;
constexpr int kMI = kBatchMaxInner;
constexpr int kM1 = kBatchMaxM1;
// slices per wave in the sparse sweeps (rows per lane): with two, the whole
// solver fits the 256 registers per lane of a 512-thread workgroup without
// spilling
constexpr int kRB = 2;

struct WsLayout {
  size_t V1, Z1, H1, V2, Z2, V3, Z3, R, total;
  __host__ __device__ static size_t up(size_t b) { return (b + 255) & ~(size_t)255; }
  __host__ __device__ WsLayout(int64_t n, int m1, int m2, int m3) {
    const size_t un = (size_t)n;
    V1 = 0;
    Z1 = V1 + up((size_t)(m1 + 1) * un * 8);
    H1 = Z1 + up((size_t)m1 * un * 4);
    V2 = H1 + up((size_t)(m1 + 1) * (size_t)m1 * 8);
    Z2 = V2 + up((size_t)(m2 + 1) * un * 4);
    V3 = Z2 + up((size_t)m2 * un * 4);
    Z3 = V3 + up((size_t)m3 * un * 4);
    R = Z3 + up((size_t)m3 * un * 2);
    total = R + up(5 * un * 2);
  }
};

// an fp32 FGMRES level (second or third): Hessenberg matrix (column-major,
// leading dimension kMI + 1), rotations, right-hand side, solution, scales
// of the lazily normalised basis and the fallback flags of its directions
struct Small {
  float H[(kMI + 1) * kMI];
  float g[kMI + 1], cs[kMI], sn[kMI], y[kMI], sc[kMI + 1];
  float cbeta;
  int fb[kMI];
  int meff, stop, bad, solved;
};

struct Shm {
  double red[2 * kBW * 8];
  double h[kM1 + 1];
  double g1[kM1 + 1], cs1[kM1], sn1[kM1], y1[kM1], sc1[kM1 + 1];
  int fb1[kM1];
  Small L2, L3;
  float om[kMI];
  double est;
  int meff1, stop1, bad1, sys;
  int fallbacks, breakdowns;
  int64_t upd_calls;
};

// ---- workgroup sums (all threads receive the result) ----------------------
template <int K, class Q> __device__ __forceinline__ void bsum(Q (&v)[K], Shm& sh, int& ph) {
  static_assert(K <= 8, "at most 8 sums at once");
  Q* buf = reinterpret_cast<Q*>(sh.red + ph * kBW * 8);
  const int wave = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
#pragma unroll
  for (int k = 0; k < K; k++) v[k] = wave_sum(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < K; k++) buf[wave * K + k] = v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; k++) {
    Q s = 0;
    for (int w = 0; w < kBW; w++) s = s + buf[w * K + k];
    v[k] = s;
  }
  ph ^= 1;  // the next sum uses the other half, so no second barrier is needed
}

// ---- loaders ---------------------------------------------------------------
// round_TT((Q)(raw_c * sc)): a lazily normalised basis vector as the
// consumer's storage type
template <class TIN, class TT, class Q> struct LdSc {
  const TIN* p;
  double sc;
  __device__ __forceinline__ Q operator()(int64_t c) const {
    const Q v = (Q)(widen<double>(p[c]) * sc);
    return widen<Q>(round_to<TT>(v));
  }
};
// a direction of the outermost level: z_c = s_c u_c with u the fp32 output
// of the second level
struct LdZS {
  const float* z;
  const double* s;
  __device__ __forceinline__ double operator()(int64_t c) const { return s[c] * (double)z[c]; }
};

// ---- Givens step and triangular solve (one thread) -----------------------
// Same operations, in the same order and precision, as the per-kernel path.
template <class Q, class E>
__device__ void givens_step(E* H, int ld, E* g, E* cs, E* sn, E* sc, E& cbeta, Q s, int j, int fbj,
                            int& meff, int& stop, int& bad, int& fallbacks, int& breakdowns) {
  const Q hn = sqrt(s);
  E* col = H + (int64_t)j * ld;
  for (int i = 0; i < j; i++) {
    const Q a0 = (Q)col[i], a1 = (Q)col[i + 1];
    const Q c = (Q)cs[i], sv = (Q)sn[i];
    col[i] = (E)(c * a0 + sv * a1);
    col[i + 1] = (E)(-sv * a0 + c * a1);
  }
  if (fbj) fallbacks++;
  const Q hjj = (Q)col[j];
  const Q rho = (Q)hypot((double)hjj, (double)hn);
  stop = 0;
  if (!(rho != (Q)0) || !isfinite((double)rho) || !isfinite((double)hn)) {
    meff = j;
    breakdowns++;
    if (!isfinite((double)rho) || !isfinite((double)hn)) bad = 1;
    stop = 1;
  } else {
    const Q c = hjj / rho, sv = hn / rho;
    cs[j] = (E)c;
    sn[j] = (E)sv;
    col[j] = (E)rho;
    col[j + 1] = (E)0;
    const Q gj = (Q)g[j];
    g[j + 1] = (E)(-sv * gj);
    g[j] = (E)(c * gj);
    meff = j + 1;
    if (hn == (Q)0) {
      breakdowns++;
      stop = 1;
    } else {
      const Q inv = (Q)1 / hn;
      sc[j + 1] = (E)inv;
      cbeta = (E)(hn * inv);
    }
  }
}

template <class Q, class E>
__device__ void back_subst(const E* H, int ld, const E* g, E* y, int meff) {
  for (int i = meff - 1; i >= 0; i--) {
    Q acc = (Q)g[i];
    for (int k = i + 1; k < meff; k++) acc = acc - (Q)H[i + (int64_t)k * ld] * (Q)y[k];
    y[i] = (E)(acc / (Q)H[i + (int64_t)i * ld]);
  }
}

// ---- epilogues of the G sweep ----------------------------------------------
template <class TT> struct EpiStoreB {
  TT* out;
  __device__ __forceinline__ void prefetch(int, int64_t) {}
  __device__ __forceinline__ void operator()(int, int64_t r, TT y) { out[r] = y; }
};
// z = round(w y) (first step) or round(z_prev + w y)
template <class TT, bool PREV> struct EpiZ {
  TT* out;
  const TT* zp;
  float w;
  int bad;
  float zv[kRB];
  __device__ __forceinline__ void prefetch(int k, int64_t r) {
    if (PREV) zv[k] = widen<float>(zp[r]);
  }
  __device__ __forceinline__ void operator()(int k, int64_t r, TT y) {
    const TT z = PREV ? round_to<TT>(zv[k] + w * widen<float>(y)) : round_to<TT>(w * widen<float>(y));
    out[r] = z;
    bad |= !finite_val(z);
  }
};

template <class TI, class T16> struct Solver {
  const BatchArgs& P;
  const BatchSys& S;
  Shm& sh;
  int ph = 0;
  int64_t n;
  SellDesc A;
  WsLayout L;
  double* V1;
  float* Z1;
  double* H1;
  float* V2;
  float* Z2;
  float* V3;
  T16* Z3;
  T16* R;
  const TI* idx;

  __device__ Solver(const BatchArgs& p, const BatchSys& s, Shm& shm)
      : P(p), S(s), sh(shm), n(s.A.n), A(s.A), L(s.A.n, p.m1, p.m2, p.m3) {
    V1 = (double*)(S.ws + L.V1);
    Z1 = (float*)(S.ws + L.Z1);
    H1 = (double*)(S.ws + L.H1);
    V2 = (float*)(S.ws + L.V2);
    Z2 = (float*)(S.ws + L.Z2);
    V3 = (float*)(S.ws + L.V3);
    Z3 = (T16*)(S.ws + L.Z3);
    R = (T16*)(S.ws + L.R);
    idx = (const TI*)A.idx;
  }

  __device__ int64_t groups() const { return (A.ns + kRB - 1) / kRB; }
  __device__ static int wave_id() { return __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave)); }

  // ---- sparse sweeps -------------------------------------------------------
  // y = round_TY(A x), entries summed left to right in Q
  template <class TA, class TY, class Q, class LD>
  __device__ void spmv(const TA* av, const LD& x, TY* y) {
    const int wave = wave_id(), lane = threadIdx.x & (kWave - 1);
    for (int64_t gw = wave; gw < groups(); gw += kBW) {
      RowSlot s[kRB];
      make_slots(A, gw, lane, s);
      int kb[kRB], ke[kRB], kc[kRB];
      Q acc[kRB];
#pragma unroll
      for (int r = 0; r < kRB; r++) {
        kb[r] = 0;
        ke[r] = s[r].w;
        kc[r] = max(s[r].w, 1);
        acc[r] = 0;
      }
      rows_sum<kUnroll, TI>(av, idx, s, kb, kc, kb, ke, acc, x);
#pragma unroll
      for (int r = 0; r < kRB; r++)
        if (s[r].ok) y[s[r].row] = round_to<TY>(acc[r]);
    }
  }

  // out = b - A x in fp64; returns this thread's part of ||out||^2
  __device__ double residual64(const double* x, double* out) {
    const int wave = wave_id(), lane = threadIdx.x & (kWave - 1);
    double sq = 0.0;
    for (int64_t gw = wave; gw < groups(); gw += kBW) {
      RowSlot s[kRB];
      make_slots(A, gw, lane, s);
      int kb[kRB], ke[kRB], kc[kRB];
      double acc[kRB];
#pragma unroll
      for (int r = 0; r < kRB; r++) {
        kb[r] = 0;
        ke[r] = s[r].w;
        kc[r] = max(s[r].w, 1);
        acc[r] = 0.0;
      }
      rows_sum<kUnroll, TI>(S.a64, idx, s, kb, kc, kb, ke, acc, LdVec<double, double>{x});
#pragma unroll
      for (int r = 0; r < kRB; r++) {
        if (s[r].ok) {
          const double rv = S.b[s[r].row] - acc[r];
          out[s[r].row] = rv;
          sq = sq + rv * rv;
        }
      }
    }
    return sq;
  }

  // t = round(v_i + sum_{j<i} m_ij v_j): the W sweep of M
  template <class LD> __device__ void w_sweep(const LD& v, T16* t) {
    const T16* mv = (const T16*)S.m16;
    const int wave = wave_id(), lane = threadIdx.x & (kWave - 1);
    for (int64_t gw = wave; gw < groups(); gw += kBW) {
      RowSlot s[kRB];
      make_slots(A, gw, lane, s);
      int lo[kRB], hi[kRB], kb[kRB], ke[kRB];
      float acc[kRB], dg[kRB];
#pragma unroll
      for (int r = 0; r < kRB; r++) {
        const int64_t slice = gw * kRB + r;
        lo[r] = 0;
        hi[r] = s[r].ok ? max(A.dell_w ? A.dell_kd : (int)(A.kdr[slice] >> 16), 1) : 1;
        kb[r] = 0;
        ke[r] = s[r].ok ? (A.dell_w ? A.dell_kd : (int)A.kd[s[r].row]) : 0;
        acc[r] = 0.f;
      }
#pragma unroll
      for (int r = 0; r < kRB; r++) dg[r] = v(s[r].row);
      rows_sum<kUnroll, TI>(mv, idx, s, lo, hi, kb, ke, acc, v, P.neg != 0);
#pragma unroll
      for (int r = 0; r < kRB; r++)
        if (s[r].ok) t[s[r].row] = round_to<T16>(acc[r] + dg[r]);
    }
  }

  // y = round(gd t_i + sum_{j>i} m_ij t_j): the G sweep, then the epilogue
  template <class EPI> __device__ void g_sweep(const T16* t, EPI& epi) {
    const T16* mv = (const T16*)S.m16;
    const int wave = wave_id(), lane = threadIdx.x & (kWave - 1);
    for (int64_t gw = wave; gw < groups(); gw += kBW) {
      RowSlot s[kRB];
      make_slots(A, gw, lane, s);
      int lo[kRB], hi[kRB], kb[kRB], ke[kRB];
      float acc[kRB];
#pragma unroll
      for (int r = 0; r < kRB; r++) {
        const int64_t slice = gw * kRB + r;
        const int kd = s[r].ok ? (A.dell_w ? A.dell_kd : (int)A.kd[s[r].row]) : 0;
        lo[r] = s[r].ok ? (A.dell_w ? A.dell_kd : (int)(A.kdr[slice] & 0xffffu)) + 1 : 0;
        hi[r] = s[r].ok ? s[r].w : 1;
        kb[r] = s[r].ok ? kd + 1 : 0;
        ke[r] = s[r].ok ? s[r].w : 0;
        acc[r] = P.gd * widen<float>(t[s[r].row]);
        epi.prefetch(r, s[r].row);
      }
      rows_sum<kUnroll, TI>(mv, idx, s, lo, hi, kb, ke, acc, LdVec<T16, float>{t}, P.neg != 0);
#pragma unroll
      for (int r = 0; r < kRB; r++)
        if (s[r].ok) epi(r, s[r].row, round_to<T16>(acc[r]));
    }
  }

  // r = round(v_i - (A z)_i) on the narrow matrix
  template <class LD> __device__ void rich_residual(const LD& v, const T16* z, T16* r) {
    const T16* av = (const T16*)S.a16;
    const int wave = wave_id(), lane = threadIdx.x & (kWave - 1);
    for (int64_t gw = wave; gw < groups(); gw += kBW) {
      RowSlot s[kRB];
      make_slots(A, gw, lane, s);
      int kb[kRB], ke[kRB], kc[kRB];
      float acc[kRB], vr[kRB];
#pragma unroll
      for (int q = 0; q < kRB; q++) {
        kb[q] = 0;
        ke[q] = s[q].w;
        kc[q] = max(s[q].w, 1);
        acc[q] = 0.f;
      }
#pragma unroll
      for (int q = 0; q < kRB; q++) vr[q] = v(s[q].row);
      rows_sum<kUnroll, TI>(av, idx, s, kb, kc, kb, ke, acc, LdVec<T16, float>{z});
#pragma unroll
      for (int q = 0; q < kRB; q++)
        if (s[q].ok) r[s[q].row] = round_to<T16>(vr[q] - acc[q]);
    }
  }

  // t = A y kept in fp32; this thread's parts of (r, t) and (t, t)
  template <class LD> __device__ void rich_tdots(const T16* y, const LD& rv, float (&p)[2]) {
    const T16* av = (const T16*)S.a16;
    const int wave = wave_id(), lane = threadIdx.x & (kWave - 1);
    for (int64_t gw = wave; gw < groups(); gw += kBW) {
      RowSlot s[kRB];
      make_slots(A, gw, lane, s);
      int kb[kRB], ke[kRB], kc[kRB];
      float acc[kRB];
#pragma unroll
      for (int q = 0; q < kRB; q++) {
        kb[q] = 0;
        ke[q] = s[q].w;
        kc[q] = max(s[q].w, 1);
        acc[q] = 0.f;
      }
      rows_sum<kUnroll, TI>(av, idx, s, kb, kc, kb, ke, acc, LdVec<T16, float>{y});
#pragma unroll
      for (int q = 0; q < kRB; q++) {
        if (s[q].ok) {
          const float r = rv(s[q].row);
          p[0] = p[0] + r * acc[q];
          p[1] = p[1] + acc[q] * acc[q];
        }
      }
    }
  }

  // ---- vector sweeps -------------------------------------------------------
  // h_i = (w, raw_i) * sc_i for i < nv, basis V_0 = v0, V_i = vb + (i-1) n
  template <class TY, class Q, class HT, class SC>
  __device__ void multidot(const TY* w, const TY* v0, const TY* vb, int nv, const SC* sc, HT* h) {
    for (int i0 = 0; i0 < nv; i0 += 4) {
      const TY* V[4];
#pragma unroll
      for (int u = 0; u < 4; u++) {
        const int i = min(i0 + u, nv - 1);
        V[u] = i == 0 ? v0 : vb + (int64_t)(i - 1) * n;
      }
      Q acc[4] = {0, 0, 0, 0};
      for (int64_t row = threadIdx.x; row < n; row += kBT) {
        const Q wv = widen<Q>(w[row]);
        Q vv[4];
#pragma unroll
        for (int u = 0; u < 4; u++) vv[u] = widen<Q>(V[u][row]);
#pragma unroll
        for (int u = 0; u < 4; u++) acc[u] = acc[u] + wv * vv[u];
      }
      bsum<4>(acc, sh, ph);
      if (threadIdx.x == 0) {
#pragma unroll
        for (int u = 0; u < 4; u++)
          if (i0 + u < nv) h[i0 + u] = (HT)(acc[u] * (Q)sc[i0 + u]);
      }
    }
    __syncthreads();
  }

  // w <- round(w - sum_i h_i round(raw_i sc_i)); returns this thread's part
  // of ||w||^2
  template <class TY, class Q, class HT, class SC>
  __device__ Q axpy_norm(TY* w, const TY* v0, const TY* vb, int nv, const HT* h, const SC* sc) {
    Q sq = 0;
    for (int64_t row = threadIdx.x; row < n; row += kBT) {
      Q acc = widen<Q>(w[row]);
      for (int l = 0; l < nv; l++) {
        const TY* V = l == 0 ? v0 : vb + (int64_t)(l - 1) * n;
        const Q v = widen<Q>(round_to<TY>(widen<Q>(V[row]) * (Q)sc[l]));
        acc = acc - (Q)h[l] * v;
      }
      const TY wr = round_to<TY>(acc);
      w[row] = wr;
      const Q q = widen<Q>(wr);
      sq = sq + q * q;
    }
    return sq;
  }

  // ---- Richardson level (Alg. 1) ------------------------------------------
  // z = R(v) for the input v = round_narrow(raw * sc); cn is the call counter
  // c_ntr of this call.  Returns nonzero when z has a non-finite entry.
  __device__ int richardson(const float* vraw, double vsc, T16* out, int64_t cn) {
    const bool upd = P.c > 0 && cn % P.c == 0;
    const LdSc<float, T16, float> vin{vraw, vsc};
    T16* rr = R;
    T16* rt = R + n;
    T16* ry = R + 2 * n;
    T16* rz[2] = {R + 3 * n, R + 4 * n};
    const T16* zprev = nullptr;
    int bad = 0;
    if (upd && threadIdx.x == 0) sh.upd_calls++;
    for (int k = 0; k < P.m4; k++) {
      const bool last = k == P.m4 - 1;
      T16* zk = last ? out : rz[k & 1];
      if (k == 0) {
        w_sweep(vin, rt);
      } else {
        rich_residual(vin, zprev, rr);
        __syncthreads();
        w_sweep(LdVec<T16, float>{rr}, rt);
      }
      __syncthreads();
      int b = 0;
      if (!upd) {
        if (k == 0) {
          EpiZ<T16, false> e{zk, nullptr, sh.om[k], 0, {}};
          g_sweep(rt, e);
          b = e.bad;
        } else {
          EpiZ<T16, true> e{zk, zprev, sh.om[k], 0, {}};
          g_sweep(rt, e);
          b = e.bad;
        }
      } else {
        EpiStoreB<T16> e{ry};
        g_sweep(rt, e);
        __syncthreads();
        float p[2] = {0.f, 0.f};
        if (k == 0)
          rich_tdots(ry, vin, p);
        else
          rich_tdots(ry, LdVec<T16, float>{rr}, p);
        bsum<2>(p, sh, ph);
        // Eq. (5) with l = c_ntr / c: the initial weight counts as a sample
        const int64_t l = cn / P.c;
        const float wp = p[0] / p[1];
        const float wold = sh.om[k];
        float wc = wold, wnew = wold;
        if (p[1] > 0.f && isfinite(wp)) {
          float v = (float)l * wold;
          v = v + wp;
          v = v / (float)(l + 1);
          wnew = v;
          wc = wp;
        }
        __syncthreads();  // every thread has read the old weight
        if (threadIdx.x == 0) sh.om[k] = wnew;
        for (int64_t row = threadIdx.x; row < n; row += kBT) {
          const float pv = wc * widen<float>(ry[row]);
          const T16 z = zprev ? round_to<T16>(widen<float>(zprev[row]) + pv) : round_to<T16>(pv);
          zk[row] = z;
          b |= !finite_val(z);
        }
      }
      b = __syncthreads_or(last ? b : 0);
      if (last) bad = b;
      zprev = zk;
    }
    return bad;
  }

  // ---- third level: FGMRES(m3), fp16/bf16 matrix, fp32 vectors -----------
  // Input: the second level's basis vector j2 (raw fp32 with scale sc2[j2]);
  // output: Z2_j2.  Returns nonzero when the output has a non-finite entry.
  __device__ int level3(int j2, int64_t cn) {
    Small& L3 = sh.L3;
    const Small& L2 = sh.L2;
    const int m3 = P.m3;
    const int ld = kMI + 1;
    const float* v0 = V2 + (int64_t)j2 * n;
    if (threadIdx.x == 0) {
      L3.sc[0] = L2.sc[j2];
      L3.g[0] = L2.cbeta;  // the input's norm: h * (1 / h)
      for (int i = 1; i <= m3; i++) L3.g[i] = 0.f;
      for (int i = 0; i < m3; i++) L3.fb[i] = 0;
      L3.meff = 0;
      L3.stop = 0;
      L3.bad = 0;
      L3.solved = 0;
    }
    __syncthreads();
    for (int j = 0; j < m3; j++) {
      const float* vj = j == 0 ? v0 : V3 + (int64_t)(j - 1) * n;
      const float scj = L3.sc[j];
      T16* zj = Z3 + (int64_t)j * n;
      const int fbj = richardson(vj, (double)scj, zj, cn + j);
      if (threadIdx.x == 0) L3.fb[j] = fbj;
      float* w = V3 + (int64_t)j * n;
      if (!fbj)
        spmv<T16, float, float>((const T16*)S.a16, LdVec<T16, float>{zj}, w);
      else
        spmv<T16, float, float>((const T16*)S.a16, LdSc<float, float, float>{vj, (double)scj}, w);
      __syncthreads();
      multidot<float, float>(w, v0, V3, j + 1, L3.sc, L3.H + j * ld);
      float sq[1] = {axpy_norm<float, float>(w, v0, V3, j + 1, L3.H + j * ld, L3.sc)};
      bsum<1>(sq, sh, ph);
      if (threadIdx.x == 0) {
        givens_step<float, float>(L3.H, ld, L3.g, L3.cs, L3.sn, L3.sc, L3.cbeta, sq[0], j, L3.fb[j],
                                  L3.meff, L3.stop, L3.bad, sh.fallbacks, sh.breakdowns);
        if (L3.stop || j == m3 - 1) {
          back_subst<float, float>(L3.H, ld, L3.g, L3.y, L3.meff);
          L3.solved = 1;
        }
      }
      __syncthreads();
      if (L3.stop) break;
    }
    // Z2_j2 = sum_j y_j z_j (a flagged direction is replaced by its input)
    const int meff = L3.meff;
    int anyfb = 0;
    for (int j = 0; j < meff; j++) anyfb |= L3.fb[j];
    float* out = Z2 + (int64_t)j2 * n;
    int bad = 0;
    for (int64_t row = threadIdx.x; row < n; row += kBT) {
      float acc = 0.f;
      for (int j = 0; j < meff; j++) {
        float zv;
        if (anyfb && L3.fb[j]) {
          const float* V = j == 0 ? v0 : V3 + (int64_t)(j - 1) * n;
          zv = widen<float>(round_to<float>(V[row] * L3.sc[j]));
        } else {
          zv = widen<float>(Z3[(int64_t)j * n + row]);
        }
        acc = acc + L3.y[j] * zv;
      }
      const float o = round_to<float>(acc);
      out[row] = o;
      bad |= !finite_val(o);
    }
    return __syncthreads_or(bad);
  }

  // ---- second level: FGMRES(m2), fp32 ---------------------------------------
  // Input: the outermost basis vector j scaled by S; output: the fp32 vector
  // u with z_j = S u stored in Z1_j.  Returns nonzero when S u is not finite.
  __device__ int level2(int j, int64_t cn) {
    Small& L2 = sh.L2;
    const int m2 = P.m2, m3 = P.m3;
    const int ld = kMI + 1;
    const double* vr = V1 + (int64_t)j * n;
    const double sc = sh.sc1[j];
    float sq[1] = {0.f};
    for (int64_t row = threadIdx.x; row < n; row += kBT) {
      const float o = round_to<float>(S.s[row] * (vr[row] * sc));
      V2[row] = o;
      sq[0] = sq[0] + o * o;
    }
    bsum<1>(sq, sh, ph);
    {
      const float beta = sqrtf(sq[0]);
      const float inv = beta > 0.f ? 1.f / beta : 0.f;
      if (threadIdx.x == 0) {
        L2.sc[0] = inv;
        L2.g[0] = beta;
        L2.cbeta = beta * inv;
        for (int i = 1; i <= m2; i++) L2.g[i] = 0.f;
        for (int i = 0; i < m2; i++) L2.fb[i] = 0;
        L2.meff = 0;
        L2.stop = beta > 0.f && isfinite(beta) ? 0 : 1;
        L2.bad = 0;
        L2.solved = 0;
      }
    }
    __syncthreads();
    if (!L2.stop) {
      for (int j2 = 0; j2 < m2; j2++) {
        const int fbj = level3(j2, cn + (int64_t)j2 * m3);
        if (threadIdx.x == 0) L2.fb[j2] = fbj;
        const float* vj = V2 + (int64_t)j2 * n;
        float* w = V2 + (int64_t)(j2 + 1) * n;
        if (!fbj)
          spmv<float, float, float>(S.a32, LdVec<float, float>{Z2 + (int64_t)j2 * n}, w);
        else
          spmv<float, float, float>(S.a32, LdSc<float, float, float>{vj, (double)L2.sc[j2]}, w);
        __syncthreads();
        multidot<float, float>(w, V2, V2 + n, j2 + 1, L2.sc, L2.H + j2 * ld);
        float s2[1] = {axpy_norm<float, float>(w, V2, V2 + n, j2 + 1, L2.H + j2 * ld, L2.sc)};
        bsum<1>(s2, sh, ph);
        if (threadIdx.x == 0) {
          givens_step<float, float>(L2.H, ld, L2.g, L2.cs, L2.sn, L2.sc, L2.cbeta, s2[0], j2,
                                    L2.fb[j2], L2.meff, L2.stop, L2.bad, sh.fallbacks,
                                    sh.breakdowns);
          if (L2.stop || j2 == m2 - 1) {
            back_subst<float, float>(L2.H, ld, L2.g, L2.y, L2.meff);
            L2.solved = 1;
          }
        }
        __syncthreads();
        if (L2.stop) break;
      }
    }
    const int meff = L2.meff;
    int anyfb = 0;
    for (int i = 0; i < meff; i++) anyfb |= L2.fb[i];
    float* out = Z1 + (int64_t)j * n;
    int bad = 0;
    for (int64_t row = threadIdx.x; row < n; row += kBT) {
      float acc = 0.f;
      for (int i = 0; i < meff; i++) {
        float zv;
        if (anyfb && L2.fb[i])
          zv = widen<float>(round_to<float>(V2[(int64_t)i * n + row] * L2.sc[i]));
        else
          zv = Z2[(int64_t)i * n + row];
        acc = acc + L2.y[i] * zv;
      }
      const float o = round_to<float>(acc);
      out[row] = o;
      bad |= !isfinite(S.s[row] * (double)o);
    }
    return __syncthreads_or(bad);
  }

  // ---- outermost level and the solve ---------------------------------------
  __device__ void run() {
    BatchOut res{};
    const int m1 = P.m1;
    const int ld1 = m1 + 1;
    const int64_t per_f2 = (int64_t)P.m2 * P.m3;  // Richardson calls of one second-level call
    double bb[1] = {0.0};
    for (int64_t row = threadIdx.x; row < n; row += kBT) bb[0] = bb[0] + S.b[row] * S.b[row];
    bsum<1>(bb, sh, ph);
    const double bnorm = sqrt(bb[0]);
    if (threadIdx.x == 0) {
      sh.fallbacks = 0;
      sh.breakdowns = 0;
      sh.upd_calls = 0;
    }
    int status = F3R_NOT_CONVERGED;
    double relres = 0.0, est = 0.0;
    int outer = 0, restarts = 0;
    int64_t cntr = 1;
    if (bnorm == 0.0) {
      for (int64_t row = threadIdx.x; row < n; row += kBT) S.x[row] = 0.0;
      status = 0;
    } else if (!isfinite(bnorm)) {
      status = F3R_ERR_ARG;
    } else {
      const double inv_bnorm = 1.0 / bnorm;
      if (!P.use_x0)
        for (int64_t row = threadIdx.x; row < n; row += kBT) S.x[row] = 0.0;
      // Alg. 1: the weights start at omega_init for the first call
      if ((int)threadIdx.x < P.m4) sh.om[threadIdx.x] = P.omega_init;
      __syncthreads();
      double rr[1] = {residual64(S.x, V1)};
      bsum<1>(rr, sh, ph);
      double beta = sqrt(rr[0]);
      relres = beta * inv_bnorm;
      if (!isfinite(relres)) status = F3R_ERR_BREAKDOWN;
      else if (relres < P.tol) status = 0;
      while (status == F3R_NOT_CONVERGED && outer < P.max_outer) {
        if (threadIdx.x == 0) {
          sh.sc1[0] = beta > 0 ? 1.0 / beta : 0.0;
          sh.g1[0] = beta;
          for (int i = 1; i <= m1; i++) sh.g1[i] = 0.0;
          sh.meff1 = 0;
          sh.stop1 = 0;
          sh.bad1 = 0;
        }
        __syncthreads();
        const int len = min(m1, P.max_outer - outer);
        int it = 0;
        bool bad = false;
        for (int j = 0; j < len; j++) {
          const int fbj = level2(j, cntr);
          cntr += per_f2;
          if (threadIdx.x == 0) sh.fb1[j] = fbj;
          double* w = V1 + (int64_t)(j + 1) * n;
          if (!fbj)
            spmv<double, double, double>(S.a64, LdZS{Z1 + (int64_t)j * n, S.s}, w);
          else
            spmv<double, double, double>(S.a64, LdSc<double, double, double>{V1 + (int64_t)j * n, sh.sc1[j]}, w);
          __syncthreads();
          multidot<double, double>(w, V1, V1 + n, j + 1, sh.sc1, sh.h);
          double s1[1] = {axpy_norm<double, double>(w, V1, V1 + n, j + 1, sh.h, sh.sc1)};
          bsum<1>(s1, sh, ph);
          if (threadIdx.x == 0) {
            double* col = H1 + (int64_t)j * ld1;
            for (int i = 0; i <= j; i++) col[i] = sh.h[i];
            double cb = 0.0;
            givens_step<double, double>(H1, ld1, sh.g1, sh.cs1, sh.sn1, sh.sc1, cb, s1[0], j, sh.fb1[j],
                                        sh.meff1, sh.stop1, sh.bad1, sh.fallbacks, sh.breakdowns);
            sh.est = fabs(sh.g1[j + 1]) * inv_bnorm;
            S.hist[outer] = sh.est;
          }
          __syncthreads();
          it++;
          outer++;
          est = sh.est;
          if (sh.bad1) {
            bad = true;
            break;
          }
          if (est < P.tol || sh.stop1) break;
        }
        if (bad) {
          status = F3R_ERR_BREAKDOWN;
          break;
        }
        if (threadIdx.x == 0) back_subst<double, double>(H1, ld1, sh.g1, sh.y1, sh.meff1);
        __syncthreads();
        // x += sum_j y_j z_j
        const int meff = sh.meff1;
        int anyfb = 0;
        for (int i = 0; i < meff; i++) anyfb |= sh.fb1[i];
        for (int64_t row = threadIdx.x; row < n; row += kBT) {
          double acc = 0.0;
          for (int i = 0; i < meff; i++) {
            const double zv = (anyfb && sh.fb1[i]) ? V1[(int64_t)i * n + row] * sh.sc1[i]
                                                   : S.s[row] * (double)Z1[(int64_t)i * n + row];
            acc = acc + sh.y1[i] * zv;
          }
          S.x[row] = S.x[row] + acc;
        }
        __syncthreads();
        double r2[1] = {residual64(S.x, V1)};
        bsum<1>(r2, sh, ph);
        beta = sqrt(r2[0]);
        relres = beta * inv_bnorm;
        if (!isfinite(relres)) {
          status = F3R_ERR_BREAKDOWN;
          break;
        }
        if (relres < P.tol) {
          status = 0;
          break;
        }
        restarts++;
        if (it == 0) break;
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      res.status = status;
      res.outer = outer;
      res.restarts = restarts;
      res.fallbacks = sh.fallbacks;
      res.breakdowns = sh.breakdowns;
      res.r_calls = (int64_t)outer * per_f2;
      res.upd_calls = sh.upd_calls;
      res.relres_est = est;
      res.relres_true = relres;
      *S.out = res;
    }
  }

};

template <class TI, class T16>
__global__ __launch_bounds__(kBT) void k_batch(BatchArgs P) {
  __shared__ Shm sh;
  for (;;) {
    if (threadIdx.x == 0) sh.sys = atomicAdd(P.queue, 1);
    __syncthreads();
    const int k = __builtin_amdgcn_readfirstlane(sh.sys);
    __syncthreads();
    if (k >= P.count) break;
    Solver<TI, T16> s(P, P.sys[P.order[k]], sh);
    s.run();
    __syncthreads();
  }
}

}  // namespace

size_t batch_ws_bytes(int64_t n, int m1, int m2, int m3) { return WsLayout(n, m1, m2, m3).total; }

hipError_t batch_launch(hipStream_t st, const BatchArgs& a, int grid) {
  if (a.m1 < 1 || a.m1 > kM1 || a.m2 < 1 || a.m2 > kMI || a.m3 < 1 || a.m3 > kMI || a.m4 < 1 ||
      a.m4 > kMI || grid < 1)
    return hipErrorInvalidValue;
  const dim3 g((unsigned)grid), b(kBT);
  if (a.idx16) {
    if (a.bf16)
      hipLaunchKernelGGL((k_batch<int16_t, bf16>), g, b, 0, st, a);
    else
      hipLaunchKernelGGL((k_batch<int16_t, f16>), g, b, 0, st, a);
  } else {
    if (a.bf16)
      hipLaunchKernelGGL((k_batch<int32_t, bf16>), g, b, 0, st, a);
    else
      hipLaunchKernelGGL((k_batch<int32_t, f16>), g, b, 0, st, a);
  }
  return hipGetLastError();
}

}  // namespace f3r
