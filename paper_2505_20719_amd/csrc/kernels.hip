// Solve-phase kernels of libf3r for gfx950.
//
// Every sparse kernel works on the SELL-64 layout described in kernels.h:
// one row per lane of a wave64 and kR slices per wave (kR rows per lane),
// 4 waves per block.  A lane walks each row in CSR column order with separate
// multiply and add (no contraction), so a row sum is rounded exactly like
// the left-to-right sum that defines the level SpMV (Table 1 precisions;
// fp32 arithmetic when inputs are narrower, Sec. 4.2).  Reductions are
// deterministic: fixed shuffle pattern inside a wave, fixed order over the
// waves of a block, one partial per block, and a fixed-order final sum in a
// separate one-block kernel (a kernel boundary is the cross-XCD sync point).
#include <type_traits>

#include "common.h"
#include "ilu.h"
#include "kernels.h"
#include "sell.h"

namespace f3r {

static_assert(kRowsPerBlock == kSysAlign, "systems are aligned to reduction blocks");


// Shape of the sweeps whose shape the set-up autotuner picks (their results
// do not depend on it), coded as 10 KR + U: KR rows per lane, entries in
// chunks of U.  Chunks of 3 (7-point stencils have 3 entries on each side of
// the diagonal) exist for narrow vectors, and for every vector type in the
// slice-offset format, whose chunks read whole positions unclamped.  With
// WHOLE (the residual, which sums whole rows): also chunks of 7, one pass
// over the rows of a 7-point stencil, for narrow vectors in that format.
template <bool WHOLE = false, class F> static hipError_t with_kr(int code, F&& f) {
  switch (code) {
    case 18: return f(std::integral_constant<int, 1>{}, std::integral_constant<int, 8>{});
    case 24: return f(std::integral_constant<int, 2>{}, std::integral_constant<int, 4>{});
    case 44: return f(std::integral_constant<int, 4>{}, std::integral_constant<int, 4>{});
    case 23: return f(std::integral_constant<int, 2>{}, std::integral_constant<int, 3>{});
    case 43: return f(std::integral_constant<int, 4>{}, std::integral_constant<int, 3>{});
    case 47:
      if constexpr (WHOLE) return f(std::integral_constant<int, 4>{}, std::integral_constant<int, 7>{});
      break;
  }
  return hipErrorInvalidValue;
}
template <int U, class TT, class TI> constexpr bool shape_ok() {
  if (U == 7) return sizeof(TT) == 2 && std::is_same<TI, SOff>::value;
  return U != 3 || sizeof(TT) == 2 || std::is_same<TI, SOff>::value;
}

static inline dim3 grid_for(int64_t n) { return dim3((unsigned)physical_grid(n_blocks(n))); }

// Storage combinations the library instantiates: a level with vectors in
// TY uses a matrix TA and preconditioned directions TX no wider than TY.
template <class TA, class TX, class TY> constexpr bool ok_level() {
  if (is_dbl<TY>::value) return is_dbl<TA>::value && is_dbl<TX>::value;
  if (std::is_same<TY, float>::value) return !is_dbl<TA>::value && !is_dbl<TX>::value;
  return std::is_same<TA, TY>::value && std::is_same<TX, TY>::value;
}

// ---------------------------------------------------------------------------
// level SpMV + CGS dots
// ---------------------------------------------------------------------------
constexpr int kDotChunk = 64;

template <class TI, class TA, class TX, class TY, class Q, class ALT>
__global__ __launch_bounds__(kBlock) void k_spmv_dots(SellDesc A, const TA* __restrict__ av,
                                                      const TX* __restrict__ x, ALT alt,
                                                      const int* fb, TY* __restrict__ y,
                                                      const TY* __restrict__ v0,
                                                      const TY* __restrict__ vb, int nv,
                                                      Q* __restrict__ part, int64_t nb,
                                                      const int* stop) {
  __shared__ Q lds[kBlock / kWave][kDotChunk];
  const int64_t lb = logical_block(nb);
  if (lb >= nb) return;
  const int sy = sys_of(A.sys, lb * kRowsPerBlock);
  stop = sys_ptr(stop, sy, A.sys.dI);
  if (A.sys.blk && stop && *stop) return;  // several systems: finished ones skip their rows
  // One system: the flags are read while the entry loads are in flight; a
  // stopped level's blocks then write nothing.
  const int stopped = read_flag(stop);
  fb = sys_ptr(fb, sy, A.sys.dI);
  const int fbv = read_flag(fb);
  alt.at_sys(sy, A.sys);
  const int wave = wave_index(), lane = threadIdx.x & (kWave - 1);
  RowSlot s[kR];
  make_slots(A, lb * 4 + wave, lane, s);
  int kb[kR], ke[kR], kc[kR];
  Q acc[kR];
#pragma unroll
  for (int r = 0; r < kR; r++) {
    kb[r] = 0;
    ke[r] = s[r].w;
    kc[r] = max(s[r].w, 1);
    acc[r] = 0;
  }
  const TI* idx = (const TI*)A.idx;
  rows_sum<kUnroll, TI>(av, idx, s, kb, kc, kb, ke, acc, LdVec<TX, Q>{x});
  if (fbv) {
    // rare: the input was non-finite and is replaced by the level's input
    // basis; the sums are formed again from it (the flag is read only here,
    // so the common pass never waits for it)
#pragma unroll
    for (int r = 0; r < kR; r++) acc[r] = 0;
    alt.init();
    rows_sum<kUnroll, TI>(av, idx, s, kb, kc, kb, ke, acc, alt);
  }
  Q yv[kR];
#pragma unroll
  for (int r = 0; r < kR; r++) {
    const TY yr = round_to<TY>(acc[r]);
    if (s[r].ok && !stopped) y[s[r].row] = yr;
    yv[r] = s[r].ok ? widen<Q>(yr) : Q(0);
  }
  for (int c0 = 0; c0 < nv; c0 += kDotChunk) {
    const int cn = nv - c0 < kDotChunk ? nv - c0 : kDotChunk;
    for (int l0 = 0; l0 < cn; l0 += 4) {
      Q vv[4][kR];
#pragma unroll
      for (int u = 0; u < 4; u++) {
        const int ll = c0 + min(l0 + u, cn - 1);
        const TY* V = ll == 0 ? v0 : vb + (int64_t)(ll - 1) * A.n;
#pragma unroll
        for (int r = 0; r < kR; r++) vv[u][r] = widen<Q>(V[s[r].row]);
      }
#pragma unroll
      for (int u = 0; u < 4; u++) {
        if (l0 + u < cn) {
          Q p = 0;
#pragma unroll
          for (int r = 0; r < kR; r++) p = p + yv[r] * vv[u][r];
          p = wave_sum(p);
          if (lane == 0) lds[wave][l0 + u] = p;
        }
      }
    }
    __syncthreads();
    if ((int)threadIdx.x < cn && !stopped) {
      const int t = threadIdx.x;
      Q sum = lds[0][t];
      sum = sum + lds[1][t];
      sum = sum + lds[2][t];
      sum = sum + lds[3][t];
      part[(int64_t)(c0 + t) * nb + lb] = sum;
    }
    __syncthreads();
  }
}

hipError_t spmv_dots(hipStream_t st, const SellDesc& A, const void* av, int ta, const void* x,
                     int tx, const Basis* alt, const int* fb, void* y, int ty, const void* v0,
                     const void* vb, int nv, void* partials, const int* stop) {
  const int64_t nb = n_blocks(A.n);
  return with_idx(A.idx16, [&](auto pi) {
    using TI = TYPE_OF(pi);
    return with_type(ta, [&](auto pa) {
      using TA = TYPE_OF(pa);
      return with_type(tx, [&](auto px) {
        using TX = TYPE_OF(px);
        return with_type(ty, [&](auto py) -> hipError_t {
          using TY = TYPE_OF(py);
          if constexpr (!ok_level<TA, TX, TY>()) {
            return hipErrorInvalidValue;
          } else {
            using Q = wider_t<TA, TY>;
            LdBasis<TY, TY, Q> ld{};
            if (alt) {
              ld.p = (const TY*)alt->raw;
              ld.scp = alt->scale;
              ld.cur = nullptr;
              ld.stride = 0;
            }
            hipLaunchKernelGGL((k_spmv_dots<TI, TA, TX, TY, Q, LdBasis<TY, TY, Q>>), grid_for(A.n),
                               dim3(kBlock), 0, st, A, (const TA*)av, (const TX*)x, ld,
                               alt ? fb : nullptr, (TY*)y, (const TY*)v0, (const TY*)vb, nv,
                               (Q*)partials, nb, stop);
            return hipGetLastError();
          }
        });
      });
    });
  });
}

// ---------------------------------------------------------------------------
// one-block finalisation of per-block partial sums
// ---------------------------------------------------------------------------
template <class Q>
__global__ __launch_bounds__(kFinBlock) void k_finalize(const Q* __restrict__ part, int64_t nb,
                                                        const double* scales, double* dst,
                                                        const int* stop, SysLayout sl) {
  __shared__ Q lds[kFinBlock / kWave];
  const int l = blockIdx.x, sy = blockIdx.y;
  int64_t lo, hi;
  sys_range(sl, sy, nb, lo, hi);
  scales = sys_ptr(scales, sy, sl.dS);
  dst = sys_ptr(dst, sy, sl.dS);
  stop = sys_ptr(stop, sy, sl.dI);
  // partial loads first; the stop flag is read while they are in flight
  Q s = thread_sum(part + (int64_t)l * nb + lo, hi - lo);
  s = fin_block_sum(s, lds);
  if (threadIdx.x == 0 && !(stop && *stop)) {
    if (scales) s = s * (Q)scales[l];
    dst[l] = (double)s;
  }
}

hipError_t finalize_sums(hipStream_t st, const SysLayout& sl, int q, const void* partials, int64_t nb,
                         int count, const double* scales, double* dst, const int* stop) {
  if (count <= 0) return hipSuccess;
  const dim3 g((unsigned)count, (unsigned)sl.nsys);
  if (q == T64)
    hipLaunchKernelGGL(k_finalize<double>, g, dim3(kFinBlock), 0, st, (const double*)partials, nb,
                       scales, dst, stop, sl);
  else
    hipLaunchKernelGGL(k_finalize<float>, g, dim3(kFinBlock), 0, st, (const float*)partials, nb,
                       scales, dst, stop, sl);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// CGS update w <- w - V h and its squared norm
// ---------------------------------------------------------------------------
constexpr int kMaxM = 1024;

template <class TY, class Q>
__global__ __launch_bounds__(kBlock) void k_axpy_norm(SysLayout sl, int64_t n, TY* __restrict__ w,
                                                      const TY* __restrict__ v0,
                                                      const TY* __restrict__ vb, int nv,
                                                      const double* __restrict__ h,
                                                      const double* __restrict__ scales,
                                                      Q* __restrict__ part, int64_t nb,
                                                      const int* stop) {
  __shared__ Q lds[kBlock / kWave];
  const int64_t lb = logical_block(nb);
  if (lb >= nb) return;
  const int sy = sys_of(sl, lb * kRowsPerBlock);
  stop = sys_ptr(stop, sy, sl.dI);
  if (sl.blk && stop && *stop) return;
  const int stopped = read_flag(stop);  // checked at the stores (one system)
  h = sys_ptr(h, sy, sl.dS);
  scales = sys_ptr(scales, sy, sl.dS);
  int64_t row[kR];
  bool ok[kR];
  Q acc[kR];
#pragma unroll
  for (int r = 0; r < kR; r++) {
    const int64_t rr = lb * kRowsPerBlock + (int64_t)r * kBlock + threadIdx.x;
    ok[r] = rr < n;
    row[r] = ok[r] ? rr : n - 1;
    acc[r] = widen<Q>(w[row[r]]);
  }
  for (int l0 = 0; l0 < nv; l0 += 4) {
    Q vv[4][kR];
#pragma unroll
    for (int u = 0; u < 4; u++) {
      const int l = min(l0 + u, nv - 1);
      const TY* V = l == 0 ? v0 : vb + (int64_t)(l - 1) * n;
#pragma unroll
      for (int r = 0; r < kR; r++) vv[u][r] = widen<Q>(V[row[r]]);
    }
#pragma unroll
    for (int u = 0; u < 4; u++) {
      const int l = min(l0 + u, nv - 1);
      const Q hl = (Q)h[l], sl = (Q)scales[l];
#pragma unroll
      for (int r = 0; r < kR; r++) {
        const Q v = widen<Q>(round_to<TY>(vv[u][r] * sl));
        const Q t = acc[r] - hl * v;
        acc[r] = (l0 + u < nv) ? t : acc[r];
      }
    }
  }
  Q sq = 0;
#pragma unroll
  for (int r = 0; r < kR; r++) {
    const TY wr = round_to<TY>(acc[r]);
    if (ok[r] && !stopped) w[row[r]] = wr;
    const Q q = ok[r] ? widen<Q>(wr) : Q(0);
    sq = sq + q * q;
  }
  const Q tot = block_sum(sq, lds);
  if (threadIdx.x == 0 && !stopped) part[lb] = tot;
}

hipError_t axpy_norm(hipStream_t st, const SysLayout& sl, int64_t n, void* w, int tw, const void* v0,
                     const void* vb, int nv, const double* h, const double* scales, void* partials,
                     const int* stop) {
  if (nv > kMaxM) return hipErrorInvalidValue;
  const int64_t nb = n_blocks(n);
  return with_type(tw, [&](auto pw) {
    using TY = TYPE_OF(pw);
    using Q = wider_t<TY, TY>;
    hipLaunchKernelGGL((k_axpy_norm<TY, Q>), grid_for(n), dim3(kBlock), 0, st, sl, n, (TY*)w,
                       (const TY*)v0, (const TY*)vb, nv, h, scales, (Q*)partials, nb, stop);
    return hipGetLastError();
  });
}

// The same update with the finalisation of the Gram-Schmidt dots folded in
// (one system, at most kFuseMaxDots dots): every block first sums the
// per-block dot partials of the level SpMV in the order of k_finalize
// (thread t of kFinBlock adds entries t, t + kFinBlock, ... in index order,
// then the waves in a fixed order), so h_l = round_q(sum * scale_l) is the
// value the separate finalisation gives, bit for bit; logical block 0 stores
// the column of H.  A block then covers kFuseRows rows (kFuseRowsPerThread
// per thread), so the squared norm leaves few partials for the Givens step.
constexpr int kFuseMaxDots = 16;
constexpr int kFuseRowsPerThread = 8;
constexpr int kFuseRows = kFinBlock * kFuseRowsPerThread;

template <class TY, class Q>
__global__ __launch_bounds__(kFinBlock) void k_axpy_norm_fin(
    int64_t n, TY* __restrict__ w, const TY* __restrict__ v0, const TY* __restrict__ vb, int nv,
    const Q* __restrict__ dpart, int64_t dnb, const double* __restrict__ scales, double* hcol,
    Q* __restrict__ npart, int64_t nnb, const int* stop) {
  __shared__ Q lds[kFinBlock / kWave][kFuseMaxDots];
  __shared__ Q hs[kFuseMaxDots];
  const int64_t lb = logical_block(nnb);
  if (lb >= nnb) return;
  const int stopped = read_flag(stop);  // checked at the stores
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  int64_t row[kFuseRowsPerThread];
  bool ok[kFuseRowsPerThread];
  Q acc[kFuseRowsPerThread];
#pragma unroll
  for (int r = 0; r < kFuseRowsPerThread; r++) {
    const int64_t rr = lb * kFuseRows + (int64_t)r * kFinBlock + threadIdx.x;
    ok[r] = rr < n;
    row[r] = ok[r] ? rr : n - 1;
    acc[r] = widen<Q>(w[row[r]]);
  }
  // the first four basis vectors are loaded before the dot reduction, so
  // their loads overlap its loads and barriers
  Q vv[4][kFuseRowsPerThread];
#pragma unroll
  for (int u = 0; u < 4; u++) {
    const int l = min(u, nv - 1);
    const TY* V = l == 0 ? v0 : vb + (int64_t)(l - 1) * n;
#pragma unroll
    for (int r = 0; r < kFuseRowsPerThread; r++) vv[u][r] = widen<Q>(V[row[r]]);
  }
  // the dots: per-thread sums in index order (four dots' loads in flight
  // together), wave sums, waves in order
  for (int l0 = 0; l0 < nv; l0 += 4) {
    Q s4[4];
    thread_sums4(dpart, dnb, l0, nv, dnb, s4);
#pragma unroll
    for (int u = 0; u < 4; u++) {
      if (l0 + u < nv) {
        const Q sl = wave_sum(s4[u]);
        if (lane == 0) lds[wv][l0 + u] = sl;
      }
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < nv) {
    const int l = threadIdx.x;
    Q sl = 0;
#pragma unroll
    for (int i = 0; i < kFinBlock / kWave; i++) sl = sl + lds[i][l];
    sl = sl * (Q)scales[l];
    hs[l] = sl;
    if (lb == 0 && !stopped) hcol[l] = (double)sl;
  }
  __syncthreads();
  for (int l0 = 0; l0 < nv; l0 += 4) {
    if (l0 > 0) {
#pragma unroll
      for (int u = 0; u < 4; u++) {
        const int l = min(l0 + u, nv - 1);
        const TY* V = l == 0 ? v0 : vb + (int64_t)(l - 1) * n;
#pragma unroll
        for (int r = 0; r < kFuseRowsPerThread; r++) vv[u][r] = widen<Q>(V[row[r]]);
      }
    }
#pragma unroll
    for (int u = 0; u < 4; u++) {
      const int l = min(l0 + u, nv - 1);
      const Q hl = hs[l], sc = (Q)scales[l];
#pragma unroll
      for (int r = 0; r < kFuseRowsPerThread; r++) {
        const Q v = widen<Q>(round_to<TY>(vv[u][r] * sc));
        const Q t = acc[r] - hl * v;
        acc[r] = (l0 + u < nv) ? t : acc[r];
      }
    }
  }
  Q sq = 0;
#pragma unroll
  for (int r = 0; r < kFuseRowsPerThread; r++) {
    const TY wr = round_to<TY>(acc[r]);
    if (ok[r] && !stopped) w[row[r]] = wr;
    const Q q = ok[r] ? widen<Q>(wr) : Q(0);
    sq = sq + q * q;
  }
  __shared__ Q red[kFinBlock / kWave];
  const Q tot = fin_block_sum(sq, red);
  if (threadIdx.x == 0 && !stopped) npart[lb] = tot;
}

hipError_t axpy_norm_fin(hipStream_t st, int64_t n, void* w, int tw, const void* v0, const void* vb,
                         int nv, const void* dot_partials, int64_t dnb, const double* scales,
                         double* hcol, void* norm_partials, int64_t* nnb, const int* stop) {
  if (nv < 1 || nv > kFuseMaxDots) return hipErrorInvalidValue;
  const int64_t nb = (n + kFuseRows - 1) / kFuseRows;
  *nnb = nb;
  return with_type(tw, [&](auto pw) {
    using TY = TYPE_OF(pw);
    using Q = wider_t<TY, TY>;
    hipLaunchKernelGGL((k_axpy_norm_fin<TY, Q>), dim3((unsigned)physical_grid(nb)), dim3(kFinBlock), 0,
                       st, n, (TY*)w, (const TY*)v0, (const TY*)vb, nv, (const Q*)dot_partials, dnb,
                       scales, hcol, (Q*)norm_partials, nb, stop);
    return hipGetLastError();
  });
}

// ---------------------------------------------------------------------------
// Givens rotations, breakdown handling and the small triangular solve
// ---------------------------------------------------------------------------
template <class Q> __device__ void back_substitute(double* S, const int* I, const LevelLayout& L) {
  // R y = g, rows from the last, each sum taken left to right
  const int meff = I[I_MEFF];
  const int ld = L.m + 1;
  const double* H = S + L.H;
  const double* g = S + L.g;
  double* y = S + L.y;
  for (int i = meff - 1; i >= 0; i--) {
    Q acc = (Q)g[i];
    for (int k = i + 1; k < meff; k++) acc = acc - (Q)H[i + (int64_t)k * ld] * (Q)y[k];
    y[i] = (double)(acc / (Q)H[i + (int64_t)i * ld]);
  }
}

// the child state of system sy
__device__ __forceinline__ ChildInit child_of(ChildInit c, const SysLayout& sl, int sy) {
  c.S = sys_ptr(c.S, sy, sl.dS);
  c.I = sys_ptr(c.I, sy, sl.dI);
  return c;
}

__device__ void init_child(const ChildInit& c, double scale0, double beta, int stop) {
  c.S[c.scale] = scale0;
  c.S[c.g] = beta;
  if (c.beta >= 0) c.S[c.beta] = beta;
  for (int i = 1; i <= c.m; i++) c.S[c.g + i] = 0.0;
  c.I[I_MEFF] = 0;
  c.I[I_STOP] = stop;
  c.I[I_BAD] = 0;
  for (int i = 0; i < c.m; i++) c.I[I_FB + i] = 0;
}

// The Givens step with the level state it reads staged in LDS: the threads
// load the column of H, the rotations, g, the flags and (for the last step)
// the leading columns of H together, while the norm partials are summed;
// thread 0 then runs the step on the staged copies, so its serial work waits
// on no global load.  The step: h_{j+1,j} = sqrt(sum of the norm partials);
// the previous rotations applied to column j; the new rotation, g, the
// residual estimate and the history; breakdown and stop handling; the next
// scale; the state of an aliased child; R y = g on the last step or a stop.
constexpr int kGivStage = 2048;  // doubles of H staged for the back substitution

template <class Q>
__global__ __launch_bounds__(kFinBlock) void k_givens(const Q* __restrict__ part, int64_t nb,
                                                      double* S, int* I, LevelLayout L, int j,
                                                      int solve_y, const double* inv_bnorm,
                                                      double* host_out, ChildInit child,
                                                      SysLayout sl, double tol, HistOut hist) {
  __shared__ Q lds[kFinBlock / kWave];
  __shared__ double hc[kMaxM + 1], csl[kMaxM], snl[kMaxM], gl[kMaxM + 1], yl[kMaxM];
  __shared__ double hm[kGivStage];
  __shared__ double sc[4];
  __shared__ int fl[4];
  const int sy = blockIdx.x;
  int64_t lo, hi;
  sys_range(sl, sy, nb, lo, hi);
  S = sys_ptr(S, sy, sl.dS);
  I = sys_ptr(I, sy, sl.dI);
  const int ld = L.m + 1;
  const int t = threadIdx.x;
  if (t <= j) {
    hc[t] = S[L.H + t + (int64_t)j * ld];
    gl[t] = S[L.g + t];
  }
  if (t < j) {
    csl[t] = S[L.cs + t];
    snl[t] = S[L.sn + t];
  }
  const int nstage = solve_y && (j + 1) * ld <= kGivStage ? (j + 1) * ld : 0;
  for (int e = t; e < nstage; e += kFinBlock) hm[e] = S[L.H + e];
  if (t == kFinBlock - 1) {
    sc[0] = S[L.g + j + 1];
    sc[1] = S[L.beta];
    sc[2] = S[L.scale + j + 1];
    sc[3] = S[L.cbeta];
  }
  if (t == kFinBlock - 2) {
    fl[0] = I[I_STOP];
    fl[1] = I[I_FB + j];
    fl[2] = I[I_HLEN];
    fl[3] = I[I_BAD];
  }
  Q s = thread_sum(part + lo, hi - lo);
  s = fin_block_sum(s, lds);  // its barriers also publish the staged values
  if (t != 0 || fl[0]) return;
  const double inv_bn = inv_bnorm ? inv_bnorm[sy] : 0.0;
  const HistOut hs = sy == 0 ? hist : HistOut{};
  if (child.S) child = child_of(child, sl, sy);
  host_out = host_out ? host_out + 4 * sy : nullptr;
  double* H = S + L.H;
  double* Hraw = S + L.Hraw;
  const Q hn = sqrt(s);
  for (int i = 0; i <= j; i++) Hraw[i + (int64_t)j * ld] = hc[i];
  Hraw[j + 1 + (int64_t)j * ld] = (double)hn;
  for (int i = 0; i < j; i++) {
    const Q a0 = (Q)hc[i], a1 = (Q)hc[i + 1];
    const Q c = (Q)csl[i], sv = (Q)snl[i];
    hc[i] = (double)(c * a0 + sv * a1);
    hc[i + 1] = (double)(-sv * a0 + c * a1);
  }
  if (fl[1]) atomicAdd(I + I_FALLBACKS, 1);
  const Q hjj = (Q)hc[j];
  const Q rho = (Q)hypot((double)hjj, (double)hn);
  int stop = 0, bad = fl[3], meff;
  double gnext = sc[0], scale_next = sc[2], cbeta = sc[3];
  const bool fail = !(rho != (Q)0) || !isfinite((double)rho) || !isfinite((double)hn);
  if (fail) {
    meff = j;
    atomicAdd(I + I_BREAKDOWNS, 1);
    if (!isfinite((double)rho) || !isfinite((double)hn)) bad = 1;
    stop = 1;
  } else {
    const Q c = hjj / rho, sv = hn / rho;
    S[L.cs + j] = (double)c;
    S[L.sn + j] = (double)sv;
    hc[j] = (double)rho;
    const Q gj = (Q)gl[j];
    gnext = (double)(-sv * gj);
    gl[j] = (double)(c * gj);
    S[L.g + j + 1] = gnext;
    S[L.g + j] = gl[j];
    meff = j + 1;
    if (hs.p && fl[2] < hs.cap) {
      hs.p[fl[2]] = fabs(gnext) / sc[1];
      I[I_HLEN] = fl[2] + 1;
    }
    if (hn == (Q)0) {
      atomicAdd(I + I_BREAKDOWNS, 1);
      stop = 1;
    } else {
      const Q inv = (Q)1 / hn;
      scale_next = (double)inv;
      cbeta = (double)(hn * inv);
      S[L.scale + j + 1] = scale_next;
      S[L.cbeta] = cbeta;
    }
  }
  for (int i = 0; i <= j; i++) H[i + (int64_t)j * ld] = hc[i];
  if (!fail) H[j + 1 + (int64_t)j * ld] = 0.0;
  I[I_MEFF] = meff;
  I[I_BAD] = bad;
  if (host_out) {
    const double est = fabs(gnext) * inv_bn;
    // outermost level: a system that reached the tolerance stops its rows
    if (tol > 0.0 && est < tol) stop = 1;
    host_out[0] = est;
    host_out[1] = (double)(stop | (bad << 1));
  }
  I[I_STOP] = stop;
  I[I_CUR] = j + 1;
  if (child.S) init_child(child, scale_next, cbeta, stop);
  if (!(solve_y || stop)) return;
  if (nstage) {
    // R y = g from the staged columns (column j as just rotated), rows from
    // the last, each sum taken left to right, as back_substitute does
    for (int i = 0; i <= j; i++) hm[i + j * ld] = hc[i];
    for (int i = meff - 1; i >= 0; i--) {
      Q acc = (Q)gl[i];
      for (int k = i + 1; k < meff; k++) acc = acc - (Q)hm[i + k * ld] * (Q)yl[k];
      yl[i] = (double)(acc / (Q)hm[i + i * ld]);
    }
    for (int i = 0; i < meff; i++) S[L.y + i] = yl[i];
  } else {
    back_substitute<Q>(S, I, L);
  }
}

hipError_t givens(hipStream_t st, const SysLayout& sl, int q, const void* partials, int64_t nb,
                  double* S, int* I, const LevelLayout& L, int j, int solve_y,
                  const double* inv_bnorm, double* host_out, const ChildInit* child, double tol,
                  HistOut hist) {
  ChildInit c = child ? *child : ChildInit{};
  const dim3 g((unsigned)sl.nsys);
  if (q == T64)
    hipLaunchKernelGGL(k_givens<double>, g, dim3(kFinBlock), 0, st, (const double*)partials, nb, S,
                       I, L, j, solve_y, inv_bnorm, host_out, c, sl, tol, hist);
  else
    hipLaunchKernelGGL(k_givens<float>, g, dim3(kFinBlock), 0, st, (const float*)partials, nb, S, I,
                       L, j, solve_y, inv_bnorm, host_out, c, sl, tol, hist);
  return hipGetLastError();
}

template <class Q> __global__ void k_backsolve(double* S, int* I, LevelLayout L, SysLayout sl) {
  const int sy = blockIdx.x;
  if (threadIdx.x == 0) back_substitute<Q>(sys_ptr(S, sy, sl.dS), sys_ptr(I, sy, sl.dI), L);
}

hipError_t backsolve(hipStream_t st, const SysLayout& sl, int q, double* S, int* I,
                     const LevelLayout& L) {
  const dim3 g((unsigned)sl.nsys);
  if (q == T64)
    hipLaunchKernelGGL(k_backsolve<double>, g, dim3(64), 0, st, S, I, L, sl);
  else
    hipLaunchKernelGGL(k_backsolve<float>, g, dim3(64), 0, st, S, I, L, sl);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// level output: sum_j y_j z_j
// ---------------------------------------------------------------------------
// A level with at most kCombineAll directions loads every column Z_j
// without waiting for meff (columns past meff are masked; they lie inside
// Z); a longer one (the outermost level) loops to meff.
constexpr int kCombineAll = 8;

template <class TZ, class TV, class Q>
__global__ __launch_bounds__(kBlock) void k_combine(SysLayout sl, int64_t n, const TZ* __restrict__ Z,
                                                    const double* y, const int* meffp, int m,
                                                    void* out, const double* s, const int* cur,
                                                    int accumulate, LdLevelBasis<TV, Q> alt,
                                                    const int* fb, int* out_fb, const int* pstop,
                                                    int64_t nb) {
  const int64_t lb = logical_block(nb);
  if (lb >= nb) return;
  const int sy = sys_of(sl, lb * kRowsPerBlock);
  pstop = sys_ptr(pstop, sy, sl.dI);
  if (sl.blk && pstop && *pstop) return;
  const int stopped = read_flag(pstop);  // checked at the stores (one system)
  y = sys_ptr(y, sy, sl.dS);
  meffp = sys_ptr(meffp, sy, sl.dI);
  cur = sys_ptr(cur, sy, sl.dI);
  fb = sys_ptr(fb, sy, sl.dI);
  out_fb = sys_ptr(out_fb, sy, sl.dI);
  alt.scales = sys_ptr(alt.scales, sy, sl.dS);
  // (a stopped system's meff may be stale: kept inside [0, m])
  const int meff = min(max(*meffp, 0), m);
  const int jend = m <= kCombineAll ? m : meff;
  // the thread's rows, clamped into the vector (a row past n is not stored)
  const int64_t row0 = lb * kRowsPerBlock + threadIdx.x;
  int64_t rowc[kR];
#pragma unroll
  for (int r = 0; r < kR; r++) rowc[r] = min(row0 + (int64_t)r * kBlock, n - 1);
  // u_i = sum over j < meff of y_j Z_j,i, j ascending
  Q acc[kR];
#pragma unroll
  for (int r = 0; r < kR; r++) acc[r] = 0;
  for (int j0 = 0; j0 < jend; j0 += 4) {
    Q zz[4][kR];
#pragma unroll
    for (int u = 0; u < 4; u++) {
      const TZ* zj = Z + (int64_t)min(j0 + u, jend - 1) * n;
#pragma unroll
      for (int r = 0; r < kR; r++) zz[u][r] = widen<Q>(zj[rowc[r]]);
    }
#pragma unroll
    for (int u = 0; u < 4; u++) {
      const int j = j0 + u;
      const Q yj = (Q)y[min(j, m - 1)];
#pragma unroll
      for (int r = 0; r < kR; r++) {
        const Q t = acc[r] + yj * zz[u][r];
        acc[r] = j < meff ? t : acc[r];
      }
    }
  }
  int anyfb = 0;
  if (fb)
    for (int j = 0; j < meff; j++) anyfb |= fb[j];
  if (anyfb) {
    // rare: flagged columns use the basis vector V_j instead of Z_j
#pragma unroll
    for (int r = 0; r < kR; r++) acc[r] = 0;
    for (int j = 0; j < meff; j++) {
      const Q yj = (Q)y[j];
      const int f = fb[j];
#pragma unroll
      for (int r = 0; r < kR; r++) {
        const Q zv = f ? alt.get(j, rowc[r]) : widen<Q>(Z[(int64_t)j * n + rowc[r]]);
        acc[r] = acc[r] + yj * zv;
      }
    }
  }
  if (stopped) return;
  const int ci = cur ? *cur : 0;
  const int64_t o = (int64_t)ci * n;
#pragma unroll
  for (int r = 0; r < kR; r++) {
    const int64_t row = row0 + (int64_t)r * kBlock;
    if (row >= n) continue;
    bool fin;
    if (s) {
      // consumer on the unscaled outermost system: z = s_i u_i in fp64
      const double v = s[row] * widen<double>(round_to<TV>(acc[r]));
      double* od = (double*)out + o;
      const double rv = accumulate ? od[row] + v : v;
      od[row] = rv;
      fin = isfinite(rv);
    } else {
      TV* ov = (TV*)out + o;
      const TV rv = accumulate ? round_to<TV>(widen<Q>(ov[row]) + acc[r]) : round_to<TV>(acc[r]);
      ov[row] = rv;
      fin = finite_val(rv);
    }
    if (out_fb && !fin) atomicOr(out_fb + ci, 1);
  }
}

hipError_t combine(hipStream_t st, const SysLayout& sl, int64_t n, const void* Z, int tz, int tv,
                   const double* y, const int* meff, int m, void* out, const double* s,
                   const int* cur, int accumulate, const LevelBasis* alt, const int* fb,
                   int* out_fb, const int* pstop) {
  if (m < 1) return hipErrorInvalidValue;
  const int64_t nb = n_blocks(n);
  return with_type(tz, [&](auto pz) {
    using TZ = TYPE_OF(pz);
    return with_type(tv, [&](auto pv) -> hipError_t {
      using TV = TYPE_OF(pv);
      using Q = wider_t<TZ, TV>;
      LdLevelBasis<TV, Q> ld{};
      if (alt) {
        if (alt->type != tv) return hipErrorInvalidValue;
        ld.v0 = (const TV*)alt->v0;
        ld.vb = (const TV*)alt->vb;
        ld.scales = alt->scales;
        ld.n = n;
      }
      hipLaunchKernelGGL((k_combine<TZ, TV, Q>), grid_for(n), dim3(kBlock), 0, st, sl, n,
                         (const TZ*)Z, y, meff, m, out, s, cur, accumulate, ld, alt ? fb : nullptr,
                         out_fb, pstop, nb);
      return hipGetLastError();
    });
  });
}

// ---------------------------------------------------------------------------
// level entry (cast + norm) and outermost residual
// ---------------------------------------------------------------------------
template <class LD, class TO, class Q>
__global__ __launch_bounds__(kBlock) void k_entry(SysLayout sl, int64_t n, LD ld, TO* __restrict__ out,
                                                  Q* __restrict__ part, int64_t nb,
                                                  const int* pstop) {
  __shared__ Q lds[kBlock / kWave];
  const int64_t lb = logical_block(nb);
  if (lb >= nb) return;
  const int sy = sys_of(sl, lb * kRowsPerBlock);
  pstop = sys_ptr(pstop, sy, sl.dI);
  if (pstop && *pstop) return;
  ld.at_sys(sy, sl);
  ld.init();
  Q sq = 0;
#pragma unroll
  for (int r = 0; r < kR; r++) {
    const int64_t row = lb * kRowsPerBlock + (int64_t)r * kBlock + threadIdx.x;
    if (row < n) {
      const TO o = round_to<TO>(ld(row));
      out[row] = o;
      const Q v = widen<Q>(o);
      sq = sq + v * v;
    }
  }
  const Q s = block_sum(sq, lds);
  if (threadIdx.x == 0) part[lb] = s;
}

hipError_t entry_cast(hipStream_t st, const SysLayout& sl, int64_t n, const Basis& in, void* out,
                      int to, void* partials, const int* parent_stop) {
  const int64_t nb = n_blocks(n);
  return with_type(to, [&](auto po) -> hipError_t {
    using TO = TYPE_OF(po);
    using Q = wider_t<TO, TO>;
    if (in.s) {
      if (in.type != T64) return hipErrorInvalidValue;
      LdSBasis<TO, double> ld{(const double*)in.raw, in.scale, in.s, in.cur, in.stride, 0.0};
      hipLaunchKernelGGL((k_entry<LdSBasis<TO, double>, TO, Q>), grid_for(n), dim3(kBlock), 0, st,
                         sl, n, ld, (TO*)out, (Q*)partials, nb, parent_stop);
      return hipGetLastError();
    }
    return with_type(in.type, [&](auto pi) -> hipError_t {
      using TIN = TYPE_OF(pi);
      using QQ = wider_t<TIN, TO>;
      if (!in.scale) {
        // a stored vector (the right-hand side a Richardson level hands to
        // an FGMRES level below it)
        if (in.cur) return hipErrorInvalidValue;
        LdVec<TIN, QQ> ld{(const TIN*)in.raw};
        hipLaunchKernelGGL((k_entry<LdVec<TIN, QQ>, TO, Q>), grid_for(n), dim3(kBlock), 0, st, sl, n,
                           ld, (TO*)out, (Q*)partials, nb, parent_stop);
        return hipGetLastError();
      }
      LdBasis<TIN, TO, QQ> ld{(const TIN*)in.raw, in.scale, in.cur, in.stride, 0.0};
      hipLaunchKernelGGL((k_entry<LdBasis<TIN, TO, QQ>, TO, Q>), grid_for(n), dim3(kBlock), 0, st,
                         sl, n, ld, (TO*)out, (Q*)partials, nb, parent_stop);
      return hipGetLastError();
    });
  });
}

template <class Q>
__global__ __launch_bounds__(kFinBlock) void k_entry_fin(const Q* __restrict__ part, int64_t nb,
                                                         ChildInit c, ChildInit child,
                                                         const int* pstop, SysLayout sl) {
  __shared__ Q lds[kFinBlock / kWave];
  const int sy = blockIdx.x;
  int64_t lo, hi;
  sys_range(sl, sy, nb, lo, hi);
  c = child_of(c, sl, sy);
  if (child.S) child = child_of(child, sl, sy);
  pstop = sys_ptr(pstop, sy, sl.dI);
  if (pstop && *pstop) {
    if (threadIdx.x == 0) {
      init_child(c, 0.0, 0.0, 1);
      if (child.S) init_child(child, 0.0, 0.0, 1);
    }
    return;
  }
  Q s = thread_sum(part + lo, hi - lo);
  s = fin_block_sum(s, lds);
  if (threadIdx.x == 0) {
    const Q beta = sqrt(s);
    const Q inv = beta > (Q)0 ? (Q)1 / beta : (Q)0;
    const int stop = beta > (Q)0 && isfinite((double)beta) ? 0 : 1;
    init_child(c, (double)inv, (double)beta, stop);
    // an aliased child starts from V_0 of this level: norm beta * (1 / beta)
    if (child.S) init_child(child, (double)inv, (double)(beta * inv), stop);
  }
}

hipError_t entry_finalize(hipStream_t st, const SysLayout& sl, int q, const void* partials,
                          int64_t nb, const ChildInit& lev, const ChildInit* child,
                          const int* parent_stop) {
  const ChildInit ch = child ? *child : ChildInit{};
  const dim3 g((unsigned)sl.nsys);
  if (q == T64)
    hipLaunchKernelGGL(k_entry_fin<double>, g, dim3(kFinBlock), 0, st, (const double*)partials, nb,
                       lev, ch, parent_stop, sl);
  else
    hipLaunchKernelGGL(k_entry_fin<float>, g, dim3(kFinBlock), 0, st, (const float*)partials, nb, lev,
                       ch, parent_stop, sl);
  return hipGetLastError();
}

__global__ void k_child_init0(double* S, int* I, LevelLayout L, ChildInit child, SysLayout sl) {
  const int sy = blockIdx.x;
  S = sys_ptr(S, sy, sl.dS);
  I = sys_ptr(I, sy, sl.dI);
  if (threadIdx.x == 0) init_child(child_of(child, sl, sy), S[L.scale], S[L.g], I[I_STOP]);
}

hipError_t child_init0(hipStream_t st, const SysLayout& sl, double* S, int* I, const LevelLayout& L,
                       const ChildInit& child) {
  hipLaunchKernelGGL(k_child_init0, dim3((unsigned)sl.nsys), dim3(64), 0, st, S, I, L, child, sl);
  return hipGetLastError();
}

template <class TI>
__global__ __launch_bounds__(kBlock) void k_residual64(SellDesc A, const double* __restrict__ av,
                                                       const double* __restrict__ x,
                                                       const double* __restrict__ b,
                                                       double* __restrict__ r,
                                                       double* __restrict__ part, int64_t nb) {
  __shared__ double lds[kBlock / kWave];
  const int64_t lb = logical_block(nb);
  if (lb >= nb) return;
  const int wave = wave_index(), lane = threadIdx.x & (kWave - 1);
  RowSlot s[kR];
  make_slots(A, lb * 4 + wave, lane, s);
  int kb[kR], ke[kR], kc[kR];
  double acc[kR];
#pragma unroll
  for (int q = 0; q < kR; q++) {
    kb[q] = 0;
    ke[q] = s[q].w;
    kc[q] = max(s[q].w, 1);
    acc[q] = 0.0;
  }
  rows_sum<kUnroll, TI>(av, (const TI*)A.idx, s, kb, kc, kb, ke, acc, LdVec<double, double>{x});
  double sq = 0.0;
#pragma unroll
  for (int q = 0; q < kR; q++) {
    if (s[q].ok) {
      const double rv = b[s[q].row] - acc[q];
      r[s[q].row] = rv;
      sq = sq + rv * rv;
    }
  }
  const double tot = block_sum(sq, lds);
  if (threadIdx.x == 0) part[lb] = tot;
}

hipError_t residual64(hipStream_t st, const SellDesc& A, const double* a64, const double* x,
                      const double* b, double* r, void* partials) {
  const int64_t nb = n_blocks(A.n);
  return with_idx(A.idx16, [&](auto pi) {
    using TI = TYPE_OF(pi);
    hipLaunchKernelGGL((k_residual64<TI>), grid_for(A.n), dim3(kBlock), 0, st, A, a64, x, b, r,
                       (double*)partials, nb);
    return hipGetLastError();
  });
}

__global__ __launch_bounds__(kFinBlock) void k_residual_fin(const double* __restrict__ part, int64_t nb,
                                                            double* S, int* I, LevelLayout L,
                                                            const double* inv_bnorm,
                                                            double* host_out, SysLayout sl) {
  __shared__ double lds[kFinBlock / kWave];
  const int sy = blockIdx.x;
  int64_t lo, hi;
  sys_range(sl, sy, nb, lo, hi);
  double s = thread_sum(part + lo, hi - lo);
  s = fin_block_sum(s, lds);
  S = sys_ptr(S, sy, sl.dS);
  I = sys_ptr(I, sy, sl.dI);
  if (threadIdx.x == 0) {
    const double beta = sqrt(s);
    S[L.scale] = beta > 0 ? 1.0 / beta : 0.0;
    S[L.g] = beta;
    for (int i = 1; i <= L.m; i++) S[L.g + i] = 0.0;
    I[I_MEFF] = 0;
    // a held system (already finished) keeps every kernel of its rows off
    I[I_STOP] = beta > 0 && !I[I_HOLD] ? 0 : 1;
    I[I_CUR] = 0;
    I[I_BAD] = isfinite(beta) ? 0 : 1;
    for (int i = 0; i < L.m; i++) I[I_FB + i] = 0;
    double* ho = host_out + 4 * sy;
    ho[0] = beta * inv_bnorm[sy];
    ho[1] = 0.0;
    ho[2] = beta;
  }
}

hipError_t residual_finalize(hipStream_t st, const SysLayout& sl, const void* partials, int64_t nb,
                             double* S, int* I, const LevelLayout& L, const double* inv_bnorm,
                             double* host_out) {
  hipLaunchKernelGGL(k_residual_fin, dim3((unsigned)sl.nsys), dim3(kFinBlock), 0, st,
                     (const double*)partials, nb, S, I, L, inv_bnorm, host_out, sl);
  return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void k_dot64(int64_t n, const double* __restrict__ x,
                                                  const double* __restrict__ y,
                                                  double* __restrict__ part, int64_t nb) {
  __shared__ double lds[kBlock / kWave];
  const int64_t lb = logical_block(nb);
  if (lb >= nb) return;
  double v = 0.0;
#pragma unroll
  for (int r = 0; r < kR; r++) {
    const int64_t row = lb * kRowsPerBlock + (int64_t)r * kBlock + threadIdx.x;
    if (row < n) v = v + x[row] * y[row];
  }
  const double s = block_sum(v, lds);
  if (threadIdx.x == 0) part[lb] = s;
}

__global__ __launch_bounds__(kFinBlock) void k_sum_to(const double* __restrict__ part, int64_t nb,
                                                      double* out, SysLayout sl) {
  __shared__ double lds[kFinBlock / kWave];
  const int sy = blockIdx.x;
  int64_t lo, hi;
  sys_range(sl, sy, nb, lo, hi);
  double s = thread_sum(part + lo, hi - lo);
  s = fin_block_sum(s, lds);
  if (threadIdx.x == 0) out[4 * sy] = s;
}

hipError_t dot64_to_host(hipStream_t st, const SysLayout& sl, int64_t n, const double* x,
                         const double* y, void* partials, double* host_out) {
  const int64_t nb = n_blocks(n);
  hipLaunchKernelGGL(k_dot64, grid_for(n), dim3(kBlock), 0, st, n, x, y, (double*)partials, nb);
  hipLaunchKernelGGL(k_sum_to, dim3((unsigned)sl.nsys), dim3(kFinBlock), 0, st, (const double*)partials,
                     nb, host_out, sl);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// primary preconditioner: W and G sweeps (Sec. 5.2: two SpMVs)
// ---------------------------------------------------------------------------
template <int KR, int U, class TI, class TM, class TT, class Q, class LD>
__global__ __launch_bounds__(kBlock) void k_mw(SellDesc A, const TM* __restrict__ mv, int neg,
                                               LD ld, TT* __restrict__ t, const int* stop,
                                               int64_t* cntr, int64_t nb) {
  if (cntr && blockIdx.x == 0 && threadIdx.x == 0) *cntr += 1;
  const int64_t lb = logical_block(nb);
  if (lb >= nb) return;
  const int sy = sys_of(A.sys, lb * (kBlock * KR));
  stop = sys_ptr(stop, sy, A.sys.dI);
  if (A.sys.blk && stop && *stop) return;
  const int stopped = read_flag(stop);  // checked at the stores (one system)
  const int wave = wave_index(), lane = threadIdx.x & (kWave - 1);
  const int64_t gw = lb * 4 + wave;
  RowSlot s[KR];
  make_slots(A, gw, lane, s);
  ld.at_sys(sy, A.sys);
  ld.init();
  int lo[KR], hi[KR], kb[KR], ke[KR];
  Q acc[KR];
#pragma unroll
  for (int r = 0; r < KR; r++) {
    lo[r] = 0;
    kb[r] = 0;
    acc[r] = 0;
    if constexpr (std::is_same<TI, SOff>::value) {
      // slice-offset format: every row's diagonal at the common position
      hi[r] = max(A.dell_kd, 1);
      ke[r] = A.dell_kd;
    } else {
      const int64_t slice = gw * KR + r;
      // loop bound from the slice; the row's own diagonal position only
      // masks (diagonal-aligned format: every row's diagonal at dell_kd)
      hi[r] = s[r].ok ? max(A.dell_w ? A.dell_kd : (int)(A.kdr[slice] >> 16), 1) : 1;
      ke[r] = s[r].ok ? (A.dell_w ? A.dell_kd : (int)A.kd[s[r].row]) : 0;
    }
  }
  typename LD::raw_t dg[KR];  // the unit-diagonal term, loaded with the matrix entries
#pragma unroll
  for (int r = 0; r < KR; r++) dg[r] = ld.raw(s[r].row);
  rows_sum<U, TI>(mv, (const TI*)A.idx, s, lo, hi, kb, ke, acc, ld, neg != 0);
#pragma unroll
  for (int r = 0; r < KR; r++)
    if (s[r].ok && !stopped) t[s[r].row] = round_to<TT>(acc[r] + ld.cook(dg[r]));
}

template <int KR, int U, class TI, class TM, class TT, class Q, class EPI>
__global__ __launch_bounds__(kBlock) void k_mg(SellDesc A, const TM* __restrict__ mv, int neg, Q gd,
                                               const TT* __restrict__ t, EPI epi, const int* stop,
                                               int64_t nb) {
  const int64_t lb = logical_block(nb);
  if (lb >= nb) return;
  const int sy = sys_of(A.sys, lb * (kBlock * KR));
  stop = sys_ptr(stop, sy, A.sys.dI);
  if (A.sys.blk && stop && *stop) return;
  const int stopped = read_flag(stop);  // checked at the stores (one system)
  const int wave = wave_index(), lane = threadIdx.x & (kWave - 1);
  const int64_t gw = lb * 4 + wave;
  RowSlot s[KR];
  make_slots(A, gw, lane, s);
  epi.at_sys(sy, A.sys);
  epi.init();
  int lo[KR], hi[KR], kb[KR], ke[KR];
  TT traw[KR];
  Q acc[KR];
#pragma unroll
  for (int r = 0; r < KR; r++) {
    if constexpr (std::is_same<TI, SOff>::value) {
      // slice-offset format: every row's diagonal at the common position
      lo[r] = kb[r] = A.dell_kd + 1;
      hi[r] = ke[r] = A.dell_w;
    } else {
      const int64_t slice = gw * KR + r;
      const int kd = s[r].ok ? (A.dell_w ? A.dell_kd : (int)A.kd[s[r].row]) : 0;
      // loop from just after the slice's smallest diagonal position
      lo[r] = s[r].ok ? (A.dell_w ? A.dell_kd : (int)(A.kdr[slice] & 0xffffu)) + 1 : 0;
      hi[r] = s[r].ok ? s[r].w : 1;
      kb[r] = s[r].ok ? kd + 1 : 0;
      ke[r] = s[r].ok ? s[r].w : 0;
    }
    traw[r] = t[s[r].row];
    epi.prefetch(r, s[r].row);
  }
  // the sums start from gd t_i, formed once the first entry loads are out
  rows_sum<U, TI>(mv, (const TI*)A.idx, s, lo, hi, kb, ke, acc, LdVec<TT, Q>{t}, neg != 0,
                  [&](Q (&a)[KR]) {
#pragma unroll
                    for (int r = 0; r < KR; r++) a[r] = gd * widen<Q>(value_barrier(traw[r]));
                  });
#pragma unroll
  for (int r = 0; r < KR; r++)
    if (s[r].ok && !stopped) epi(r, s[r].row, round_to<TT>(acc[r]));
}


hipError_t m_apply_w(hipStream_t st, const SellDesc& A, const void* mv, int tm, int neg,
                     const Basis& in, void* t, int tt, const int* stop, int64_t* cntr, int kr) {
  if (A.ilu) return ilu_apply_fwd(st, A, mv, tm, in, t, tt, stop, cntr);
  return with_kr(kr, [&](auto KRc, auto Uc) {
  constexpr int KR = decltype(KRc)::value, U = decltype(Uc)::value;
  const int64_t nb = n_blocks_kr(A.n, KR);
  const dim3 grid((unsigned)physical_grid(nb));
  return with_idx(A.idx16, [&](auto pi) {
    using TI = TYPE_OF(pi);
    return with_type(tm, [&](auto pm) {
      using TM = TYPE_OF(pm);
      return with_type(tt, [&](auto pt) -> hipError_t {
        using TT = TYPE_OF(pt);
        if constexpr (!ok_m<TM, TT>() || !shape_ok<U, TT, TI>()) {
          return hipErrorInvalidValue;
        } else {
          using Q = wider_t<TM, TT>;
          if (in.s) {
            if (in.type != T64 || !is_dbl<TT>::value) return hipErrorInvalidValue;
            LdSBasis<TT, Q> ld{(const double*)in.raw, in.scale, in.s, in.cur, in.stride, 0.0};
            hipLaunchKernelGGL((k_mw<KR, U, TI, TM, TT, Q, LdSBasis<TT, Q>>), grid, dim3(kBlock),
                               0, st, A, (const TM*)mv, neg, ld, (TT*)t, stop, cntr, nb);
            return hipGetLastError();
          }
          if (!in.scale) {
            if (in.type != tt) return hipErrorInvalidValue;
            LdVec<TT, Q> ld{(const TT*)in.raw};
            hipLaunchKernelGGL((k_mw<KR, U, TI, TM, TT, Q, LdVec<TT, Q>>), grid, dim3(kBlock), 0,
                               st, A, (const TM*)mv, neg, ld, (TT*)t, stop, cntr, nb);
            return hipGetLastError();
          }
          return with_type(in.type, [&](auto pin) -> hipError_t {
            using TIN = TYPE_OF(pin);
            using QQ = wider_t<TIN, Q>;
            LdBasis<TIN, TT, QQ> ld{(const TIN*)in.raw, in.scale, in.cur, in.stride, 0.0};
            hipLaunchKernelGGL((k_mw<KR, U, TI, TM, TT, QQ, LdBasis<TIN, TT, QQ>>), grid,
                               dim3(kBlock), 0, st, A, (const TM*)mv, neg, ld, (TT*)t, stop, cntr, nb);
            return hipGetLastError();
          });
        }
      });
    });
  });
});
}

hipError_t m_apply_g(hipStream_t st, const SellDesc& A, const void* mv, int tm, int neg, double gd,
                     const void* t, int tt, int mode, const double* omega, const void* zprev,
                     void* out, int tout, const double* s, int* fbflag, const int* stop,
                     const int* cur, int kr) {
  // block-Jacobi ILU(0): the backward sweep, y kept in place of t
  if (A.ilu)
    return ilu_apply_bwd(st, A, mv, tm, const_cast<void*>(t), tt, mode, omega, zprev, out, tout, s,
                         fbflag, stop, cur);
  if (mode != 3 && tout != tt) return hipErrorInvalidValue;
  return with_kr(kr, [&](auto KRc, auto Uc) {
  constexpr int KR = decltype(KRc)::value, U = decltype(Uc)::value;
  const int64_t nb = n_blocks_kr(A.n, KR);
  return with_idx(A.idx16, [&](auto pi) {
    using TI = TYPE_OF(pi);
    return with_type(tm, [&](auto pm) {
      using TM = TYPE_OF(pm);
      return with_type(tt, [&](auto pt) -> hipError_t {
        using TT = TYPE_OF(pt);
        if constexpr (!ok_m<TM, TT>() || !shape_ok<U, TT, TI>()) {
          return hipErrorInvalidValue;
        } else {
          using Q = wider_t<TM, TT>;
          const dim3 g((unsigned)physical_grid(nb)), b(kBlock);
          if (mode == 0) {
            EpiStore<TT, Q> ep{(TT*)out, fbflag};
            hipLaunchKernelGGL((k_mg<KR, U, TI, TM, TT, Q, EpiStore<TT, Q>>), g, b, 0, st, A,
                               (const TM*)mv, neg, (Q)gd, (const TT*)t, ep, stop, nb);
          } else if (mode == 1) {
            EpiZ1<TT, Q> ep{(TT*)out, omega, fbflag, (Q)0};
            hipLaunchKernelGGL((k_mg<KR, U, TI, TM, TT, Q, EpiZ1<TT, Q>>), g, b, 0, st, A, (const TM*)mv,
                               neg, (Q)gd, (const TT*)t, ep, stop, nb);
          } else if (mode == 2) {
            EpiZK<TT, Q> ep{(TT*)out, (const TT*)zprev, omega, fbflag, (Q)0};
            hipLaunchKernelGGL((k_mg<KR, U, TI, TM, TT, Q, EpiZK<TT, Q>>), g, b, 0, st, A, (const TM*)mv,
                               neg, (Q)gd, (const TT*)t, ep, stop, nb);
          } else {
            if constexpr (!is_dbl<TT>::value) {
              return hipErrorInvalidValue;
            } else {
              EpiS64 ep{(double*)out, s, fbflag, cur, A.n};
              hipLaunchKernelGGL((k_mg<KR, U, TI, TM, TT, Q, EpiS64>), g, b, 0, st, A, (const TM*)mv, neg,
                                 (Q)gd, (const TT*)t, ep, stop, nb);
            }
          }
          return hipGetLastError();
        }
      });
    });
  });
});
}

// ---------------------------------------------------------------------------
// Richardson pieces (Alg. 1)
// ---------------------------------------------------------------------------
template <int KR, int U, class TI, class TA, class TR, class Q, class LD>
__global__ __launch_bounds__(kBlock) void k_rres(SellDesc A, const TA* __restrict__ av, LD ld,
                                                 const TR* __restrict__ z, TR* __restrict__ r,
                                                 const int* stop, int64_t nb) {
  const int64_t lb = logical_block(nb);
  if (lb >= nb) return;
  const int sy = sys_of(A.sys, lb * (kBlock * KR));
  stop = sys_ptr(stop, sy, A.sys.dI);
  if (A.sys.blk && stop && *stop) return;
  const int stopped = read_flag(stop);  // checked at the stores (one system)
  const int wave = wave_index(), lane = threadIdx.x & (kWave - 1);
  RowSlot s[KR];
  make_slots(A, lb * 4 + wave, lane, s);
  ld.at_sys(sy, A.sys);
  ld.init();
  int kb[KR], ke[KR], kc[KR];
  Q acc[KR];
#pragma unroll
  for (int q = 0; q < KR; q++) {
    kb[q] = 0;
    ke[q] = s[q].w;
    kc[q] = max(s[q].w, 1);
    acc[q] = 0;
  }
  typename LD::raw_t vr[KR];  // v at the row, loaded with the matrix entries
#pragma unroll
  for (int q = 0; q < KR; q++) vr[q] = ld.raw(s[q].row);
  rows_sum<U, TI>(av, (const TI*)A.idx, s, kb, kc, kb, ke, acc, LdVec<TR, Q>{z});
#pragma unroll
  for (int q = 0; q < KR; q++)
    if (s[q].ok && !stopped) r[s[q].row] = round_to<TR>(ld.cook(vr[q]) - acc[q]);
}

hipError_t rich_residual(hipStream_t st, const SellDesc& A, const void* av, int ta,
                         const Basis& in, const void* z, void* r, int tr, const int* stop, int kr) {
  return with_kr<true>(kr, [&](auto KRc, auto Uc) {
  constexpr int KR = decltype(KRc)::value, U = decltype(Uc)::value;
  const int64_t nb = n_blocks_kr(A.n, KR);
  const dim3 grid((unsigned)physical_grid(nb));
  return with_idx(A.idx16, [&](auto pi) {
    using TI = TYPE_OF(pi);
    return with_type(ta, [&](auto pa) {
      using TA = TYPE_OF(pa);
      return with_type(tr, [&](auto pr) -> hipError_t {
        using TR = TYPE_OF(pr);
        if constexpr (!ok_m<TA, TR>() || !shape_ok<U, TR, TI>()) {
          return hipErrorInvalidValue;
        } else {
          using Q = wider_t<TA, TR>;
          if (!in.scale) {
            // a stored vector of the level's own type (the input a Richardson
            // level receives from a Richardson level above it)
            if (in.type != tr || in.cur) return hipErrorInvalidValue;
            LdVec<TR, Q> ld{(const TR*)in.raw};
            hipLaunchKernelGGL((k_rres<KR, U, TI, TA, TR, Q, LdVec<TR, Q>>), grid, dim3(kBlock), 0, st,
                               A, (const TA*)av, ld, (const TR*)z, (TR*)r, stop, nb);
            return hipGetLastError();
          }
          return with_type(in.type, [&](auto pin) -> hipError_t {
            using TIN = TYPE_OF(pin);
            using QQ = wider_t<TIN, Q>;
            LdBasis<TIN, TR, QQ> ld{(const TIN*)in.raw, in.scale, in.cur, in.stride, 0.0};
            hipLaunchKernelGGL((k_rres<KR, U, TI, TA, TR, QQ, LdBasis<TIN, TR, QQ>>), grid,
                               dim3(kBlock), 0, st, A, (const TA*)av, ld, (const TR*)z, (TR*)r, stop,
                               nb);
            return hipGetLastError();
          });
        }
      });
    });
  });
});
}

template <class TI, class TA, class TR, class Q, class LD>
__global__ __launch_bounds__(kBlock) void k_rtdots(SellDesc A, const TA* __restrict__ av,
                                                   const TR* __restrict__ y, LD rld,
                                                   Q* __restrict__ part, int64_t nb,
                                                   const int* stop) {
  __shared__ Q lds[kBlock / kWave];
  const int64_t lb = logical_block(nb);
  if (lb >= nb) return;
  const int sy = sys_of(A.sys, lb * kRowsPerBlock);
  stop = sys_ptr(stop, sy, A.sys.dI);
  if (stop && *stop) return;
  const int wave = wave_index(), lane = threadIdx.x & (kWave - 1);
  RowSlot s[kR];
  make_slots(A, lb * 4 + wave, lane, s);
  rld.at_sys(sy, A.sys);
  rld.init();
  int kb[kR], ke[kR], kc[kR];
  Q acc[kR];
#pragma unroll
  for (int q = 0; q < kR; q++) {
    kb[q] = 0;
    ke[q] = s[q].w;
    kc[q] = max(s[q].w, 1);
    acc[q] = 0;
  }
  rows_sum<kUnroll, TI>(av, (const TI*)A.idx, s, kb, kc, kb, ke, acc, LdVec<TR, Q>{y});
  Q p1 = 0, p2 = 0;
#pragma unroll
  for (int q = 0; q < kR; q++) {
    if (s[q].ok) {
      const Q rv = rld(s[q].row);
      p1 = p1 + rv * acc[q];
      p2 = p2 + acc[q] * acc[q];
    }
  }
  const Q s1 = block_sum(p1, lds);
  const Q s2 = block_sum(p2, lds);
  if (threadIdx.x == 0) {
    part[lb] = s1;
    part[nb + lb] = s2;
  }
}

hipError_t rich_tdots(hipStream_t st, const SellDesc& A, const void* av, int ta, const void* y,
                      int ty, const Basis& rin, void* partials, const int* stop) {
  const int64_t nb = n_blocks(A.n);
  return with_idx(A.idx16, [&](auto pi) {
    using TI = TYPE_OF(pi);
    return with_type(ta, [&](auto pa) {
      using TA = TYPE_OF(pa);
      return with_type(ty, [&](auto py) -> hipError_t {
        using TR = TYPE_OF(py);
        if constexpr (!ok_m<TA, TR>()) {
          return hipErrorInvalidValue;
        } else {
          using Q = wider_t<TA, TR>;
          if (!rin.scale) {
            LdVec<TR, Q> ld{(const TR*)rin.raw};
            hipLaunchKernelGGL((k_rtdots<TI, TA, TR, Q, LdVec<TR, Q>>), grid_for(A.n), dim3(kBlock),
                               0, st, A, (const TA*)av, (const TR*)y, ld, (Q*)partials, nb, stop);
            return hipGetLastError();
          }
          return with_type(rin.type, [&](auto pin) -> hipError_t {
            using TIN = TYPE_OF(pin);
            if constexpr (!std::is_same<wider_t<TIN, Q>, Q>::value) {
              return hipErrorInvalidValue;
            } else {
              LdBasis<TIN, TR, Q> ld{(const TIN*)rin.raw, rin.scale, rin.cur, rin.stride, 0.0};
              hipLaunchKernelGGL((k_rtdots<TI, TA, TR, Q, LdBasis<TIN, TR, Q>>), grid_for(A.n),
                                 dim3(kBlock), 0, st, A, (const TA*)av, (const TR*)y, ld,
                                 (Q*)partials, nb, stop);
              return hipGetLastError();
            }
          });
        }
      });
    });
  });
}

template <class Q>
__global__ __launch_bounds__(kFinBlock) void k_romega(const Q* __restrict__ part, int64_t nb,
                                                      double* om, double* wcur,
                                                      const int64_t* cntr, int c, const int* stop,
                                                      SysLayout sl) {
  const int sy = blockIdx.x;
  stop = sys_ptr(stop, sy, sl.dI);
  if (stop && *stop) return;
  om = sys_ptr(om, sy, sl.dS);
  wcur = sys_ptr(wcur, sy, sl.dS);
  int64_t lo, hi;
  sys_range(sl, sy, nb, lo, hi);
  __shared__ Q lds[kFinBlock / kWave];
  const Q num = fin_block_sum(thread_sum(part + lo, hi - lo), lds);
  const Q den = fin_block_sum(thread_sum(part + nb + lo, hi - lo), lds);
  if (threadIdx.x == 0) {
    const int64_t l = (*cntr - 1) / c;  // Eq. (5): l = c_ntr / c
    const Q wp = num / den;
    const Q ok = (Q)(*om);
    if (den > (Q)0 && isfinite((double)wp)) {
      Q v = (Q)l * ok;
      v = v + wp;
      v = v / (Q)(l + 1);
      *om = (double)v;
      *wcur = (double)wp;
    } else {
      *wcur = (double)ok;
    }
  }
}

__global__ void k_cntr_advance(int64_t* c) {
  if (threadIdx.x == 0) *c += 1;
}

hipError_t cntr_advance(hipStream_t st, int64_t* cntr) {
  hipLaunchKernelGGL(k_cntr_advance, dim3(1), dim3(64), 0, st, cntr);
  return hipGetLastError();
}

hipError_t rich_omega(hipStream_t st, const SysLayout& sl, int q, const void* partials, int64_t nb,
                      double* omega_k, double* wcur, const int64_t* cntr, int c, const int* stop) {
  if (c <= 0) return hipErrorInvalidValue;
  const dim3 g((unsigned)sl.nsys);
  if (q == T64)
    hipLaunchKernelGGL(k_romega<double>, g, dim3(kFinBlock), 0, st, (const double*)partials, nb,
                       omega_k, wcur, cntr, c, stop, sl);
  else
    hipLaunchKernelGGL(k_romega<float>, g, dim3(kFinBlock), 0, st, (const float*)partials, nb,
                       omega_k, wcur, cntr, c, stop, sl);
  return hipGetLastError();
}

template <class TR, class Q>
__global__ __launch_bounds__(kBlock) void k_zupd(SysLayout sl, int64_t n, const TR* __restrict__ zp,
                                                 const TR* __restrict__ y, const double* wcur,
                                                 TR* __restrict__ z, int* fb, const int* stop,
                                                 int64_t nb) {
  const int64_t lb = logical_block(nb);
  if (lb >= nb) return;
  const int sy = sys_of(sl, lb * kRowsPerBlock);
  stop = sys_ptr(stop, sy, sl.dI);
  if (stop && *stop) return;
  wcur = sys_ptr(wcur, sy, sl.dS);
  fb = sys_ptr(fb, sy, sl.dI);
  const Q w = (Q)(*wcur);
#pragma unroll
  for (int r = 0; r < kR; r++) {
    const int64_t row = lb * kRowsPerBlock + (int64_t)r * kBlock + threadIdx.x;
    if (row >= n) continue;
    const Q p = w * widen<Q>(y[row]);
    const TR zz = zp ? round_to<TR>(widen<Q>(zp[row]) + p) : round_to<TR>(p);
    z[row] = zz;
    if (fb && !finite_val(zz)) atomicOr(fb, 1);
  }
}

hipError_t rich_zupdate(hipStream_t st, const SysLayout& sl, int64_t n, const void* zprev, const void* y, int tr,
                        const double* wcur, void* z, int* fbflag, const int* stop) {
  const int64_t nb = n_blocks(n);
  return with_type(tr, [&](auto pr) {
    using TR = TYPE_OF(pr);
    using Q = wider_t<TR, TR>;
    hipLaunchKernelGGL((k_zupd<TR, Q>), grid_for(n), dim3(kBlock), 0, st, sl, n, (const TR*)zprev,
                       (const TR*)y, wcur, (TR*)z, fbflag, stop, nb);
    return hipGetLastError();
  });
}

// ---------------------------------------------------------------------------
// utilities
// ---------------------------------------------------------------------------
template <class TI, class TO>
__global__ void k_convert(int64_t n, const TI* __restrict__ in, TO* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = round_to<TO>(widen<double>(in[i]));
}

hipError_t convert(hipStream_t st, int64_t n, const void* in, int ti, void* out, int to) {
  return with_type(ti, [&](auto pi) {
    using TI = TYPE_OF(pi);
    return with_type(to, [&](auto po) {
      using TO = TYPE_OF(po);
      hipLaunchKernelGGL((k_convert<TI, TO>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n,
                         (const TI*)in, (TO*)out);
      return hipGetLastError();
    });
  });
}

template <class T> __global__ void k_fill_nan(T* p, int64_t count, int* flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = round_to<T>((double)NAN);
  if (i == 0 && flag) *flag = 1;
}

hipError_t fill_nan(hipStream_t st, void* p, int t, int64_t count, int* flag) {
  return with_type(t, [&](auto pt) {
    using T = TYPE_OF(pt);
    hipLaunchKernelGGL((k_fill_nan<T>), dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st,
                       (T*)p, count, flag);
    return hipGetLastError();
  });
}

__global__ void k_set(double* p, int m, double v, SysLayout sl) {
  p = sys_ptr(p, (int)blockIdx.x, sl.dS);
  if ((int)threadIdx.x < m) p[threadIdx.x] = v;
}

hipError_t set_omega(hipStream_t st, const SysLayout& sl, double* omega, int m, double v) {
  hipLaunchKernelGGL(k_set, dim3((unsigned)sl.nsys), dim3(64), 0, st, omega, m, v, sl);
  return hipGetLastError();
}

// holds every system s with mask[s]: I[I_HOLD] = I[I_STOP] = 1 (the host's
// per-system decision that a system has finished)
__global__ void k_sys_hold(int* I, const int* mask, SysLayout sl) {
  const int sy = blockIdx.x * blockDim.x + threadIdx.x;
  if (sy < sl.nsys && mask[sy]) {
    int* Is = sys_ptr(I, sy, sl.dI);
    Is[I_HOLD] = 1;
    Is[I_STOP] = 1;
  }
}

hipError_t sys_hold(hipStream_t st, const SysLayout& sl, int* I, const int* mask) {
  hipLaunchKernelGGL(k_sys_hold, dim3((unsigned)((sl.nsys + 255) / 256)), dim3(256), 0, st, I, mask, sl);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// stacked systems
// ---------------------------------------------------------------------------
__global__ void k_stack(StackIo io, double* cat, int to_cat) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= io.n) return;
  const int sy = sys_of(io.sl, i);
  const int64_t local = i - io.row0[sy];
  const bool own = local < io.nrows[sy];
  if (to_cat)
    cat[i] = own ? io.ptrs[sy][local] : 0.0;
  else if (own)
    io.ptrs[sy][local] = cat[i];
}

hipError_t stack_gather(hipStream_t st, const StackIo& io, double* cat) {
  hipLaunchKernelGGL(k_stack, dim3((unsigned)((io.n + 255) / 256)), dim3(256), 0, st, io, cat, 1);
  return hipGetLastError();
}

hipError_t stack_scatter(hipStream_t st, const StackIo& io, const double* cat) {
  hipLaunchKernelGGL(k_stack, dim3((unsigned)((io.n + 255) / 256)), dim3(256), 0, st, io,
                     const_cast<double*>(cat), 0);
  return hipGetLastError();
}

}  // namespace f3r
