// Block-Jacobi ILU(0) (see ilu.h): level schedules, the factorisation and
// the two triangular sweeps, one workgroup per row block.
//
// Every row is processed by one thread, in the order of the definition: the
// factorisation walks the row's entries left of the diagonal in increasing
// column order (l_ik = a_ik / u_kk, then a_ij -= l_ik u_kj for the later
// entries j that row k also holds); the forward sweep forms
// t_i = r_i - sum_k l_ik t_k and the backward sweep
// y_i = (t_i - sum_j u_ij y_j) / u_ii, terms in column order with separate
// multiply and subtract.  Rows of one level do not depend on each other, so
// the order inside a level changes nothing.
#include "ilu.h"

#include "common.h"
#include "kernels.h"
#include "sell.h"
#include "setup.h"

namespace f3r {

namespace {

__device__ __forceinline__ int64_t blk_start(int64_t b, int64_t n, int nb) { return (b * n) / nb; }

// one row of the device format: first element, width, diagonal position
struct RowAt {
  uint32_t e0;
  int w, dp;
};
__device__ __forceinline__ RowAt row_at(const SellDesc& A, int64_t i) {
  const int64_t s = i / kWave;
  const uint32_t lane = (uint32_t)(i % kWave);
  RowAt r;
  if (A.dell_w > 0) {
    r.e0 = (uint32_t)(s * kWave * A.dell_w) + lane;
    r.w = A.dell_w;
  } else {
    const uint32_t o0 = A.off[s];
    r.e0 = o0 + lane;
    r.w = (int)((A.off[s + 1] - o0) / kWave);
  }
  r.dp = (int)A.kd[i];  // the diagonal-aligned format stores the common position
  return r;
}
template <class TI>
__device__ __forceinline__ int64_t col_at(const SellDesc& A, const RowAt& r, int64_t i, int p) {
  return col_of<TI>(idx_lane<TI>((const TI*)A.idx, r.e0, p), i, A.n);
}
__device__ __forceinline__ uint32_t at(const RowAt& r, int p) { return r.e0 + (uint32_t)p * kWave; }

// Levels of both sweeps and the rows sorted by level, one block per
// workgroup, computed by its first thread (set-up only).
template <class TI>
__global__ void k_ilu_sched(SellDesc A, IluBuild b) {
  if (threadIdx.x != 0) return;
  const int bk = blockIdx.x;
  const int64_t n = A.n;
  const int64_t r0 = blk_start(bk, n, b.blocks), r1 = blk_start(bk + 1, n, b.blocks);
  for (int dir = 0; dir < 2; dir++) {
    int* rows = dir == 0 ? b.rows_lo : b.rows_up;
    int* lptr = (dir == 0 ? b.lptr_lo : b.lptr_up) + r0 + bk;
    int maxl = 0;
    for (int64_t q = 0; q < r1 - r0; q++) {
      const int64_t i = dir == 0 ? r0 + q : r1 - 1 - q;
      const RowAt ra = row_at(A, i);
      int l = 0;
      for (int p = 0; p < ra.w; p++) {
        if (p == ra.dp) continue;
        const int64_t c = col_at<TI>(A, ra, i, p);
        if (c == i || c < r0 || c >= r1) continue;  // padding, dropped coupling
        if (dir == 0 ? c < i : c > i) l = max(l, b.lev[c] + 1);
      }
      b.lev[i] = l;
      maxl = max(maxl, l);
    }
    const int nl = maxl + 1;
    for (int l = 0; l <= nl; l++) lptr[l] = 0;
    for (int64_t i = r0; i < r1; i++) lptr[b.lev[i] + 1]++;
    for (int l = 0; l < nl; l++) lptr[l + 1] += lptr[l];
    for (int64_t i = r0; i < r1; i++) rows[r0 + lptr[b.lev[i]]++] = (int)i;
    for (int l = nl; l > 0; l--) lptr[l] = lptr[l - 1];
    lptr[0] = 0;
    (dir == 0 ? b.nlev_lo : b.nlev_up)[bk] = nl;
  }
}

template <class TI>
__global__ __launch_bounds__(kIluThreads) void k_ilu_factor(SellDesc A, IluBuild b,
                                                            double* __restrict__ v) {
  const int bk = blockIdx.x;
  const int64_t n = A.n;
  const int64_t r0 = blk_start(bk, n, b.blocks);
  const int* lptr = b.lptr_lo + r0 + bk;
  const int nl = b.nlev_lo[bk];
  for (int l = 0; l < nl; l++) {
    for (int q = lptr[l] + (int)threadIdx.x; q < lptr[l + 1]; q += kIluThreads) {
      const int64_t i = b.rows_lo[r0 + q];
      const RowAt ra = row_at(A, i);
      for (int p = 0; p < ra.dp; p++) {
        const int64_t k = col_at<TI>(A, ra, i, p);
        if (k == i || k < r0) continue;  // padding, dropped coupling
        const RowAt rk = row_at(A, k);
        const double lik = v[at(ra, p)] / v[at(rk, rk.dp)];
        v[at(ra, p)] = lik;
        int qk = rk.dp + 1;
        for (int pj = p + 1; pj < ra.w; pj++) {
          const int64_t j = col_at<TI>(A, ra, i, pj);
          if (j == i && pj != ra.dp) continue;  // padding
          // row k's upper entries ascend; its padding (column k) never matches
          while (qk < rk.w && col_at<TI>(A, rk, k, qk) < j) qk++;
          if (qk < rk.w && col_at<TI>(A, rk, k, qk) == j)
            v[at(ra, pj)] = v[at(ra, pj)] - lik * v[at(rk, qk)];
        }
      }
    }
    __syncthreads();
  }
}

// fp64 factors checked, narrow copies rounded from them
template <class T>
__device__ __forceinline__ void put_narrow(void* p, int64_t e, double x, int* bad) {
  if (!p) return;
  const T r = round_to<T>(x);
  ((T*)p)[e] = r;
  if (!finite_val(r)) *bad |= SF_RANGE;
}
__global__ void k_ilu_finish(int64_t count, const double* __restrict__ v, void* n32, void* n16,
                             void* nb16, int* flags) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count) return;
  const double x = v[e];
  int bad = isfinite(x) ? 0 : SF_MATRIX;
  put_narrow<float>(n32, e, x, &bad);
  put_narrow<f16>(n16, e, x, &bad);
  put_narrow<bf16>(nb16, e, x, &bad);
  if (bad) atomicOr(flags, bad);
}

// Offsets of each position's in-block entries inside the block's CSR range
// (first thread of the block, sequentially); the block's end follows its
// last position, hence n + blocks + 1 offsets.
template <class TI>
__global__ void k_ilu_pack_ptr(SellDesc A, IluBuild b, const int32_t* __restrict__ rp) {
  if (threadIdx.x != 0) return;
  const int bk = blockIdx.x;
  const int64_t n = A.n;
  const int64_t r0 = blk_start(bk, n, b.blocks), r1 = blk_start(bk + 1, n, b.blocks);
  for (int dir = 0; dir < 2; dir++) {
    const int* rows = dir == 0 ? b.rows_lo : b.rows_up;
    int* ptr = dir == 0 ? b.ptr_lo : b.ptr_up;
    int acc = rp[r0];
    for (int64_t q = 0; q < r1 - r0; q++) {
      ptr[r0 + bk + q] = acc;
      const int64_t i = rows[r0 + q];
      const RowAt ra = row_at(A, i);
      for (int p = 0; p < ra.w; p++) {
        if (p == ra.dp) continue;
        const int64_t c = col_at<TI>(A, ra, i, p);
        if (c == i || c < r0 || c >= r1) continue;
        if (dir == 0 ? c < i : c > i) acc++;
      }
    }
    ptr[r1 + bk] = acc;  // this block's end
  }
}

// Entries of one position in column order; cols when write_cols.
template <class TI, class TM>
__global__ void k_ilu_pack_fill(SellDesc A, IluBuild b, const TM* __restrict__ mv, TM* val_lo,
                                TM* val_up, TM* diag_up, int write_cols) {
  const int64_t pos = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = A.n;
  if (pos >= n) return;
  // the block of this position (positions r0 .. r1 belong to block b)
  int64_t bk = (pos * b.blocks) / n;
  while (bk + 1 <= b.blocks && blk_start(bk + 1, n, b.blocks) <= pos) bk++;
  while (bk > 0 && blk_start(bk, n, b.blocks) > pos) bk--;
  const int64_t r0 = blk_start(bk, n, b.blocks), r1 = blk_start(bk + 1, n, b.blocks);
  for (int dir = 0; dir < 2; dir++) {
    const int64_t i = (dir == 0 ? b.rows_lo : b.rows_up)[pos];
    int e = (dir == 0 ? b.ptr_lo : b.ptr_up)[pos + bk];
    const RowAt ra = row_at(A, i);
    for (int p = 0; p < ra.w; p++) {
      if (p == ra.dp) continue;
      const int64_t c = col_at<TI>(A, ra, i, p);
      if (c == i || c < r0 || c >= r1) continue;
      if (dir == 0 ? c < i : c > i) {
        if (write_cols) (dir == 0 ? b.col_lo : b.col_up)[e] = (int)(c - r0);
        (dir == 0 ? val_lo : val_up)[e] = mv[at(ra, p)];
        e++;
      }
    }
    if (dir == 1) diag_up[pos] = mv[at(ra, ra.dp)];
  }
}

// Levels grouped greedily into windows of at most win_pos positions and
// win_ent entries, both sweeps (first thread of the block).
__global__ void k_ilu_windows(SellDesc A, IluBuild b, int* flags) {
  if (threadIdx.x != 0) return;
  const int bk = blockIdx.x;
  const int64_t r0 = blk_start(bk, A.n, b.blocks);
  for (int dir = 0; dir < 2; dir++) {
    const int* lptr = (dir == 0 ? b.lptr_lo : b.lptr_up) + r0 + bk;
    const int* pk = (dir == 0 ? b.ptr_lo : b.ptr_up) + r0 + bk;
    int* wst = (dir == 0 ? b.wst_lo : b.wst_up) + r0 + bk;
    const int nl = (dir == 0 ? b.nlev_lo : b.nlev_up)[bk];
    int w = 0, pos = 0, ent = 0, bad = 0;
    wst[0] = 0;
    for (int l = 0; l < nl; l++) {
      const int pl = lptr[l + 1] - lptr[l];
      const int el = pk[lptr[l + 1]] - pk[lptr[l]];
      if (pl > b.win_pos || el > b.win_ent) bad = 1;
      if (pos + pl > b.win_pos || ent + el > b.win_ent) {
        wst[++w] = l;
        pos = ent = 0;
      }
      pos += pl;
      ent += el;
    }
    wst[w + 1] = nl;
    (dir == 0 ? b.nwin_lo : b.nwin_up)[bk] = w + 1;
    if (bad) atomicOr(flags, SF_ILU_NOWIN);
  }
}

// LDS carve-up of the windowed sweeps: the block's vector, then the window
// (rows as offsets from r0, entry offsets, level bounds, entry columns,
// entry values, and U's diagonal for the backward sweep)
struct WinLds {
  int row, ptr, lev, col, val, du, total;
  int ent;  // entry capacity of the window
};
__host__ __device__ inline int al16(int x) { return (x + 15) & ~15; }
__host__ __device__ inline WinLds win_lds(int rows_max, int stt, int stm, int pos, int ent) {
  WinLds w;
  int o = al16(rows_max * stt);
  w.row = o;
  o += al16(pos * 4);
  w.ptr = o;
  o += al16((pos + 1) * 4);
  w.lev = o;
  o += al16((pos + 1) * 4);
  w.col = o;
  o += al16(ent * 4);
  w.val = o;
  o += al16(ent * stm);
  w.du = o;
  o += al16(pos * stm);
  w.total = o;
  w.ent = ent;
  return w;
}

// acc minus the sum over the row's window entries [p0, p1) of val * t[col],
// in entry order, four at a time: the four columns and values are read
// together, then the four vector values, then the differences are formed in
// order; positions past p1 (still inside the window arrays) are masked and
// read column 0.  Taken for long rows (27-point stencils: 13 entries per
// sweep row); rows of three entries are faster one entry at a time.
template <class Q, class TM, class TT>
__device__ __forceinline__ Q row_sub(Q acc, int p0, int p1, const int* wcol, const TM* wval, const TT* tl,
                                     int ent) {
  for (int p = p0; p < p1; p += 4) {
    int c[4];
    TM v[4];
#pragma unroll
    for (int u = 0; u < 4; u++) {
      const int pu = min(p + u, ent - 1);
      const int cw = wcol[pu];
      c[u] = p + u < p1 ? cw : 0;
      v[u] = wval[pu];
    }
    TT x[4];
#pragma unroll
    for (int u = 0; u < 4; u++) x[u] = tl[c[u]];
#pragma unroll
    for (int u = 0; u < 4; u++) {
      const Q t = acc - widen<Q>(v[u]) * widen<Q>(x[u]);
      acc = p + u < p1 ? t : acc;
    }
  }
  return acc;
}

// One window of sweep data into LDS (every thread, then a barrier).
template <class TM>
__device__ __forceinline__ void load_window(const int* rows, const int* pk, const int* lptr, const int* col,
                                            const TM* val, const TM* du, int64_t r0, int la, int lb, int qa,
                                            int qb, int ea, int eb, int* wrow, int* wptr, int* wlev, int* wcol,
                                            TM* wval, TM* wdu) {
  for (int q = qa + (int)threadIdx.x; q < qb; q += kIluThreads) {
    wrow[q - qa] = (int)(rows[r0 + q] - r0);
    wptr[q - qa] = pk[q] - ea;
    if (du) wdu[q - qa] = du[r0 + q];
  }
  for (int l = la + (int)threadIdx.x; l <= lb; l += kIluThreads) wlev[l - la] = lptr[l] - qa;
  if (threadIdx.x == 0) wptr[qb - qa] = eb - ea;
  for (int e = ea + (int)threadIdx.x; e < eb; e += kIluThreads) {
    wcol[e - ea] = col[e];
    wval[e - ea] = val[e];
  }
  __syncthreads();
}

// t = L^-1 r from LDS: the input is first placed in the block's LDS vector
// (each loader returns values of the vector type, so this is exact), every
// level then reads and writes LDS only.
template <class TM, class TT, class Q, class LD, bool CH>
__global__ __launch_bounds__(kIluThreads) void k_ilu_fwd_win(SellDesc A, IluDesc D, const TM* __restrict__ vl,
                                                             LD ld, TT* __restrict__ t, const int* stop,
                                                             int64_t* cntr, WinLds L) {
  extern __shared__ __align__(16) unsigned char ilu_lds[];
  if (cntr && blockIdx.x == 0 && threadIdx.x == 0) *cntr += 1;
  if (read_flag(stop)) return;
  const int bk = blockIdx.x;
  const int64_t r0 = blk_start(bk, A.n, D.blocks), r1 = blk_start(bk + 1, A.n, D.blocks);
  const int rows = (int)(r1 - r0);
  TT* tl = reinterpret_cast<TT*>(ilu_lds);
  int* wrow = reinterpret_cast<int*>(ilu_lds + L.row);
  int* wptr = reinterpret_cast<int*>(ilu_lds + L.ptr);
  int* wlev = reinterpret_cast<int*>(ilu_lds + L.lev);
  int* wcol = reinterpret_cast<int*>(ilu_lds + L.col);
  TM* wval = reinterpret_cast<TM*>(ilu_lds + L.val);
  ld.at_sys(0, A.sys);
  ld.init();
#pragma unroll 4
  for (int i = threadIdx.x; i < rows; i += kIluThreads) tl[i] = round_to<TT>(ld(r0 + i));
  const int* lptr = D.lptr_lo + r0 + bk;
  const int* pk = D.ptr_lo + r0 + bk;
  const int* wst = D.wst_lo + r0 + bk;
  const int nw = D.nwin_lo[bk];
  for (int w = 0; w < nw; w++) {
    const int la = wst[w], lb = wst[w + 1];
    const int qa = lptr[la], qb = lptr[lb];
    __syncthreads();  // the previous window's levels (or the input) are done
    load_window<TM>(D.rows_lo, pk, lptr, D.col_lo, vl, nullptr, r0, la, lb, qa, qb, pk[qa], pk[qb], wrow,
                    wptr, wlev, wcol, wval, nullptr);
    for (int l = 0; l < lb - la; l++) {
      const int q1 = wlev[l + 1];
      for (int q = wlev[l] + (int)threadIdx.x; q < q1; q += kIluThreads) {
        const int i = wrow[q];
        Q acc = widen<Q>(tl[i]);
        if constexpr (CH) {
          acc = row_sub<Q>(acc, wptr[q], wptr[q + 1], wcol, wval, tl, L.ent);
        } else {
          const int p1 = wptr[q + 1];
          for (int p = wptr[q]; p < p1; p++) acc = acc - widen<Q>(wval[p]) * widen<Q>(tl[wcol[p]]);
        }
        tl[i] = round_to<TT>(acc);
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < rows; i += kIluThreads) t[r0 + i] = tl[i];
}

// y = U^-1 t from LDS, in place of t; the epilogue is a separate pass over
// all rows (k_ilu_epi), so no level waits for its loads.
template <class TM, class TT, class Q, bool CH>
__global__ __launch_bounds__(kIluThreads) void k_ilu_bwd_win(SellDesc A, IluDesc D, const TM* __restrict__ vu,
                                                             const TM* __restrict__ du, TT* __restrict__ t,
                                                             const int* stop, WinLds L) {
  extern __shared__ __align__(16) unsigned char ilu_lds[];
  if (read_flag(stop)) return;
  const int bk = blockIdx.x;
  const int64_t r0 = blk_start(bk, A.n, D.blocks), r1 = blk_start(bk + 1, A.n, D.blocks);
  const int rows = (int)(r1 - r0);
  TT* tl = reinterpret_cast<TT*>(ilu_lds);
  int* wrow = reinterpret_cast<int*>(ilu_lds + L.row);
  int* wptr = reinterpret_cast<int*>(ilu_lds + L.ptr);
  int* wlev = reinterpret_cast<int*>(ilu_lds + L.lev);
  int* wcol = reinterpret_cast<int*>(ilu_lds + L.col);
  TM* wval = reinterpret_cast<TM*>(ilu_lds + L.val);
  TM* wdu = reinterpret_cast<TM*>(ilu_lds + L.du);
#pragma unroll 4
  for (int i = threadIdx.x; i < rows; i += kIluThreads) tl[i] = t[r0 + i];
  const int* lptr = D.lptr_up + r0 + bk;
  const int* pk = D.ptr_up + r0 + bk;
  const int* wst = D.wst_up + r0 + bk;
  const int nw = D.nwin_up[bk];
  for (int w = 0; w < nw; w++) {
    const int la = wst[w], lb = wst[w + 1];
    const int qa = lptr[la], qb = lptr[lb];
    __syncthreads();
    load_window<TM>(D.rows_up, pk, lptr, D.col_up, vu, du, r0, la, lb, qa, qb, pk[qa], pk[qb], wrow, wptr,
                    wlev, wcol, wval, wdu);
    for (int l = 0; l < lb - la; l++) {
      const int q1 = wlev[l + 1];
      for (int q = wlev[l] + (int)threadIdx.x; q < q1; q += kIluThreads) {
        const int i = wrow[q];
        Q acc = widen<Q>(tl[i]);
        if constexpr (CH) {
          acc = row_sub<Q>(acc, wptr[q], wptr[q + 1], wcol, wval, tl, L.ent);
        } else {
          const int p1 = wptr[q + 1];
          for (int p = wptr[q]; p < p1; p++) acc = acc - widen<Q>(wval[p]) * widen<Q>(tl[wcol[p]]);
        }
        tl[i] = round_to<TT>(acc / widen<Q>(wdu[q]));
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < rows; i += kIluThreads) t[r0 + i] = tl[i];
}

// the G sweep's epilogue over y = t, four rows per thread
template <class TT, class EPI>
__global__ __launch_bounds__(256) void k_ilu_epi(SellDesc A, const TT* __restrict__ t, EPI epi,
                                                 const int* stop) {
  if (read_flag(stop)) return;
  epi.at_sys(0, A.sys);
  epi.init();
  const int64_t base = ((int64_t)blockIdx.x * 256 * 4) + threadIdx.x;
  TT y[4];
#pragma unroll
  for (int k = 0; k < 4; k++) {
    const int64_t i = base + (int64_t)k * 256;
    const int64_t ic = i < A.n ? i : A.n - 1;
    epi.prefetch(k, ic);
    y[k] = t[ic];
  }
#pragma unroll
  for (int k = 0; k < 4; k++) {
    const int64_t i = base + (int64_t)k * 256;
    if (i < A.n) epi(k, i, y[k]);
  }
}

// The block's part of t lives in LDS when it fits (lds = true): a level
// then reads the previous levels' results from LDS instead of L2, and the
// block copies its rows to t once at the end.
template <class TM, class TT, class Q, class LD, bool LDS>
__global__ __launch_bounds__(kIluThreads) void k_ilu_fwd(SellDesc A, IluDesc D, const TM* __restrict__ vl,
                                                         LD ld, TT* __restrict__ t, const int* stop,
                                                         int64_t* cntr) {
  extern __shared__ __align__(16) unsigned char ilu_lds[];
  TT* tl = reinterpret_cast<TT*>(ilu_lds);
  if (cntr && blockIdx.x == 0 && threadIdx.x == 0) *cntr += 1;
  if (read_flag(stop)) return;  // one system: the whole launch is stopped or not
  const int bk = blockIdx.x;
  const int64_t r0 = blk_start(bk, A.n, D.blocks), r1 = blk_start(bk + 1, A.n, D.blocks);
  TT* tb = LDS ? tl : t + r0;  // the block's rows, from its first one
  ld.at_sys(0, A.sys);
  ld.init();
  const int* lptr = D.lptr_lo + r0 + bk;
  const int nl = D.nlev_lo[bk];
  for (int l = 0; l < nl; l++) {
    for (int q = lptr[l] + (int)threadIdx.x; q < lptr[l + 1]; q += kIluThreads) {
      const int64_t i = D.rows_lo[r0 + q];
      const int p0 = D.ptr_lo[r0 + bk + q], p1 = D.ptr_lo[r0 + bk + q + 1];
      Q acc = ld(i);
      for (int p = p0; p < p1; p++) acc = acc - widen<Q>(vl[p]) * widen<Q>(tb[D.col_lo[p]]);
      tb[i - r0] = round_to<TT>(acc);
    }
    __syncthreads();
  }
  if (LDS)
    for (int64_t i = r0 + threadIdx.x; i < r1; i += kIluThreads) t[i] = tl[i - r0];
}

template <class TM, class TT, class Q, class EPI, bool LDS>
__global__ __launch_bounds__(kIluThreads) void k_ilu_bwd(SellDesc A, IluDesc D, const TM* __restrict__ vu,
                                                         const TM* __restrict__ du, TT* __restrict__ t,
                                                         EPI epi, const int* stop) {
  extern __shared__ __align__(16) unsigned char ilu_lds[];
  TT* tl = reinterpret_cast<TT*>(ilu_lds);
  if (read_flag(stop)) return;
  const int bk = blockIdx.x;
  const int64_t r0 = blk_start(bk, A.n, D.blocks), r1 = blk_start(bk + 1, A.n, D.blocks);
  TT* tb = LDS ? tl : t + r0;
  epi.at_sys(0, A.sys);
  epi.init();
  if (LDS) {
    for (int64_t i = r0 + threadIdx.x; i < r1; i += kIluThreads) tl[i - r0] = t[i];
    __syncthreads();
  }
  const int* lptr = D.lptr_up + r0 + bk;
  const int nl = D.nlev_up[bk];
  for (int l = 0; l < nl; l++) {
    for (int q = lptr[l] + (int)threadIdx.x; q < lptr[l + 1]; q += kIluThreads) {
      const int64_t i = D.rows_up[r0 + q];
      const int p0 = D.ptr_up[r0 + bk + q], p1 = D.ptr_up[r0 + bk + q + 1];
      epi.prefetch(0, i);
      Q acc = widen<Q>(tb[i - r0]);
      for (int p = p0; p < p1; p++) acc = acc - widen<Q>(vu[p]) * widen<Q>(tb[D.col_up[p]]);
      const Q yq = acc / widen<Q>(du[r0 + q]);
      const TT y = round_to<TT>(yq);
      tb[i - r0] = y;
      epi(0, i, y);
    }
    __syncthreads();
  }
  if (LDS)
    for (int64_t i = r0 + threadIdx.x; i < r1; i += kIluThreads) t[i] = tl[i - r0];
}

}  // namespace

hipError_t ilu_schedule(hipStream_t st, const SellDesc& A, const IluBuild& b) {
  return with_idx(A.idx16, [&](auto pi) {
    using TI = TYPE_OF(pi);
    hipLaunchKernelGGL((k_ilu_sched<TI>), dim3((unsigned)b.blocks), dim3(64), 0, st, A, b);
    return hipGetLastError();
  });
}

hipError_t ilu_factor(hipStream_t st, const SellDesc& A, const IluBuild& b, double* v64,
                      void* const narrow[4], int* flags) {
  hipError_t e = with_idx(A.idx16, [&](auto pi) {
    using TI = TYPE_OF(pi);
    hipLaunchKernelGGL((k_ilu_factor<TI>), dim3((unsigned)b.blocks), dim3(kIluThreads), 0, st, A, b,
                       v64);
    return hipGetLastError();
  });
  if (e != hipSuccess) return e;
  int64_t count = 0;
  {
    // the arrays hold every position of the format, padding included
    const int64_t ns = n_slices(A.n);
    count = A.dell_w > 0 ? ns * kWave * A.dell_w : -1;
  }
  if (count < 0) {
    uint32_t last = 0;
    e = hipMemcpyAsync(&last, A.off + n_slices(A.n), sizeof(uint32_t), hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    count = last;
  }
  hipLaunchKernelGGL(k_ilu_finish, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, count, v64,
                     narrow[T32], narrow[T16], narrow[TB16], flags);
  return hipGetLastError();
}

hipError_t ilu_pack(hipStream_t st, const SellDesc& A, const IluBuild& b, const int32_t* rp,
                    const void* const mv[4], int* flags) {
  hipError_t e = with_idx(A.idx16, [&](auto pi) {
    using TI = TYPE_OF(pi);
    hipLaunchKernelGGL((k_ilu_pack_ptr<TI>), dim3((unsigned)b.blocks), dim3(64), 0, st, A, b, rp);
    return hipGetLastError();
  });
  if (e != hipSuccess) return e;
  int first = 1;
  for (int tg = 0; tg < 4; tg++) {
    if (!mv[tg]) continue;
    e = with_idx(A.idx16, [&](auto pi) {
      using TI = TYPE_OF(pi);
      return with_type(tg, [&](auto pm) {
        using TM = TYPE_OF(pm);
        hipLaunchKernelGGL((k_ilu_pack_fill<TI, TM>), dim3((unsigned)((A.n + 255) / 256)), dim3(256), 0,
                           st, A, b, (const TM*)mv[tg], (TM*)b.val_lo[tg], (TM*)b.val_up[tg],
                           (TM*)b.diag_up[tg], first);
        return hipGetLastError();
      });
    });
    if (e != hipSuccess) return e;
    first = 0;
  }
  hipLaunchKernelGGL(k_ilu_windows, dim3((unsigned)b.blocks), dim3(64), 0, st, A, b, flags);
  return hipGetLastError();
}

// LDS bytes for the largest block's part of a vector of type tt, or 0 when
// it does not fit in the 64 KB a workgroup may take
static size_t lds_bytes(const SellDesc& A, int blocks, int tt, int lds_max) {
  const int64_t rows = (A.n + blocks - 1) / blocks + 1;
  const size_t bytes = (size_t)rows * type_size(tt);
  return bytes <= (size_t)lds_max ? bytes : 0;
}

void ilu_window_size(int64_t n, int blocks, int lds_max, int cus, int* win_pos, int* win_ent) {
  // the workgroups that share a compute unit share its LDS; per position
  // 14 bytes (row, entry offset, level bound, fp16 diagonal), per entry 6
  // (column, fp16 value), about four entries per position; no window needs
  // more positions than its block has rows
  // (at most 8 workgroups of kIluThreads threads fit a compute unit's 32
  // wave slots)
  int64_t per_cu = cus > 0 ? (blocks + cus - 1) / cus : 1;
  per_cu = per_cu < 1 ? 1 : (per_cu > 8 ? 8 : per_cu);
  const int64_t lds = (int64_t)lds_max / per_cu;
  const int64_t rows = (n + blocks - 1) / blocks + 1;
  const int64_t budget = lds - al16((int)(rows * 2)) - 1024;
  int64_t pos = budget > 0 ? budget / (14 + 4 * 6) : 0;
  const int64_t cap = (rows + 63) & ~(int64_t)63;
  pos = pos > cap ? cap : pos;
  pos = pos > 4096 ? 4096 : pos;
  pos &= ~(int64_t)63;
  pos = pos < 64 ? 64 : pos;
  *win_pos = (int)pos;
  *win_ent = (int)(4 * pos);
}

hipError_t ilu_apply_fwd(hipStream_t st, const SellDesc& A, const void* mv, int tm, const Basis& in,
                         void* t, int tt, const int* stop, int64_t* cntr) {
  const IluDesc D = *A.ilu;
  const dim3 grid((unsigned)D.blocks), blk(kIluThreads);
  const size_t lb = lds_bytes(A, D.blocks, tt, D.lds_max);
  if (!mv || tm < 0 || tm > 3 || !D.val_lo[tm]) return hipErrorInvalidValue;
  const int rows_max = (int)((A.n + D.blocks - 1) / D.blocks + 1);
  return with_type(tm, [&](auto pm) {
    using TM = TYPE_OF(pm);
    const TM* vl = (const TM*)D.val_lo[tm];
    return with_type(tt, [&](auto pt) -> hipError_t {
      using TT = TYPE_OF(pt);
      if constexpr (!ok_m<TM, TT>()) {
        return hipErrorInvalidValue;
      } else {
        const WinLds wl = win_lds(rows_max, (int)sizeof(TT), (int)sizeof(TM), D.win_pos, D.win_ent);
        const bool win = D.win && wl.total <= D.lds_max;
        // windowed LDS sweep when the block vector and a window fit, else
        // the LDS vector alone, else the global vector
        if (D.used) *D.used |= win ? 1 : (lb ? 2 : 4);
        auto go = [&](auto ld, auto qtag) -> hipError_t {
          using LDT = decltype(ld);
          using QQ = TYPE_OF(qtag);
          if (win)
            if (D.chunk)
              hipLaunchKernelGGL((k_ilu_fwd_win<TM, TT, QQ, LDT, true>), grid, blk, (size_t)wl.total, st, A, D,
                                 vl, ld, (TT*)t, stop, cntr, wl);
            else
              hipLaunchKernelGGL((k_ilu_fwd_win<TM, TT, QQ, LDT, false>), grid, blk, (size_t)wl.total, st, A, D,
                                 vl, ld, (TT*)t, stop, cntr, wl);
          else if (lb)
            hipLaunchKernelGGL((k_ilu_fwd<TM, TT, QQ, LDT, true>), grid, blk, lb, st, A, D, vl, ld, (TT*)t,
                               stop, cntr);
          else
            hipLaunchKernelGGL((k_ilu_fwd<TM, TT, QQ, LDT, false>), grid, blk, 0, st, A, D, vl, ld, (TT*)t,
                               stop, cntr);
          return hipGetLastError();
        };
        using Q = wider_t<TM, TT>;
        if (in.s) {
          if (in.type != T64 || !is_dbl<TT>::value) return hipErrorInvalidValue;
          return go(LdSBasis<TT, Q>{(const double*)in.raw, in.scale, in.s, in.cur, in.stride, 0.0}, (Q*)nullptr);
        }
        if (!in.scale) {
          if (in.type != tt) return hipErrorInvalidValue;
          return go(LdVec<TT, Q>{(const TT*)in.raw}, (Q*)nullptr);
        }
        return with_type(in.type, [&](auto pin) -> hipError_t {
          using TIN = TYPE_OF(pin);
          using QQ = wider_t<TIN, Q>;
          return go(LdBasis<TIN, TT, QQ>{(const TIN*)in.raw, in.scale, in.cur, in.stride, 0.0}, (QQ*)nullptr);
        });
      }
    });
  });
}

hipError_t ilu_apply_bwd(hipStream_t st, const SellDesc& A, const void* mv, int tm, void* t, int tt,
                         int mode, const double* omega, const void* zprev, void* out, int tout,
                         const double* s, int* fbflag, const int* stop, const int* cur) {
  if (mode != 3 && tout != tt) return hipErrorInvalidValue;
  const IluDesc D = *A.ilu;
  const dim3 g((unsigned)D.blocks), b(kIluThreads);
  const size_t lb = lds_bytes(A, D.blocks, tt, D.lds_max);
  if (!mv || tm < 0 || tm > 3 || !D.val_up[tm] || !D.diag_up[tm]) return hipErrorInvalidValue;
  const int rows_max = (int)((A.n + D.blocks - 1) / D.blocks + 1);
  return with_type(tm, [&](auto pm) {
    using TM = TYPE_OF(pm);
    const TM* vu = (const TM*)D.val_up[tm];
    const TM* du = (const TM*)D.diag_up[tm];
    return with_type(tt, [&](auto pt) -> hipError_t {
      using TT = TYPE_OF(pt);
      if constexpr (!ok_m<TM, TT>()) {
        return hipErrorInvalidValue;
      } else {
        using Q = wider_t<TM, TT>;
        const WinLds wl = win_lds(rows_max, (int)sizeof(TT), (int)sizeof(TM), D.win_pos, D.win_ent);
        const bool win = D.win && wl.total <= D.lds_max;
        if (D.used) *D.used |= win ? 1 : (lb ? 2 : 4);
        auto go = [&](auto ep) -> hipError_t {
          using EPI = decltype(ep);
          if (win) {
            if (D.chunk)
              hipLaunchKernelGGL((k_ilu_bwd_win<TM, TT, Q, true>), g, b, (size_t)wl.total, st, A, D, vu, du,
                                 (TT*)t, stop, wl);
            else
              hipLaunchKernelGGL((k_ilu_bwd_win<TM, TT, Q, false>), g, b, (size_t)wl.total, st, A, D, vu, du,
                                 (TT*)t, stop, wl);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
            const unsigned ge = (unsigned)((A.n + 1023) / 1024);
            hipLaunchKernelGGL((k_ilu_epi<TT, EPI>), dim3(ge), dim3(256), 0, st, A, (const TT*)t, ep, stop);
          } else if (lb) {
            hipLaunchKernelGGL((k_ilu_bwd<TM, TT, Q, EPI, true>), g, b, lb, st, A, D, vu, du, (TT*)t, ep, stop);
          } else {
            hipLaunchKernelGGL((k_ilu_bwd<TM, TT, Q, EPI, false>), g, b, 0, st, A, D, vu, du, (TT*)t, ep, stop);
          }
          return hipGetLastError();
        };
        if (mode == 0) return go(EpiStore<TT, Q>{(TT*)out, fbflag});
        if (mode == 1) return go(EpiZ1<TT, Q>{(TT*)out, omega, fbflag, (Q)0});
        if (mode == 2) return go(EpiZK<TT, Q>{(TT*)out, (const TT*)zprev, omega, fbflag, (Q)0});
        if constexpr (!is_dbl<TT>::value) {
          return hipErrorInvalidValue;
        } else {
          return go(EpiS64{(double*)out, s, fbflag, cur, A.n});
        }
      }
    });
  });
}

}  // namespace f3r
