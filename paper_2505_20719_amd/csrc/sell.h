// SELL-64 row machinery shared by the per-kernel path and the persistent
// batch kernel: the lane/row slots of a wave, the unconditional-load row
// sums and the vector loaders that convert between level precisions.
#pragma once
#include <type_traits>

#include "common.h"
#include "kernels.h"

namespace f3r {

// ---- several systems in one descriptor --------------------------------------
// system of the rows starting at row0 (a block never spans two systems)
__device__ __forceinline__ int sys_of(const SysLayout& s, int64_t row0) {
  return s.blk ? s.blk[row0 >> 10] : 0;
}
template <class T> __device__ __forceinline__ T* sys_ptr(T* p, int sy, int64_t d) {
  return p ? p + (int64_t)sy * d : p;
}
// partial-sum range [lo, hi) of system sy among nb block partials
__device__ __forceinline__ void sys_range(const SysLayout& s, int sy, int64_t nb, int64_t& lo,
                                          int64_t& hi) {
  lo = s.b0 ? s.b0[sy] : 0;
  hi = s.b0 ? s.b0[sy + 1] : nb;
}

template <class T> struct is_dbl : std::is_same<T, double> {};
template <class A, class B, class C = float> using wider_t =
    typename std::conditional<is_dbl<A>::value || is_dbl<B>::value || is_dbl<C>::value, double, float>::type;

// Column of an entry from what the format stores for it: a 16-bit offset
// from the row, a 32-bit column, or (slice-offset format) a 32-bit offset
// shared by the 64 rows of a slice.  A shared offset can point outside the
// matrix for a row that has no entry there (its value is zero); such a
// column is replaced by the row's own.
struct SOff {
  int32_t d;
};
template <class TI> __device__ __forceinline__ int64_t col_of(TI d, int64_t row, int64_t n);
template <> __device__ __forceinline__ int64_t col_of<int16_t>(int16_t d, int64_t row, int64_t) {
  return row + d;
}
template <> __device__ __forceinline__ int64_t col_of<int32_t>(int32_t d, int64_t, int64_t) { return d; }
template <> __device__ __forceinline__ int64_t col_of<SOff>(SOff d, int64_t row, int64_t n) {
  const int64_t c = row + d.d;
  return (uint64_t)c < (uint64_t)n ? c : row;
}

// What the format stores for position k of the row whose first element is
// e0 (e0 = slice base + lane; the slice-offset table has one row of the
// common width per slice, at e0 / 64).  idx_wave: the position is the same
// for every row of the slice, so the table read is one wave-uniform load.
template <class TI> __device__ __forceinline__ TI idx_lane(const TI* idx, uint32_t e0, int k) {
  return idx[e0 + (uint32_t)k * 64];
}
template <> __device__ __forceinline__ SOff idx_lane<SOff>(const SOff* idx, uint32_t e0, int k) {
  return idx[(e0 >> 6) + (uint32_t)k];
}
template <class TI> __device__ __forceinline__ TI idx_wave(const TI* idx, uint32_t e0, int k) {
  return idx_lane<TI>(idx, e0, k);
}
template <> __device__ __forceinline__ SOff idx_wave<SOff>(const SOff* idx, uint32_t e0, int k) {
  // every lane of a real row computes the same position; a missing row's
  // own position is also inside the table, so any lane's value is safe
  const uint32_t j = (uint32_t)__builtin_amdgcn_readfirstlane((int)((e0 >> 6) + (uint32_t)k));
  return idx[j];
}

// The KR rows of one lane: row index, first element of the row in the SELL
// arrays, slice width, and whether the row exists.  A missing row (past n or
// past the last slice) is pointed at entry 0 of row 0 so that every load it
// takes part in stays inside the arrays; its sums are never used.  In the
// diagonal-aligned format the position and width follow from the slice
// index, so no offset load precedes the entry loads.
struct RowSlot {
  int64_t row;
  int64_t n;
  uint32_t e0;
  int w;
  bool ok;
};

// gw (the wave's group of KR slices) is wave-uniform, so the offsets are
// scalar loads, issued together.
template <int KR>
__device__ __forceinline__ void make_slots(const SellDesc& A, int64_t gw, int lane,
                                           RowSlot (&s)[KR]) {
  uint32_t o0[KR];
  int w[KR];
  if (A.dell_w > 0) {
#pragma unroll
    for (int r = 0; r < KR; r++) {
      const int64_t slice = gw * KR + r;
      const int64_t sl = slice < A.ns ? slice : 0;
      o0[r] = (uint32_t)(sl * kWave * A.dell_w);
      w[r] = A.dell_w;
    }
  } else {
#pragma unroll
    for (int r = 0; r < KR; r++) {
      const int64_t slice = gw * KR + r;
      const int64_t sl = slice < A.ns ? slice : 0;
      o0[r] = A.off[sl];
      w[r] = (int)((A.off[sl + 1] - o0[r]) / kWave);
    }
  }
#pragma unroll
  for (int r = 0; r < KR; r++) {
    const int64_t slice = gw * KR + r;
    const int64_t row = slice * kWave + lane;
    const bool ok = slice < A.ns && row < A.n;
    s[r].ok = ok;
    s[r].row = ok ? row : 0;
    s[r].n = A.n;
    s[r].e0 = ok ? o0[r] + (uint32_t)lane : 0u;
    s[r].w = ok ? w[r] : 0;
  }
}

// ---- range-checked gathers -------------------------------------------------
// A raw buffer resource over [p, p + bytes): a load at a byte offset at or
// past the end (a negative offset counts as a large unsigned one) returns
// zero and reads no memory.  Word 3 selects the 32-bit data format, with no
// swizzle and no thread-id addressing; the byte count must stay below 2^31.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_over(const void* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}
template <class T> __device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, uint32_t off);
template <> __device__ __forceinline__ f16 buf_load<f16>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(f16, __builtin_amdgcn_raw_buffer_load_b16(r, (int)off, 0, 0));
}
template <> __device__ __forceinline__ bf16 buf_load<bf16>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return bf16{__builtin_amdgcn_raw_buffer_load_b16(r, (int)off, 0, 0)};
}
template <> __device__ __forceinline__ float buf_load<float>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}
template <> __device__ __forceinline__ double buf_load<double>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}

// Row sums in the slice-offset format (the same sums as rows_sum below, in
// the same order).  Everything that locates an entry is uniform over the
// wave: the slice, the position k, the value row (the 64 values of position
// k are consecutive) and the column offset d_k from the table, so the value
// of a lane is a load at a wave-uniform address plus the lane, and its
// gather is the loader's range-checked load at byte offset (row + d_k) x
// the element size.  A column outside the vector reads zero (the entry's
// value is zero there: the row has no such entry).  The positions of a chunk
// are not clamped to the slice's range (the arrays are padded; the sums
// mask them), except in fp64 (below).  The ranges are the first lane's of
// the first slice: every
// existing row has the same ones in this format, and a missing row's sums
// are left as they were before the first entry, as with per-row ranges.
template <int U, bool NEG, class TV, class Q, class XF, int KR, class INIT>
__device__ __forceinline__ void rows_sum_slice(const TV* __restrict__ val, const SOff* __restrict__ idx,
                                               const RowSlot (&s)[KR], const int (&lo)[KR],
                                               const int (&hi)[KR], const int (&kb)[KR],
                                               const int (&ke)[KR], Q (&acc)[KR], const XF& x0,
                                               const INIT& init) {
  static_assert(U <= kSlicePad, "chunk longer than the padding");
  XF x = x0;
  x.bind(s[0].n);
  const uint32_t lane = threadIdx.x & (kWave - 1);
  // One set of ranges for all the lane's slices: they follow from the
  // format's common widths, the same for every slice (the first slice's are
  // taken; a missing slice, which can only follow it, keeps its sums as
  // they were and is never stored).
  const int ulo = __builtin_amdgcn_readfirstlane(lo[0]);
  const int ukb = __builtin_amdgcn_readfirstlane(kb[0]);
  const int uke = __builtin_amdgcn_readfirstlane(ke[0]);
  const int it = __builtin_amdgcn_readfirstlane(hi[0]) - ulo;
  // fp64 sums read a chunk's positions past the range as the range's last
  // one (cached), not the next positions: with 8-byte values the unsummed
  // reads of chunks of eight over 13 entries cost more than the clamp
  // (fp64-F3R on the 27-point matrices); narrower sums read them unclamped
  constexpr bool kClampChunk = std::is_same<Q, double>::value;
  const int last = max(it - 1, 0);
  const TV* vrow[KR];
  const int32_t* trow[KR];
  uint32_t xrow[KR];
#pragma unroll
  for (int r = 0; r < KR; r++) {
    // slice x width: the table row, and the value row of position 0
    const uint32_t sb = (uint32_t)__builtin_amdgcn_readfirstlane((int)(s[r].e0 >> 6));
    // from the first position of the range on; a chunk reads at a uniform
    // base plus constant position offsets
    vrow[r] = val + ((size_t)sb + (size_t)ulo) * kWave;
    trow[r] = (const int32_t*)idx + sb + ulo;
    xrow[r] = (uint32_t)s[r].row * XF::kBytes;
  }
  Q a0[KR];
  int i0 = 0;
  do {
    TV v[KR][U];
    int32_t d[KR][U];
#pragma unroll
    for (int r = 0; r < KR; r++) {
#pragma unroll
      for (int u = 0; u < U; u++) {
        if constexpr (kClampChunk) {
          const int kk = min(i0 + u, last);
          v[r][u] = (vrow[r] + (uint32_t)kk * kWave)[lane];
          d[r][u] = trow[r][kk];
        } else {
          v[r][u] = (vrow[r] + (uint32_t)i0 * kWave)[u * kWave + lane];
          d[r][u] = (trow[r] + i0)[u];
        }
      }
    }
    typename XF::raw_t xr[KR][U];
#pragma unroll
    for (int r = 0; r < KR; r++) {
#pragma unroll
      for (int u = 0; u < U; u++) xr[r][u] = x.raw_b(xrow[r] + (uint32_t)d[r][u] * XF::kBytes);
    }
    if (i0 == 0) x.pin();
    Q xv[KR][U];
#pragma unroll
    for (int r = 0; r < KR; r++) {
#pragma unroll
      for (int u = 0; u < U; u++) {
        xv[r][u] = x.cook(xr[r][u]);
        if constexpr (XF::kCostlyCook) {
          xv[r][u] = value_barrier(xv[r][u]);
          v[r][u] = value_barrier(v[r][u]);
        }
      }
    }
    if (i0 == 0) {
      init(acc);
#pragma unroll
      for (int r = 0; r < KR; r++) a0[r] = acc[r];
    }
    bool in[U];
#pragma unroll
    for (int u = 0; u < U; u++) in[u] = ulo + i0 + u >= ukb && ulo + i0 + u < uke;
#pragma unroll
    for (int r = 0; r < KR; r++) {
#pragma unroll
      for (int u = 0; u < U; u++) {
        const Q m = NEG ? -widen<Q>(v[r][u]) : widen<Q>(v[r][u]);
        const Q t = acc[r] + m * xv[r][u];
        acc[r] = in[u] ? t : acc[r];
      }
    }
    i0 += U;
  } while (i0 < it);
#pragma unroll
  for (int r = 0; r < KR; r++) acc[r] = s[r].ok ? acc[r] : a0[r];
}

// Row sums in SELL-64 and the diagonal-aligned format (16-bit offsets from
// the row or 32-bit columns per entry; the same sums as rows_sum below, in
// the same order), for fp32 arithmetic.  A slice's entries of position k
// are 64 consecutive elements at a wave-uniform address, so values and
// indices load at a uniform base plus the lane; the gather is the loader's
// range-checked load at byte offset column x element size.  Positions past a slice's width are
// read unclamped (the next slice's entries, or the zero padding after the
// last slice) and masked by the rows' own ranges, which also mask every
// position of a missing row.
template <class TI> __device__ __forceinline__ uint32_t sell_col(TI d, uint32_t row);
template <> __device__ __forceinline__ uint32_t sell_col<int16_t>(int16_t d, uint32_t row) {
  return row + (uint32_t)(int32_t)d;
}
template <> __device__ __forceinline__ uint32_t sell_col<int32_t>(int32_t d, uint32_t) { return (uint32_t)d; }

template <int U, bool NEG, class TI, class TV, class Q, class XF, int KR, class INIT>
__device__ __forceinline__ void rows_sum_sell(const TV* __restrict__ val, const TI* __restrict__ idx,
                                              const RowSlot (&s)[KR], const int (&lo)[KR],
                                              const int (&hi)[KR], const int (&kb)[KR],
                                              const int (&ke)[KR], Q (&acc)[KR], const XF& x0,
                                              const INIT& init) {
  static_assert(U <= kSlicePad, "chunk longer than the padding");
  XF x = x0;
  x.bind(s[0].n);
  const uint32_t lane = threadIdx.x & (kWave - 1);
  int ulo[KR];
  const TV* vrow[KR];
  const TI* irow[KR];
  uint32_t row[KR];
  int it = 0;
#pragma unroll
  for (int r = 0; r < KR; r++) {
    // slice range and first element: uniform over the slice (first lane's)
    ulo[r] = __builtin_amdgcn_readfirstlane(lo[r]);
    const int uhi = __builtin_amdgcn_readfirstlane(hi[r]);
    const uint32_t e0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)s[r].e0);
    vrow[r] = val + (size_t)e0 + (size_t)ulo[r] * kWave;
    irow[r] = idx + (size_t)e0 + (size_t)ulo[r] * kWave;
    row[r] = (uint32_t)s[r].row;
    it = max(it, uhi - ulo[r]);
  }
  int i0 = 0;
  do {
    TV v[KR][U];
    TI d[KR][U];
#pragma unroll
    for (int r = 0; r < KR; r++) {
#pragma unroll
      for (int u = 0; u < U; u++) {
        v[r][u] = (vrow[r] + (uint32_t)i0 * kWave)[u * kWave + lane];
        d[r][u] = (irow[r] + (uint32_t)i0 * kWave)[u * kWave + lane];
      }
    }
    typename XF::raw_t xr[KR][U];
#pragma unroll
    for (int r = 0; r < KR; r++) {
#pragma unroll
      for (int u = 0; u < U; u++) xr[r][u] = x.raw_b(sell_col<TI>(d[r][u], row[r]) * XF::kBytes);
    }
    if (i0 == 0) x.pin();
    Q xv[KR][U];
#pragma unroll
    for (int r = 0; r < KR; r++) {
#pragma unroll
      for (int u = 0; u < U; u++) {
        xv[r][u] = x.cook(xr[r][u]);
        if constexpr (XF::kCostlyCook) {
          xv[r][u] = value_barrier(xv[r][u]);
          v[r][u] = value_barrier(v[r][u]);
        }
      }
    }
    if (i0 == 0) init(acc);
#pragma unroll
    for (int r = 0; r < KR; r++) {
#pragma unroll
      for (int u = 0; u < U; u++) {
        const int k = ulo[r] + i0 + u;
        const Q m = NEG ? -widen<Q>(v[r][u]) : widen<Q>(v[r][u]);
        const Q t = acc[r] + m * xv[r][u];
        acc[r] = (k >= kb[r] && k < ke[r]) ? t : acc[r];
      }
    }
    i0 += U;
  } while (i0 < it);
}

// For each of the lane's rows, acc_r += sum over entries k in [kb_r, ke_r)
// of round(a_k x_{c_k}), left to right.  The loop runs over [lo_r, hi_r), a
// range that is uniform over the slice (so the loads never wait for per-row
// data) and contains [kb_r, ke_r).  Entries go in chunks of U: every value
// and index load of a chunk (all rows) is issued unconditionally, with k
// clamped into [0, hi_r) (entries the wave reads anyway), then every gather,
// then the sums, whose predicate is a select.  No load sits behind a branch,
// so a wave keeps KR x U entries in flight; the order of the sums of a row
// (and so its rounding) is that of the definition.
//
// init(acc), when given, sets the starting values of the sums inside the
// first iteration, after its loads are issued: a starting value computed
// before the loop makes the wave wait for its operands before the loop's
// first load (init must keep its arithmetic from being hoisted out of the
// loop; value_barrier does that).  The first iteration always runs (its
// clamped loads stay inside the arrays; its sums are masked when the range
// is empty).
struct NoInit {
  template <class A> __device__ __forceinline__ void operator()(A&) const {}
};
// loaders that split a load (raw) from its conversion (cook)
template <class T, class = void> struct has_raw : std::false_type {};
template <class T> struct has_raw<T, std::void_t<typename T::raw_t>> : std::true_type {};
template <int U, class TI, class TV, class Q, class XF, int KR, class INIT = NoInit>
__device__ __forceinline__ void rows_sum(const TV* __restrict__ val, const TI* __restrict__ idx,
                                         const RowSlot (&s)[KR], const int (&lo)[KR],
                                         const int (&hi)[KR], const int (&kb)[KR],
                                         const int (&ke)[KR], Q (&acc)[KR], const XF& x,
                                         bool neg = false, const INIT& init = INIT()) {
  if constexpr (std::is_same<TI, SOff>::value && has_raw<XF>::value) {
    if (neg)
      rows_sum_slice<U, true>(val, idx, s, lo, hi, kb, ke, acc, x, init);
    else
      rows_sum_slice<U, false>(val, idx, s, lo, hi, kb, ke, acc, x, init);
    return;
  } else if constexpr (has_raw<XF>::value && !std::is_same<Q, double>::value) {
    // (fp64 sums keep the per-lane path: with their wide values and gathers
    // the compiler serialised the loads of the uniform one to save
    // registers, 154 against 135 us for the 636 MB SpMV of the elasticity
    // matrix)
    if (neg)
      rows_sum_sell<U, true, TI>(val, idx, s, lo, hi, kb, ke, acc, x, init);
    else
      rows_sum_sell<U, false, TI>(val, idx, s, lo, hi, kb, ke, acc, x, init);
    return;
  }
  int it = 0;
#pragma unroll
  for (int r = 0; r < KR; r++) it = max(it, hi[r] - lo[r]);
  int i0 = 0;
  do {
    TV v[KR][U];
    TI d[KR][U];
#pragma unroll
    for (int r = 0; r < KR; r++) {
#pragma unroll
      for (int u = 0; u < U; u++) {
        const int k = max(min(lo[r] + i0 + u, hi[r] - 1), 0);
        v[r][u] = val[s[r].e0 + (uint32_t)k * 64];
        d[r][u] = idx_wave<TI>(idx, s[r].e0, k);
      }
    }
    Q xv[KR][U];
    if constexpr (has_raw<XF>::value) {
      // every gather issued before any conversion: a conversion may hold an
      // empty volatile asm (the fp32 rounding point), across which the
      // compiler does not move loads, and each gather would then wait for
      // the one before it
      typename XF::raw_t xr[KR][U];
#pragma unroll
      for (int r = 0; r < KR; r++) {
#pragma unroll
        for (int u = 0; u < U; u++) xr[r][u] = x.raw(col_of<TI>(d[r][u], s[r].row, s[r].n));
      }
#pragma unroll
      for (int r = 0; r < KR; r++) {
#pragma unroll
        for (int u = 0; u < U; u++) {
          xv[r][u] = x.cook(xr[r][u]);
          // a costly conversion (and the entry value) is made here for every
          // entry, so the compiler does not move it, with its load, into the
          // branch of the entries that count, where the wait for that load
          // would be left open at the end of the chunk
          if constexpr (XF::kCostlyCook) {
            xv[r][u] = value_barrier(xv[r][u]);
            v[r][u] = value_barrier(v[r][u]);
          }
        }
      }
    } else {
#pragma unroll
      for (int r = 0; r < KR; r++) {
#pragma unroll
        for (int u = 0; u < U; u++) xv[r][u] = x(col_of<TI>(d[r][u], s[r].row, s[r].n));
      }
    }
    if (i0 == 0) init(acc);
#pragma unroll
    for (int r = 0; r < KR; r++) {
#pragma unroll
      for (int u = 0; u < U; u++) {
        const int k = lo[r] + i0 + u;
        Q m = widen<Q>(v[r][u]);
        m = neg ? -m : m;
        const Q t = acc[r] + m * xv[r][u];
        acc[r] = (k >= kb[r] && k < ke[r]) ? t : acc[r];
      }
    }
    i0 += U;
  } while (i0 < it);
}

constexpr int kUnroll = 4;

// ---------------------------------------------------------------------------
// vector loaders (value of entry c as the consumer's arithmetic type Q)
// ---------------------------------------------------------------------------
// raw(c) loads what entry c needs and cook(raw) converts it; a kernel that
// uses the row's own value after its sums loads it with raw() first and
// converts it at the end, so nothing waits for it before the entry loads.
//
// bind(n) / raw_b(byte offset): the same loads through a range-checked
// buffer over the n entries of the vector (the slice-offset gathers).
template <class TT, class Q> struct LdVec {
  using raw_t = TT;
  static constexpr bool kCostlyCook = false;
  static constexpr uint32_t kBytes = sizeof(TT);
  const TT* p;
  uint32_t nb;
  __device__ __forceinline__ void at_sys(int, const SysLayout&) {}
  __device__ __forceinline__ void init() {}
  __device__ __forceinline__ void bind(int64_t n) { nb = (uint32_t)(n * kBytes); }
  __device__ __forceinline__ raw_t raw_b(uint32_t off) const { return buf_load<TT>(buf_over(p, nb), off); }
  __device__ __forceinline__ void pin() {}
  __device__ __forceinline__ raw_t raw(int64_t c) const { return p[c]; }
  __device__ __forceinline__ Q cook(raw_t v) const { return widen<Q>(v); }
  __device__ __forceinline__ Q operator()(int64_t c) const { return widen<Q>(p[c]); }
};

// round_to<TT>(raw_c * sc) with the product rounded to Q.  The scale is a Q
// value (a level with vectors no wider than fp32 computes in fp32, so its
// scales are fp32 values), kept as the double it is stored as.  For fp32
// consumers the product is the fp32 product of the raw value and the scale
// converted once at init; for fp64 ones it is formed in fp64.
template <class TIN, class TT, class Q> struct LdBasis {
  using raw_t = TIN;
  // fp32 consumers (with a rounding to a narrower storage type, an fp32
  // rounding point first); measured: the fp64 levels run best without
  static constexpr bool kCostlyCook = !std::is_same<Q, double>::value;
  static constexpr uint32_t kBytes = sizeof(TIN);
  const TIN* p;
  const double* scp;
  const int* cur;
  int64_t stride;
  double sc;
  uint32_t nb;
  // after init (which selects the basis vector)
  __device__ __forceinline__ void bind(int64_t n) { nb = (uint32_t)(n * kBytes); }
  __device__ __forceinline__ raw_t raw_b(uint32_t off) const { return buf_load<TIN>(buf_over(p, nb), off); }
  // the scale and basis index of system sy
  __device__ __forceinline__ void at_sys(int sy, const SysLayout& sl) {
    scp = sys_ptr(scp, sy, sl.dS);
    cur = sys_ptr(cur, sy, sl.dI);
  }
  __device__ __forceinline__ void init() {
    // the same index for every lane: kept wave-uniform, so the vector's
    // address (and a buffer over it) is too
    int64_t j = cur ? __builtin_amdgcn_readfirstlane(vload(cur)) : 0;
    p += j * stride;
    sc = vload(scp + j);
  }
  // the scale as loaded here, after the chunk's loads: its conversion for
  // the cooks cannot be hoisted ahead of them (and wait for the scale)
  __device__ __forceinline__ void pin() { sc = value_barrier(sc); }
  __device__ __forceinline__ raw_t raw(int64_t c) const { return p[c]; }
  __device__ __forceinline__ Q cook(raw_t r) const {
    if constexpr (std::is_same<Q, float>::value) {
      // the exact product of two fp32 values fits in fp64, so rounding it
      // to fp32 once is the fp32 product
      const float v = widen<float>(r) * (float)sc;  // exact conversion: an fp32 value
      return widen<Q>(round_to<TT>(v));
    } else {
      const Q v = (Q)(widen<double>(r) * sc);
      return widen<Q>(round_to<TT>(v));
    }
  }
  __device__ __forceinline__ Q operator()(int64_t c) const { return cook(p[c]); }
};

// round_to<TT>(s_c * (raw_c * sc)) with fp64 products (outermost -> scaled
// inner system, P(v) = S F(S v))
struct SRaw {
  double v, s;
};
template <class TT, class Q> struct LdSBasis {
  using raw_t = SRaw;
  static constexpr bool kCostlyCook = false;
  static constexpr uint32_t kBytes = 8;
  const double* p;
  const double* scp;
  const double* s;
  const int* cur;
  int64_t stride;
  double sc;
  uint32_t nb;
  __device__ __forceinline__ void bind(int64_t n) { nb = (uint32_t)(n * kBytes); }
  __device__ __forceinline__ raw_t raw_b(uint32_t off) const {
    return SRaw{buf_load<double>(buf_over(p, nb), off), buf_load<double>(buf_over(s, nb), off)};
  }
  __device__ __forceinline__ void at_sys(int sy, const SysLayout& sl) {
    scp = sys_ptr(scp, sy, sl.dS);
    cur = sys_ptr(cur, sy, sl.dI);
  }
  __device__ __forceinline__ void init() {
    int64_t j = cur ? __builtin_amdgcn_readfirstlane(vload(cur)) : 0;
    p += j * stride;
    sc = vload(scp + j);
  }
  __device__ __forceinline__ void pin() { sc = value_barrier(sc); }
  __device__ __forceinline__ raw_t raw(int64_t c) const { return SRaw{p[c], s[c]}; }
  __device__ __forceinline__ Q cook(raw_t r) const {
    double v = r.s * (r.v * sc);
    return widen<Q>(round_to<TT>(v));
  }
  __device__ __forceinline__ Q operator()(int64_t c) const { return cook(raw(c)); }
};

// j-th vector of a level basis (V_0 separate, V_j = vb + (j-1) n), used by
// the non-finite fallback
template <class TIN, class Q> struct LdLevelBasis {
  const TIN* v0;
  const TIN* vb;
  const double* scales;
  int64_t n;
  __device__ __forceinline__ Q get(int j, int64_t c) const {
    const TIN* V = j == 0 ? v0 : vb + (int64_t)(j - 1) * n;
    Q v = widen<Q>(V[c]) * (Q)scales[j];
    return widen<Q>(round_to<TIN>(v));
  }
};

// ---------------------------------------------------------------------------
// host-side type dispatch of the launchers
// ---------------------------------------------------------------------------
template <class F> static hipError_t with_type(int t, F&& f) {
  switch (t) {
    case T64: return f((double*)nullptr);
    case T32: return f((float*)nullptr);
    case T16: return f((f16*)nullptr);
    case TB16: return f((bf16*)nullptr);
  }
  return hipErrorInvalidValue;
}
// idx16: 0 = 32-bit columns, 1 = 16-bit offsets, 2 = offsets per slice
template <class F> static hipError_t with_idx(int idx16, F&& f) {
  if (idx16 == 2) return f((SOff*)nullptr);
  return idx16 ? f((int16_t*)nullptr) : f((int32_t*)nullptr);
}
#define TYPE_OF(p) typename std::remove_pointer<decltype(p)>::type

template <class TM, class TT> constexpr bool ok_m() {
  // M stored no wider than the vectors it is applied to
  if (is_dbl<TT>::value) return true;
  if (std::is_same<TT, float>::value) return !is_dbl<TM>::value;
  return std::is_same<TM, TT>::value;
}

// ---------------------------------------------------------------------------
// Epilogues of the G sweep.  prefetch(k, row) issues the row-local loads of
// lane slot k before the row sums so they overlap the matrix loads.
template <class TT, class Q> struct EpiStore {
  TT* out;
  int* fb;
  __device__ __forceinline__ void at_sys(int sy, const SysLayout& sl) { fb = sys_ptr(fb, sy, sl.dI); }
  __device__ __forceinline__ void init() {}
  __device__ __forceinline__ void prefetch(int, int64_t) {}
  __device__ __forceinline__ void operator()(int, int64_t r, TT y) const {
    out[r] = y;
    if (fb && !finite_val(y)) atomicOr(fb, 1);
  }
};
template <class TT, class Q> struct EpiZ1 {
  TT* out;
  const double* wp;
  int* fb;
  Q w;
  __device__ __forceinline__ void at_sys(int sy, const SysLayout& sl) {
    wp = sys_ptr(wp, sy, sl.dS);
    fb = sys_ptr(fb, sy, sl.dI);
  }
  __device__ __forceinline__ void init() { w = (Q)vload(wp); }
  __device__ __forceinline__ void prefetch(int, int64_t) {}
  __device__ __forceinline__ void operator()(int, int64_t r, TT y) const {
    const TT z = round_to<TT>(w * widen<Q>(y));
    out[r] = z;
    if (fb && !finite_val(z)) atomicOr(fb, 1);
  }
};
template <class TT, class Q> struct EpiZK {
  TT* out;
  const TT* zp;
  const double* wp;
  int* fb;
  Q w;
  TT zv[4];  // one per row of the lane (at most four), converted when used
  __device__ __forceinline__ void at_sys(int sy, const SysLayout& sl) {
    wp = sys_ptr(wp, sy, sl.dS);
    fb = sys_ptr(fb, sy, sl.dI);
  }
  __device__ __forceinline__ void init() { w = (Q)vload(wp); }
  __device__ __forceinline__ void prefetch(int k, int64_t r) { zv[k] = zp[r]; }
  __device__ __forceinline__ void operator()(int k, int64_t r, TT y) const {
    const TT z = round_to<TT>(widen<Q>(zv[k]) + w * widen<Q>(y));
    out[r] = z;
    if (fb && !finite_val(z)) atomicOr(fb, 1);
  }
};
struct EpiS64 {
  double* out;
  const double* s;
  int* fb;
  const int* cur;
  int64_t n;
  __device__ __forceinline__ void at_sys(int sy, const SysLayout& sl) {
    fb = sys_ptr(fb, sy, sl.dI);
    cur = sys_ptr(cur, sy, sl.dI);
  }
  __device__ __forceinline__ void init() {
    if (cur) {
      out += (int64_t)(*cur) * n;
      if (fb) fb += *cur;
    }
  }
  __device__ __forceinline__ void prefetch(int, int64_t) {}
  __device__ __forceinline__ void operator()(int, int64_t r, double y) const {
    const double z = s[r] * y;
    out[r] = z;
    if (fb && !isfinite(z)) atomicOr(fb, 1);
  }
};


}  // namespace f3r
