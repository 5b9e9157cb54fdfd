// Device-side helpers shared by every kernel of libf3r: storage types,
// round-to-nearest-even conversions, the XCD-aware block mapping and the
// deterministic wave/block reductions.
//
// The whole library is compiled with floating-point contraction off, so a
// product followed by a sum is two separately rounded operations, exactly as
// an IEEE implementation of the level arithmetic of Table 1 spells it.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace f3r {

typedef _Float16 f16;
struct bf16 {
  uint16_t u;
};

// ---- widening (exact) ------------------------------------------------------
__device__ __forceinline__ float bf16_to_float(bf16 x) { return __uint_as_float((uint32_t)x.u << 16); }

template <class Q> __device__ __forceinline__ Q widen(double x);
template <class Q> __device__ __forceinline__ Q widen(float x);
template <class Q> __device__ __forceinline__ Q widen(f16 x);
template <class Q> __device__ __forceinline__ Q widen(bf16 x);
template <> __device__ __forceinline__ double widen<double>(double x) { return x; }
template <> __device__ __forceinline__ double widen<double>(float x) { return (double)x; }
template <> __device__ __forceinline__ double widen<double>(f16 x) { return (double)(float)x; }
template <> __device__ __forceinline__ double widen<double>(bf16 x) { return (double)bf16_to_float(x); }
template <> __device__ __forceinline__ float widen<float>(double x) { return (float)x; }  // only for fp32-exact values
template <> __device__ __forceinline__ float widen<float>(float x) { return x; }
template <> __device__ __forceinline__ float widen<float>(f16 x) { return (float)x; }
template <> __device__ __forceinline__ float widen<float>(bf16 x) { return bf16_to_float(x); }

// ---- rounding to a storage type (RNE) -------------------------------------
__device__ __forceinline__ bf16 float_to_bf16(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return bf16{(uint16_t)((u >> 16) | 0x40u)};  // quiet NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return bf16{(uint16_t)(u >> 16)};
}

// fp64 -> fp32 with round-to-odd: truncate toward zero, then force the last
// bit to 1 when the truncation was inexact.  Followed by a round-to-nearest-
// even to a format with at most 22 significand bits it gives the correctly
// rounded result of the direct conversion (24 >= p + 2 for p = 11 and 8).
__device__ __forceinline__ float f64_to_f32_odd(double x) {
  float f = (float)x;  // RNE
  if (fabs((double)f) > fabs(x)) f = __uint_as_float(__float_as_uint(f) - 1u);  // step toward zero
  if ((double)f != x && !isnan(x)) f = __uint_as_float(__float_as_uint(f) | 1u);
  return f;
}

// An fp32 value that the compiler must materialise as such.  Without it the
// compiler folds "fp32 product, then convert to fp16" into one mixed
// multiply-add that rounds the exact product straight to fp16, which is not
// the fp32-arithmetic-then-store rounding the levels are defined with.
__device__ __forceinline__ float fp32_value(float x) {
  asm volatile("" : "+v"(x));
  return x;
}

template <class T> __device__ __forceinline__ T round_to(float x);
template <class T> __device__ __forceinline__ T round_to(double x);
template <> __device__ __forceinline__ float round_to<float>(float x) { return x; }
template <> __device__ __forceinline__ f16 round_to<f16>(float x) { return (f16)fp32_value(x); }
template <> __device__ __forceinline__ bf16 round_to<bf16>(float x) { return float_to_bf16(x); }
template <> __device__ __forceinline__ double round_to<double>(float x) { return (double)x; }
template <> __device__ __forceinline__ double round_to<double>(double x) { return x; }
template <> __device__ __forceinline__ float round_to<float>(double x) { return (float)x; }
template <> __device__ __forceinline__ f16 round_to<f16>(double x) { return (f16)f64_to_f32_odd(x); }
template <> __device__ __forceinline__ bf16 round_to<bf16>(double x) { return float_to_bf16(f64_to_f32_odd(x)); }

template <class T> __device__ __forceinline__ bool finite_val(T x);
template <> __device__ __forceinline__ bool finite_val<double>(double x) { return isfinite(x); }
template <> __device__ __forceinline__ bool finite_val<float>(float x) { return isfinite(x); }
template <> __device__ __forceinline__ bool finite_val<f16>(f16 x) { return isfinite((float)x); }
template <> __device__ __forceinline__ bool finite_val<bf16>(bf16 x) { return isfinite(bf16_to_float(x)); }

// A value the compiler must treat as produced at this point (an empty
// volatile asm that may change it): arithmetic on it cannot move above.
template <class T> __device__ __forceinline__ T value_barrier(T x) {
  asm volatile("" : "+v"(x));
  return x;
}

// ---- launch geometry -------------------------------------------------------
// Rows are processed in slices of 64 (one row per lane of a wave64).  Each
// wave takes kR consecutive slices, so a lane owns kR rows and issues the
// loads of all of them together (a single slice per wave leaves the waves
// too short to keep enough bytes in flight); a 256-thread block covers
// 4 kR slices = kRowsPerBlock rows.  Row-parallel kernels without a matrix
// give each thread kR rows of the same block range.  Blocks are dispatched
// round-robin over the 8 XCDs; logical block b is placed on XCD b / per, so
// every row-parallel kernel touches the same rows on the same XCD and that
// XCD's L2 keeps the vectors the previous kernel wrote.
constexpr int kWave = 64;
constexpr int kBlock = 256;
constexpr int kR = 4;
constexpr int kRowsPerBlock = kBlock * kR;
constexpr int kXcd = 8;
// Positions read past a slice's last one by a chunk of the slice-offset
// sums: the value arrays and the offset table of that format carry this
// many positions of padding (zeros) after the last slice, so a chunk of up
// to 8 positions is read without clamping.
constexpr int kSlicePad = 8;

// index of the calling wave in its block, as a wave-uniform (scalar) value
__device__ __forceinline__ int wave_index() {
  return __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
}

// A load of a device-resident scalar (flag, weight, scale) that stays a
// vector load: its index is a per-lane zero the compiler cannot see through.
// Scalar loads complete out of order, so the wave would wait for such a
// value as soon as it waits for any scalar operand of its first entry loads;
// vector loads complete in order and are waited for where they are used.
template <class T> __device__ __forceinline__ T vload(const T* p) {
  int z;
  asm("v_mov_b32 %0, 0" : "=v"(z));
  return p[z];
}

// A flag that is never set: a kernel given no flag reads this one, so every
// flag is read with an unconditional load (a branch around the load would
// make the wave wait at the branch).
static __device__ int kNoFlag;
__device__ __forceinline__ int read_flag(const int* p) { return vload(p ? p : &kNoFlag); }

__device__ __forceinline__ int64_t logical_block(int64_t nb) {
  int64_t per = (nb + kXcd - 1) / kXcd;
  int64_t b = blockIdx.x;
  return (b % kXcd) * per + b / kXcd;
}
inline int64_t physical_grid(int64_t nb) { return ((nb + kXcd - 1) / kXcd) * kXcd; }

// ---- deterministic reductions ---------------------------------------------
template <class T> __device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v = v + __shfl_xor(v, o, kWave);
  return v;
}

// Sum of one value per thread over a 256-thread block, fixed order.  The
// result is valid in thread 0.  `lds` needs kBlock / kWave entries.
template <class T> __device__ __forceinline__ T block_sum(T v, T* lds) {
  v = wave_sum(v);
  int w = threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0) lds[w] = v;
  __syncthreads();
  T s = 0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < kBlock / kWave; i++) s = s + lds[i];
  }
  __syncthreads();
  return s;
}

// One-block reductions of per-block partials use kFinBlock threads; each
// thread sums the entries t, t + kFinBlock, ... in index order with eight
// loads in flight, then the block sums the threads in a fixed order.
constexpr int kFinBlock = 1024;

template <class Q> __device__ __forceinline__ Q thread_sum(const Q* __restrict__ p, int64_t cnt) {
  const int nt = kFinBlock;
  Q s = 0;
  int64_t i = threadIdx.x;
  for (; i + 7 * (int64_t)nt < cnt; i += 8 * (int64_t)nt) {
    Q v[8];
#pragma unroll
    for (int u = 0; u < 8; u++) v[u] = p[i + (int64_t)u * nt];
#pragma unroll
    for (int u = 0; u < 8; u++) s = s + v[u];
  }
  for (; i < cnt; i += nt) s = s + p[i];
  return s;
}

// thread_sum of four series at once, p + l stride for l = l0 .. l0 + 3
// (past nv - 1 the last one is read again and its sums are unused): each
// sum adds the thread's terms in index order, as thread_sum does, with the
// loads of four terms of every series in flight together
template <class Q>
__device__ __forceinline__ void thread_sums4(const Q* __restrict__ p, int64_t stride, int l0, int nv,
                                             int64_t cnt, Q (&s)[4]) {
  const int nt = kFinBlock;
#pragma unroll
  for (int u = 0; u < 4; u++) s[u] = 0;
  for (int64_t i = threadIdx.x; i < cnt; i += 4 * (int64_t)nt) {
    Q v[4][4];
#pragma unroll
    for (int u = 0; u < 4; u++) {
      const Q* P = p + (int64_t)min(l0 + u, nv - 1) * stride;
#pragma unroll
      for (int k = 0; k < 4; k++) v[u][k] = P[min(i + (int64_t)k * nt, cnt - 1)];
    }
#pragma unroll
    for (int u = 0; u < 4; u++) {
#pragma unroll
      for (int k = 0; k < 4; k++) s[u] = i + (int64_t)k * nt < cnt ? s[u] + v[u][k] : s[u];
    }
  }
}

// sum over a kFinBlock-thread block, valid in thread 0 (lds: 16 entries)
template <class T> __device__ __forceinline__ T fin_block_sum(T v, T* lds) {
  v = wave_sum(v);
  const int w = threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0) lds[w] = v;
  __syncthreads();
  T s = 0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < kFinBlock / kWave; i++) s = s + lds[i];
  }
  __syncthreads();
  return s;
}

}  // namespace f3r
