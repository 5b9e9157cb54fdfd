// Set-up kernels: one thread per row of the CSR input.
#include <algorithm>
#include <vector>

#include "common.h"
#include "host.h"
#include "ilu.h"
#include "kernels.h"
#include "setup.h"

namespace f3r {

__global__ void k_row_check(int64_t n, const int32_t* __restrict__ rp,
                            const int32_t* __restrict__ ci, const double* __restrict__ val,
                            double* __restrict__ s, uint16_t* __restrict__ kd,
                            int32_t* __restrict__ len, int* flags) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t lo = rp[i], hi = rp[i + 1];
  int bad = 0;
  if (hi < lo) {
    atomicOr(flags, SF_MATRIX);
    len[i] = 0;
    kd[i] = 0;
    s[i] = 0.0;
    return;
  }
  int64_t dpos = -1;
  double d = 0.0;
  int64_t far = 0;
  for (int64_t k = lo; k < hi; k++) {
    const int64_t c = ci[k];
    if (c < 0 || c >= n) bad |= SF_MATRIX;
    if (k > lo && c <= (int64_t)ci[k - 1]) bad |= SF_MATRIX;
    if (!isfinite(val[k])) bad |= SF_MATRIX;
    if (c == i) {
      dpos = k - lo;
      d = val[k];
    }
    const int64_t dd = c - i < 0 ? i - c : c - i;
    far = dd > far ? dd : far;
  }
  if (dpos < 0 || d == 0.0) bad |= SF_MATRIX;
  if (hi - lo > 65535) bad |= SF_LONGROW;
  if (far > 32767) bad |= SF_IDX32;
  if (bad) atomicOr(flags, bad);
  len[i] = (int32_t)(hi - lo);
  kd[i] = (uint16_t)(dpos < 0 ? 0 : dpos);
  s[i] = 1.0 / sqrt(fabs(d));
}

hipError_t row_check(hipStream_t st, int64_t n, const int32_t* rp, const int32_t* ci,
                     const double* val, double* s, uint16_t* kd, int32_t* len, int* flags) {
  hipLaunchKernelGGL(k_row_check, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, rp, ci, val,
                     s, kd, len, flags);
  return hipGetLastError();
}

__global__ void k_slice_widths(int64_t n, const int32_t* __restrict__ len,
                               const uint16_t* __restrict__ kd, uint32_t* __restrict__ w,
                               uint32_t* __restrict__ kdr, uint32_t* __restrict__ upm) {
  const int64_t sl = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (sl >= n_slices(n)) return;
  int32_t m = 0, u = 0;
  int kmax = 0, kmin = 65535;
  for (int64_t r = sl * 64; r < sl * 64 + 64 && r < n; r++) {
    m = len[r] > m ? len[r] : m;
    kmax = kd[r] > kmax ? kd[r] : kmax;
    kmin = kd[r] < kmin ? kd[r] : kmin;
    const int32_t up = len[r] - 1 - (int32_t)kd[r];
    u = up > u ? up : u;
  }
  w[sl] = (uint32_t)m;
  kdr[sl] = (uint32_t)kmin | ((uint32_t)kmax << 16);
  upm[sl] = (uint32_t)u;
}

hipError_t slice_widths(hipStream_t st, int64_t n, const int32_t* len, const uint16_t* kd,
                        uint32_t* width, uint32_t* kdr, uint32_t* upm) {
  const int64_t ns = n_slices(n);
  hipLaunchKernelGGL(k_slice_widths, dim3((unsigned)((ns + 255) / 256)), dim3(256), 0, st, n, len,
                     kd, width, kdr, upm);
  return hipGetLastError();
}

__global__ void k_fill_kd(int64_t n, uint16_t* __restrict__ kd, int v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) kd[i] = (uint16_t)v;
}

hipError_t fill_kd(hipStream_t st, int64_t n, uint16_t* kd, int v) {
  hipLaunchKernelGGL(k_fill_kd, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, kd, v);
  return hipGetLastError();
}

// The sorted union of the column offsets c - i (c != i) over the rows of
// slice sl, one thread per slice: uni[sl * kSliceUnion ...], lc | uc << 16
// (counts below and above the diagonal) in luc[sl], or 0xFFFFFFFF when the
// union has more than kSliceUnion offsets.
__global__ void k_slice_union(int64_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                              int32_t* __restrict__ uni, uint32_t* __restrict__ luc) {
  const int64_t sl = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (sl >= n_slices(n)) return;
  int32_t* u = uni + sl * kSliceUnion;
  int cnt = 0;
  for (int64_t r = sl * 64; r < sl * 64 + 64 && r < n; r++) {
    for (int64_t k = rp[r]; k < rp[r + 1]; k++) {
      const int32_t d = (int32_t)((int64_t)ci[k] - r);
      if (d == 0) continue;
      int pos = 0;
      while (pos < cnt && u[pos] < d) pos++;
      if (pos < cnt && u[pos] == d) continue;
      if (cnt == kSliceUnion) {
        luc[sl] = 0xFFFFFFFFu;
        return;
      }
      for (int q = cnt; q > pos; q--) u[q] = u[q - 1];
      u[pos] = d;
      cnt++;
    }
  }
  int lc = 0;
  while (lc < cnt && u[lc] < 0) lc++;
  luc[sl] = (uint32_t)lc | ((uint32_t)(cnt - lc) << 16);
}

hipError_t slice_union(hipStream_t st, int64_t n, const int32_t* rp, const int32_t* ci, int32_t* uni,
                       uint32_t* luc) {
  const int64_t ns = n_slices(n);
  hipLaunchKernelGGL(k_slice_union, dim3((unsigned)((ns + 127) / 128)), dim3(128), 0, st, n, rp, ci, uni,
                     luc);
  return hipGetLastError();
}

// Row sl of the slice-offset table (common width w, diagonal at kdp): the
// slice's lower offsets end at kdp - 1, its upper ones start at kdp + 1,
// every other position holds offset 0 (no entry).
__global__ void k_slice_table(int64_t ns, const int32_t* __restrict__ uni, const uint32_t* __restrict__ luc,
                              int w, int kdp, int32_t* __restrict__ tab) {
  const int64_t sl = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (sl >= ns) return;
  const int lc = (int)(luc[sl] & 0xFFFFu), uc = (int)(luc[sl] >> 16);
  const int32_t* u = uni + sl * kSliceUnion;
  int32_t* t = tab + sl * w;
  for (int p = 0; p < w; p++) t[p] = 0;
  for (int q = 0; q < lc; q++) t[kdp - lc + q] = u[q];
  for (int q = 0; q < uc; q++) t[kdp + 1 + q] = u[lc + q];
}

hipError_t slice_table(hipStream_t st, int64_t ns, const int32_t* uni, const uint32_t* luc, int w, int kdp,
                       int32_t* tab) {
  hipLaunchKernelGGL(k_slice_table, dim3((unsigned)((ns + 255) / 256)), dim3(256), 0, st, ns, uni, luc, w,
                     kdp, tab);
  return hipGetLastError();
}

template <class T> __device__ __forceinline__ void put(void* p, uint32_t e, double v, int tag,
                                                       int mask, int* bad) {
  if (!p) return;
  const T r = round_to<T>(v);
  ((T*)p)[e] = r;
  if ((mask >> tag) & 1)
    if (!finite_val(r)) *bad |= SF_RANGE;
}

__global__ void k_to_sell(int64_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                          const double* __restrict__ val, const double* __restrict__ s,
                          const uint32_t* __restrict__ off, const int32_t* __restrict__ len,
                          const uint16_t* __restrict__ kd, int dkd, SellOut o, int* flags) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t sl = i / 64;
  const int lane = (int)(i % 64);
  if (sl * 64 >= n) return;
  const uint32_t base = off[sl] + lane;
  const int w = (int)((off[sl + 1] - off[sl]) / 64);
  if (i >= n) {
    // lanes of the last slice past the last row: zero values and column 0,
    // so that every stored position holds defined, finite data (the ILU
    // finish pass and the format converters walk whole slices)
    for (int p = 0; p < w; p++) {
      const uint32_t e = base + (uint32_t)p * 64;
      if (o.soff) {
      } else if (o.idx16) {
        ((int16_t*)o.idx)[e] = 0;
      } else {
        ((int32_t*)o.idx)[e] = 0;
      }
      o.a64[e] = 0.0;
      for (int t = 0; t < 4; t++) {
        if (o.ah[t]) {
          if (t == T64) ((double*)o.ah[t])[e] = 0.0;
          else if (t == T32) ((float*)o.ah[t])[e] = 0.f;
          else ((uint16_t*)o.ah[t])[e] = 0;
        }
        if (o.mv[t]) {
          if (t == T64) ((double*)o.mv[t])[e] = 0.0;
          else if (t == T32) ((float*)o.mv[t])[e] = 0.f;
          else ((uint16_t*)o.mv[t])[e] = 0;
        }
      }
    }
    return;
  }
  const int64_t lo = rp[i];
  const int L = len[i];
  const double si = s[i];
  // position p holds CSR entry p - shift (padding outside [0, L)); with
  // offsets per slice, the entry whose column is i + soff[p] when the row
  // has one (the real offsets ascend with p, so one walk finds them all)
  const int shift = dkd >= 0 ? dkd - (int)kd[i] : 0;
  const int32_t* so = o.soff ? o.soff + sl * w : nullptr;
  int walk = 0;
  int bad = 0;
  for (int p = 0; p < w; p++) {
    const uint32_t e = base + (uint32_t)p * 64;
    int k = p - shift;
    if (so) {
      k = -1;
      if (so[p] != 0 || p == dkd) {
        const int64_t want = i + so[p];
        while (walk < L && ci[lo + walk] < want) walk++;
        if (walk < L && ci[lo + walk] == want) k = walk;
      }
    }
    int64_t c = i;
    double a = 0.0, ah = 0.0, mvv = 0.0;
    if (k >= 0 && k < L) {
      c = ci[lo + k];
      a = val[lo + k];
      ah = (si * a) * s[c];
      if (o.ilu_blocks > 0) {
        // block-Jacobi ILU(0) input: diagonal times alpha, couplings to other
        // row blocks dropped (block b holds rows [b n / B, (b + 1) n / B))
        const int64_t nb = o.ilu_blocks;
        int64_t b = (i * nb) / n;
        while (b + 1 <= nb && ((b + 1) * n) / nb <= i) b++;
        while (b > 0 && (b * n) / nb > i) b--;
        const int64_t r0 = (b * n) / nb, r1 = ((b + 1) * n) / nb;
        mvv = c == i ? o.alpha * ah : (c >= r0 && c < r1 ? ah : 0.0);
      } else {
        if (c < i) mvv = -ah / o.alpha;
        if (c > i) mvv = (-ah / o.alpha) / o.alpha;
      }
    }
    if (o.soff) {
      // no per-entry index
    } else if (o.idx16) {
      ((int16_t*)o.idx)[e] = (int16_t)(c - i);
    } else {
      ((int32_t*)o.idx)[e] = (int32_t)c;
    }
    o.a64[e] = a;
    put<double>(o.ah[T64], e, ah, T64, o.range_mask, &bad);
    put<float>(o.ah[T32], e, ah, T32, o.range_mask, &bad);
    put<f16>(o.ah[T16], e, ah, T16, o.range_mask, &bad);
    put<bf16>(o.ah[TB16], e, ah, TB16, o.range_mask, &bad);
    put<double>(o.mv[T64], e, mvv, T64, o.range_mask, &bad);
    put<float>(o.mv[T32], e, mvv, T32, o.range_mask, &bad);
    put<f16>(o.mv[T16], e, mvv, T16, o.range_mask, &bad);
    put<bf16>(o.mv[TB16], e, mvv, TB16, o.range_mask, &bad);
  }
  if (bad) atomicOr(flags, bad);
}

hipError_t to_sell(hipStream_t st, int64_t n, const int32_t* rp, const int32_t* ci,
                   const double* val, const double* s, const uint32_t* off, const int32_t* len,
                   const uint16_t* kd, int dkd, const SellOut& o, int* flags) {
  // whole slices: the lanes past row n - 1 clear their positions
  const int64_t rows = (n + 63) / 64 * 64;
  hipLaunchKernelGGL(k_to_sell, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, st, n, rp, ci, val, s,
                     off, len, kd, dkd, o, flags);
  return hipGetLastError();
}

__global__ void k_m_diag(double alpha, double* out) {
  if (threadIdx.x != 0) return;
  const double v = 1.0 / alpha;
  out[T64] = v;
  out[T32] = (double)round_to<float>(v);
  out[T16] = (double)(float)round_to<f16>(v);
  out[TB16] = (double)bf16_to_float(round_to<bf16>(v));
}

hipError_t m_diag(hipStream_t st, double alpha, double* out) {
  hipLaunchKernelGGL(k_m_diag, dim3(1), dim3(64), 0, st, alpha, out);
  return hipGetLastError();
}

template <class T>
__global__ void k_sell_to_csr(int64_t n, const int32_t* __restrict__ rp, const uint32_t* __restrict__ off,
                              const uint16_t* __restrict__ kdt, int dkd, const int32_t* __restrict__ ci,
                              const int32_t* __restrict__ soff, const T* __restrict__ v,
                              double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int shift = kdt ? dkd - (int)kdt[i] : 0;
  const int64_t sl = i / 64;
  const uint32_t base = off[sl] + (uint32_t)(i % 64);
  const int w = (int)((off[sl + 1] - off[sl]) / 64);
  for (int64_t k = rp[i]; k < rp[i + 1]; k++) {
    int p = (int)(k - rp[i]) + shift;
    if (soff) {
      const int64_t d = (int64_t)ci[k] - i;
      p = dkd;
      for (int q = 0; q < w && d != 0; q++)
        if (soff[sl * w + q] == d) p = q;
    }
    out[k] = widen<double>(v[base + (uint32_t)p * 64]);
  }
}

hipError_t sell_to_csr_values(hipStream_t st, int64_t n, const int32_t* rp, const uint32_t* off,
                              const uint16_t* kdt, int dkd, const int32_t* ci, const int32_t* soff,
                              const void* v, int t, double* out) {
  const dim3 g((unsigned)((n + 255) / 256)), b(256);
  switch (t) {
    case T64: hipLaunchKernelGGL(k_sell_to_csr<double>, g, b, 0, st, n, rp, off, kdt, dkd, ci, soff, (const double*)v, out); break;
    case T32: hipLaunchKernelGGL(k_sell_to_csr<float>, g, b, 0, st, n, rp, off, kdt, dkd, ci, soff, (const float*)v, out); break;
    case T16: hipLaunchKernelGGL(k_sell_to_csr<f16>, g, b, 0, st, n, rp, off, kdt, dkd, ci, soff, (const f16*)v, out); break;
    case TB16: hipLaunchKernelGGL(k_sell_to_csr<bf16>, g, b, 0, st, n, rp, off, kdt, dkd, ci, soff, (const bf16*)v, out); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// host driver of the set-up kernels
// ---------------------------------------------------------------------------
f3r_status build_matrix(hipStream_t st, const f3r_csr* A, const f3r_params* p, const bool need_in[4],
                        DevAllocs& al, MatrixDev& m, bool allow_slice) {
  if (!A || !A->row_ptr || !A->col_idx || !A->val || A->n <= 0 || A->nnz < A->n) return F3R_ERR_ARG;
  if (A->n >= ((int64_t)1 << 31) - 64 || A->nnz >= ((int64_t)1 << 31)) return F3R_ERR_ARG;
  if (A->row_ptr[0] != 0 || A->row_ptr[A->n] != A->nnz) return F3R_ERR_MATRIX;
  // every row range must lie inside [0, nnz] before a kernel walks it
  for (int64_t i = 0; i < A->n; i++)
    if (A->row_ptr[i + 1] < A->row_ptr[i]) return F3R_ERR_MATRIX;
  const int64_t n = A->n, nnz = A->nnz, ns = n_slices(n);
  m.n = n;
  m.nnz = nnz;
  int32_t* ci = (int32_t*)al.get((size_t)nnz * 4);
  double* val = (double*)al.get((size_t)nnz * 8);
  m.rp = (int32_t*)al.get((size_t)(n + 1) * 4);
  HIPCHK(hipMemcpyAsync(m.rp, A->row_ptr, (size_t)(n + 1) * 4, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(ci, A->col_idx, (size_t)nnz * 4, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(val, A->val, (size_t)nnz * 8, hipMemcpyHostToDevice, st));
  m.s = (double*)al.get((size_t)n * 8);
  uint16_t* kd = (uint16_t*)al.get((size_t)n * 2);
  int32_t* len = (int32_t*)al.get((size_t)n * 4);
  int* flags = (int*)al.get(sizeof(int));
  HIPCHK(hipMemsetAsync(flags, 0, sizeof(int), st));
  HIPCHK(row_check(st, n, m.rp, ci, val, m.s, kd, len, flags));
  uint32_t* wdev = (uint32_t*)al.get((size_t)ns * 4);
  uint32_t* kdr = (uint32_t*)al.get((size_t)ns * 4);
  uint32_t* upmd = (uint32_t*)al.get((size_t)ns * 4);
  HIPCHK(slice_widths(st, n, len, kd, wdev, kdr, upmd));
  int hflags = 0;
  HIPCHK(hipMemcpyAsync(&hflags, flags, sizeof(int), hipMemcpyDeviceToHost, st));
  std::vector<uint32_t> w((size_t)ns), off((size_t)ns + 1), kdrh((size_t)ns), upmh((size_t)ns);
  HIPCHK(hipMemcpyAsync(w.data(), wdev, (size_t)ns * 4, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(kdrh.data(), kdr, (size_t)ns * 4, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(upmh.data(), upmd, (size_t)ns * 4, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (hflags & SF_MATRIX) return F3R_ERR_MATRIX;
  if (hflags & SF_LONGROW) return F3R_ERR_ARG;
  uint64_t acc = 0;
  for (int64_t sidx = 0; sidx < ns; sidx++) {
    off[(size_t)sidx] = (uint32_t)acc;
    acc += (uint64_t)w[(size_t)sidx] * 64;
    if (acc >= 0xFFFFFFF0ull) return F3R_ERR_ARG;
  }
  off[(size_t)ns] = (uint32_t)acc;
  // the diagonal-aligned format: common width KD + 1 + UP over all rows
  uint32_t dkd = 0, dup = 0;
  for (int64_t sidx = 0; sidx < ns; sidx++) {
    dkd = std::max(dkd, kdrh[(size_t)sidx] >> 16);
    dup = std::max(dup, upmh[(size_t)sidx]);
  }
  const uint64_t dw = (uint64_t)dkd + 1 + dup;
  const uint64_t dacc = (uint64_t)ns * 64 * dw;
  const bool dfits = dacc < 0xFFFFFFF0ull;
  const bool ilu = p->m_kind == F3R_M_ILU;
  // the slice-offset format: union of each slice's column offsets (it has
  // no per-row pattern, which ILU(0) needs)
  const bool try_slice = (p->layout == F3R_LAYOUT_SLICE || (p->layout == F3R_LAYOUT_AUTO && allow_slice)) && !ilu;
  if (p->layout == F3R_LAYOUT_SLICE && (!allow_slice || ilu)) return F3R_ERR_ARG;
  int32_t* uni = nullptr;
  uint32_t* lucd = nullptr;
  uint64_t sw = 0, skd = 0, sacc = 0;
  bool sfits = false;
  if (try_slice) {
    uni = (int32_t*)al.get((size_t)ns * kSliceUnion * 4);
    lucd = (uint32_t*)al.get((size_t)ns * 4);
    HIPCHK(slice_union(st, n, m.rp, ci, uni, lucd));
    std::vector<uint32_t> luc((size_t)ns);
    HIPCHK(hipMemcpyAsync(luc.data(), lucd, (size_t)ns * 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    uint64_t lmax = 0, umax = 0;
    bool over = false;
    for (int64_t sidx = 0; sidx < ns; sidx++) {
      const uint32_t v = luc[(size_t)sidx];
      if (v == 0xFFFFFFFFu) {
        over = true;
        break;
      }
      lmax = std::max<uint64_t>(lmax, v & 0xFFFFu);
      umax = std::max<uint64_t>(umax, v >> 16);
    }
    skd = lmax;
    sw = lmax + 1 + umax;
    sacc = (uint64_t)ns * 64 * sw;
    // the gathers of this format go through range-checked buffers of at
    // most 2^31 - 1 bytes (an fp64 vector of n entries)
    sfits = !over && sacc + (uint64_t)kSlicePad * 64 < 0xFFFFFFF0ull && (uint64_t)n * 8 < 0x7FFFFFFFull;
  }
  bool diag = false, slice = false;
  if (p->layout == F3R_LAYOUT_DIAG) {
    if (!dfits) return F3R_ERR_ARG;
    diag = true;
  } else if (p->layout == F3R_LAYOUT_SLICE) {
    if (!sfits) return F3R_ERR_ARG;
    slice = true;
  } else if (p->layout == F3R_LAYOUT_AUTO) {
    diag = dfits && dacc * 100 <= acc * 103;
    // no index bytes: taken when it stores at most 25 % more entries than
    // the better of the other two (the fp64 level still moves fewer bytes)
    slice = sfits && sacc * 100 <= std::min(acc, diag ? dacc : acc) * 125;
    if (slice) diag = false;
  }
  if (slice) {
    for (int64_t sidx = 0; sidx <= ns; sidx++) off[(size_t)sidx] = (uint32_t)((uint64_t)sidx * 64 * sw);
    acc = sacc;
  } else if (diag) {
    for (int64_t sidx = 0; sidx <= ns; sidx++) off[(size_t)sidx] = (uint32_t)((uint64_t)sidx * 64 * dw);
    acc = dacc;
  }
  m.padded = (int64_t)acc;
  uint32_t* offd = (uint32_t*)al.get((size_t)(ns + 1) * 4);
  HIPCHK(hipMemcpyAsync(offd, off.data(), (size_t)(ns + 1) * 4, hipMemcpyHostToDevice, st));
  SellOut so;
  int32_t* stab = nullptr;
  // value and index arrays: the row sums read up to kSlicePad positions
  // past the last slice (zeros, never summed)
  const size_t vcount = (size_t)acc + (size_t)kSlicePad * 64;
  if (slice) {
    stab = (int32_t*)al.get(((size_t)ns * sw + kSlicePad) * 4);
    HIPCHK(hipMemsetAsync(stab + (size_t)ns * sw, 0, kSlicePad * 4, st));
    HIPCHK(slice_table(st, ns, uni, lucd, (int)sw, (int)skd, stab));
    so.soff = stab;
    so.idx16 = 2;
    so.idx = nullptr;
  } else {
    so.idx16 = (hflags & SF_IDX32) ? 0 : 1;
    so.idx = al.get(vcount * (so.idx16 ? 2 : 4));
    HIPCHK(hipMemsetAsync((char*)so.idx + (size_t)acc * (so.idx16 ? 2 : 4), 0,
                          (size_t)kSlicePad * 64 * (so.idx16 ? 2 : 4), st));
  }
  if (uni) al.release(uni);
  if (lucd) al.release(lucd);
  so.a64 = (double*)al.get(vcount * 8);
  so.alpha = p->alpha;
  if (ilu && (p->ilu_blocks < 1 || p->ilu_blocks > n)) return F3R_ERR_ARG;
  so.ilu_blocks = ilu ? p->ilu_blocks : 0;
  // M reads the matrix values when it is the alpha = 1 truncated inverse
  m.m_shared = p->alpha == 1.0 && !ilu;
  bool need[4] = {need_in[0], need_in[1], need_in[2], need_in[3]};
  int mask = 0;
  for (int d = 1; d < p->nlev; d++) {
    need[p->lev[d].prec_a] = true;
    mask |= 1 << p->lev[d].prec_a;
  }
  if (m.m_shared) {
    need[p->prec_m] = true;
    mask |= 1 << p->prec_m;
  } else {
    so.mv[p->prec_m] = al.get(vcount * type_size(p->prec_m));
    if (p->prec_m != T64) so.mv[T64] = al.get(vcount * 8);
    mask |= 1 << p->prec_m;
  }
  for (int t = 0; t < 4; t++)
    if (need[t]) so.ah[t] = al.get(vcount * type_size(t));
  {
    const size_t tail = (size_t)kSlicePad * 64;
    HIPCHK(hipMemsetAsync(so.a64 + acc, 0, tail * 8, st));
    for (int t = 0; t < 4; t++) {
      if (so.ah[t]) HIPCHK(hipMemsetAsync((char*)so.ah[t] + (size_t)acc * type_size(t), 0, tail * type_size(t), st));
      if (so.mv[t]) HIPCHK(hipMemsetAsync((char*)so.mv[t] + (size_t)acc * type_size(t), 0, tail * type_size(t), st));
    }
  }
  so.range_mask = mask;
  HIPCHK(to_sell(st, n, m.rp, ci, val, m.s, offd, len, kd, diag ? (int)dkd : (slice ? (int)skd : -1), so,
                 flags));
  uint16_t* kdk = kd;
  if (slice) {
    // every row's diagonal at the common position; the columns stay for
    // reading values back in CSR order
    kdk = (uint16_t*)al.get((size_t)n * 2);
    HIPCHK(fill_kd(st, n, kdk, (int)skd));
    std::fill(kdrh.begin(), kdrh.end(), (uint32_t)(skd | (skd << 16)));
    HIPCHK(hipMemcpyAsync(kdr, kdrh.data(), (size_t)ns * 4, hipMemcpyHostToDevice, st));
    m.ci = ci;
    m.A.dell_w = (int)sw;
    m.A.dell_kd = (int)skd;
  } else if (diag) {
    // the kernels see the common diagonal position; the true one is kept
    // for reading values back in CSR order
    kdk = (uint16_t*)al.get((size_t)n * 2);
    HIPCHK(fill_kd(st, n, kdk, (int)dkd));
    std::fill(kdrh.begin(), kdrh.end(), dkd | (dkd << 16));
    HIPCHK(hipMemcpyAsync(kdr, kdrh.data(), (size_t)ns * 4, hipMemcpyHostToDevice, st));
    m.kd_true = kd;
    m.A.dell_w = (int)dw;
    m.A.dell_kd = (int)dkd;
  }
  double* gd = (double*)al.get(4 * sizeof(double));
  HIPCHK(m_diag(st, p->alpha, gd));
  HIPCHK(hipMemcpyAsync(m.gd, gd, 4 * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(&hflags, flags, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (hflags & SF_RANGE) return F3R_ERR_RANGE;
  m.a64 = so.a64;
  for (int t = 0; t < 4; t++) {
    m.ah[t] = so.ah[t];
    m.mv[t] = so.mv[t];
  }
  m.A.n = n;
  m.A.ns = ns;
  m.A.off = offd;
  m.A.idx = slice ? (const void*)stab : so.idx;
  m.A.idx16 = so.idx16;
  m.A.kd = kdk;
  m.A.kdr = kdr;
  if (ilu) {
    // level schedules, then the factorisation in place of the fp64 M values
    // and their narrow copies
    IluBuild ib;
    ib.blocks = p->ilu_blocks;
    const int64_t lp = n + p->ilu_blocks + 1;
    ib.lev = (int*)al.get((size_t)n * sizeof(int));
    ib.rows_lo = (int*)al.get((size_t)n * sizeof(int));
    ib.rows_up = (int*)al.get((size_t)n * sizeof(int));
    ib.lptr_lo = (int*)al.get((size_t)lp * sizeof(int));
    ib.lptr_up = (int*)al.get((size_t)lp * sizeof(int));
    ib.nlev_lo = (int*)al.get((size_t)p->ilu_blocks * sizeof(int));
    ib.nlev_up = (int*)al.get((size_t)p->ilu_blocks * sizeof(int));
    HIPCHK(ilu_schedule(st, m.A, ib));
    void* narrow[4] = {nullptr, so.mv[T32], so.mv[T16], so.mv[TB16]};
    HIPCHK(ilu_factor(st, m.A, ib, so.mv[T64] ? (double*)so.mv[T64] : nullptr, narrow, flags));
    // the factors packed in sweep order for the triangular solves
    ib.ptr_lo = (int*)al.get((size_t)lp * sizeof(int));
    ib.ptr_up = (int*)al.get((size_t)lp * sizeof(int));
    ib.col_lo = (int*)al.get((size_t)nnz * sizeof(int));
    ib.col_up = (int*)al.get((size_t)nnz * sizeof(int));
    for (int t = 0; t < 4; t++) {
      if (!so.mv[t]) continue;
      ib.val_lo[t] = al.get((size_t)nnz * type_size(t));
      ib.val_up[t] = al.get((size_t)nnz * type_size(t));
      ib.diag_up[t] = al.get((size_t)n * type_size(t));
    }
    // LDS a workgroup may take (gfx950: 160 KB) sizes the sweep windows
    int dev = 0, lds_max = 65536, cus = 1;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    ilu_window_size(n, p->ilu_blocks, lds_max, cus, &ib.win_pos, &ib.win_ent);
    ib.wst_lo = (int*)al.get((size_t)lp * sizeof(int));
    ib.wst_up = (int*)al.get((size_t)lp * sizeof(int));
    ib.nwin_lo = (int*)al.get((size_t)p->ilu_blocks * sizeof(int));
    ib.nwin_up = (int*)al.get((size_t)p->ilu_blocks * sizeof(int));
    HIPCHK(ilu_pack(st, m.A, ib, m.rp, so.mv, flags));
    al.release(ib.lev);
    m.ilu.blocks = ib.blocks;
    m.ilu.rows_lo = ib.rows_lo;
    m.ilu.rows_up = ib.rows_up;
    m.ilu.lptr_lo = ib.lptr_lo;
    m.ilu.lptr_up = ib.lptr_up;
    m.ilu.nlev_lo = ib.nlev_lo;
    m.ilu.nlev_up = ib.nlev_up;
    m.ilu.ptr_lo = ib.ptr_lo;
    m.ilu.ptr_up = ib.ptr_up;
    m.ilu.col_lo = ib.col_lo;
    m.ilu.col_up = ib.col_up;
    m.ilu.wst_lo = ib.wst_lo;
    m.ilu.wst_up = ib.wst_up;
    m.ilu.nwin_lo = ib.nwin_lo;
    m.ilu.nwin_up = ib.nwin_up;
    for (int t = 0; t < 4; t++) {
      m.ilu.val_lo[t] = ib.val_lo[t];
      m.ilu.val_up[t] = ib.val_up[t];
      m.ilu.diag_up[t] = ib.diag_up[t];
    }
    HIPCHK(hipMemcpyAsync(&hflags, flags, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (hflags & SF_MATRIX) return F3R_ERR_MATRIX;
    if (hflags & SF_RANGE) return F3R_ERR_RANGE;
    m.ilu.win = !(hflags & SF_ILU_NOWIN);
    m.ilu.win_pos = ib.win_pos;
    m.ilu.win_ent = ib.win_ent;
    m.ilu.lds_max = lds_max;
    // more than four entries per sweep row on average, and at most four
    // workgroups per compute unit (the chunked loop needs the registers that
    // eight co-resident workgroups would not leave)
    m.ilu.chunk = nnz > 9 * n && (int64_t)p->ilu_blocks <= 4 * (int64_t)cus;
  }
  // the CSR copies are no longer needed (the slice-offset format keeps the
  // columns for reading values back)
  if (!slice) al.release(ci);
  al.release(val);
  al.release(len);
  al.release(wdev);
  al.release(upmd);
  al.release(flags);
  al.release(gd);
  return F3R_OK;
}

}  // namespace f3r
