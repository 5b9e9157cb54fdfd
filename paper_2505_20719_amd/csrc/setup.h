// Set-up kernels of libf3r: CSR validation, symmetric diagonal scaling
// (Sec. 5), per-level value copies rounded directly from fp64 (Table 1), the
// two factors of the primary preconditioner (Sec. 5.2) and the conversion
// to the SELL-64 device format.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace f3r {

enum SetupFlags {
  SF_MATRIX = 1,    // unsorted/duplicate/out-of-range column, missing or zero diagonal, non-finite
  SF_IDX32 = 2,     // some |col - row| does not fit in int16
  SF_LONGROW = 4,   // a row has more than 65535 entries
  SF_RANGE = 8,     // a narrow copy that is used overflowed (inf)
  SF_ILU_NOWIN = 16,  // an ILU level exceeds an LDS window (not an error)
};

// Per row: checks, kd = position of the diagonal, len = row length,
// s_i = 1 / sqrt(|a_ii|).  Errors are OR-ed into *flags.
hipError_t row_check(hipStream_t st, int64_t n, const int32_t* rp, const int32_t* ci,
                     const double* val, double* s, uint16_t* kd, int32_t* len, int* flags);

// width[s] = max row length, kdr[s] = min | max << 16 of the diagonal
// positions, upm[s] = max count of entries right of the diagonal, over the
// rows of slice s
hipError_t slice_widths(hipStream_t st, int64_t n, const int32_t* len, const uint16_t* kd,
                        uint32_t* width, uint32_t* kdr, uint32_t* upm);

// kd[i] = v for every row (diagonal-aligned format)
hipError_t fill_kd(hipStream_t st, int64_t n, uint16_t* kd, int v);

// Slice-offset format: per slice, the sorted union of the rows' column
// offsets c - i (c != i), at most kSliceUnion of them (uni: ns x
// kSliceUnion), with luc[s] = below | above << 16 (0xFFFFFFFF: too many);
// then the table (ns x w, int32) with the diagonal at position kdp.
constexpr int kSliceUnion = 64;
hipError_t slice_union(hipStream_t st, int64_t n, const int32_t* rp, const int32_t* ci, int32_t* uni,
                       uint32_t* luc);
hipError_t slice_table(hipStream_t st, int64_t ns, const int32_t* uni, const uint32_t* luc, int w, int kdp,
                       int32_t* tab);

struct SellOut {
  void* idx = nullptr;          // int16 offsets or int32 columns (null with soff)
  int idx16 = 1;
  const int32_t* soff = nullptr;  // slice-offset format: the table (ns x width)
  double* a64 = nullptr;        // original values
  void* ah[4] = {};             // scaled values per precision tag (nullptr: not needed)
  void* mv[4] = {};             // M values per precision (lower part W, upper part G)
  double alpha = 1.0;
  int range_mask = 0;           // precision tags (bit t) whose overflow is an error
  int ilu_blocks = 0;           // > 0: M values are the shifted in-block matrix (ILU input)
};

// Scatters every row into the SELL-64 arrays (padding included) and
// computes ahat = (s_i a_ij) s_j, its rounded copies and the M values
// W_ij = -ahat_ij / alpha (j < i), G_ij = (-ahat_ij / alpha) / alpha (j > i).
// dkd >= 0: diagonal-aligned positions (entry j of row i at dkd - kd[i] + j);
// with o.soff, entry (i, c) sits where the slice's table holds c - i.
hipError_t to_sell(hipStream_t st, int64_t n, const int32_t* rp, const int32_t* ci,
                   const double* val, const double* s, const uint32_t* off, const int32_t* len,
                   const uint16_t* kd, int dkd, const SellOut& o, int* flags);

// gd = round_t(1 / alpha) for every precision tag, written to out[4]
hipError_t m_diag(hipStream_t st, double alpha, double* out);

// vals[k] (CSR order, fp64) = SELL value array of type t, for debugging;
// kdt/dkd as in to_sell (kdt = nullptr for the plain layout); ci and soff
// (the CSR columns and the table) for the slice-offset format, else null
hipError_t sell_to_csr_values(hipStream_t st, int64_t n, const int32_t* rp, const uint32_t* off,
                              const uint16_t* kdt, int dkd, const int32_t* ci, const int32_t* soff,
                              const void* v, int t, double* out);

}  // namespace f3r
