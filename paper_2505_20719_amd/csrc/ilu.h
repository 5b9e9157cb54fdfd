// Block-Jacobi ILU(0) as the primary preconditioner (Sec. 5.1): the rows
// are split into `blocks` contiguous ranges, row r0(b) = b n / blocks; the
// couplings between ranges are dropped; each diagonal block of the scaled
// matrix, its diagonal multiplied by alpha, is factored as L U with the
// sparsity of A.  The factors live in M's value arrays, at the positions of
// the matrix entries in the device format (L strictly left of each row's
// diagonal with a unit diagonal implied, U on and right of it).
//
// Triangular solves and the factorisation run one workgroup per block,
// level by level: a row's level is one more than the largest level of the
// in-block rows it depends on, the rows of a level are independent, and a
// workgroup barrier separates the levels.  Rows are stored sorted by level
// per block (rows[r0 .. r1)), with level boundaries lptr[r0 + b + l].
// For the sweeps, each row's in-block factor entries are also packed in
// that order (position q of block b: entries ptr[r0 + b + q] ..
// ptr[r0 + b + q + 1], columns as offsets from r0, values per stored
// precision, U's diagonal at r0 + q), inside the block's own CSR range
// [rp[r0], rp[r1]); a level then reads its rows' entries with one
// dependent load instead of walking the device format.
//
// When the block's part of the vector fits in LDS, the sweeps run from LDS
// only: consecutive levels are grouped into windows of at most win_pos
// positions and win_ent entries, sized at set-up from the LDS a workgroup
// may take (window w of block b: levels
// wst[r0 + b + w] .. wst[r0 + b + w + 1]), each window's rows, entry
// offsets, entries and level bounds are copied to LDS by the whole
// workgroup, and its levels then read nothing from global memory.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace f3r {

constexpr int kIluThreads = 256;
// set-up: window capacities for a device whose workgroups may take
// lds_max bytes of LDS and that has cus compute units (the block vector in
// fp16 plus one window fit in each workgroup's share)
void ilu_window_size(int64_t n, int blocks, int lds_max, int cus, int* win_pos, int* win_ent);

struct IluDesc {
  int blocks = 0;
  const int* rows_lo = nullptr;  // forward sweep order (lower dependencies)
  const int* lptr_lo = nullptr;
  const int* nlev_lo = nullptr;  // levels per block
  const int* rows_up = nullptr;  // backward sweep order (upper dependencies)
  const int* lptr_up = nullptr;
  const int* nlev_up = nullptr;
  const int* ptr_lo = nullptr;   // packed entries (n + blocks + 1 each)
  const int* ptr_up = nullptr;
  const int* col_lo = nullptr;   // offsets from the block's first row
  const int* col_up = nullptr;
  const void* val_lo[4] = {};    // per precision tag held by M
  const void* val_up[4] = {};
  const void* diag_up[4] = {};   // u_ii at each backward position
  const int* wst_lo = nullptr;   // first level of each window, then the level count
  const int* wst_up = nullptr;
  const int* nwin_lo = nullptr;  // windows per block
  const int* nwin_up = nullptr;
  bool win = false;              // every level fits a window (host flag)
  int win_pos = 0, win_ent = 0;  // window capacities (positions, entries)
  int lds_max = 65536;           // LDS bytes a workgroup may take
  bool chunk = false;            // long rows: entries summed four at a time
  int* used = nullptr;           // host word: forms launched (1 windows, 2 LDS
                                 // vector, 4 global vector), or null
};

// Writable arrays of the schedule, filled at set-up.
struct IluBuild {
  int blocks = 0;
  int *lev = nullptr, *rows_lo = nullptr, *lptr_lo = nullptr, *nlev_lo = nullptr;
  int *rows_up = nullptr, *lptr_up = nullptr, *nlev_up = nullptr;
  int *ptr_lo = nullptr, *ptr_up = nullptr, *col_lo = nullptr, *col_up = nullptr;
  void* val_lo[4] = {};
  void* val_up[4] = {};
  void* diag_up[4] = {};
  int *wst_lo = nullptr, *wst_up = nullptr, *nwin_lo = nullptr, *nwin_up = nullptr;
  int win_pos = 0, win_ent = 0;
};

// level schedules of both sweeps (A's pattern, in-block couplings only)
hipError_t ilu_schedule(hipStream_t st, const SellDesc& A, const IluBuild& b);
// in-place ILU(0) of the fp64 values v64 (initial values: the shifted
// in-block matrix, zero across blocks), then rounded copies to each non-null
// narrow[t]; non-finite fp64 factors set SF_MATRIX, overflowing copies
// SF_RANGE in *flags
hipError_t ilu_factor(hipStream_t st, const SellDesc& A, const IluBuild& b, double* v64,
                      void* const narrow[4], int* flags);
// packs the factors (M's value arrays mv[t], device format) for the sweeps
// and groups the levels into LDS windows; rp: CSR row pointers of A
// (bounds of each block's packed range); sets SF_ILU_NOWIN in *flags when a
// level does not fit a window
hipError_t ilu_pack(hipStream_t st, const SellDesc& A, const IluBuild& b, const int32_t* rp,
                    const void* const mv[4], int* flags);

// t = L^-1 r (input as in m_apply_w), y = U^-1 t in place of t with the
// epilogue of m_apply_g applied to y
hipError_t ilu_apply_fwd(hipStream_t st, const SellDesc& A, const void* mv, int tm,
                         const Basis& in, void* t, int tt, const int* stop, int64_t* cntr);
hipError_t ilu_apply_bwd(hipStream_t st, const SellDesc& A, const void* mv, int tm, void* t,
                         int tt, int mode, const double* omega, const void* zprev, void* out,
                         int tout, const double* s, int* fbflag, const int* stop, const int* cur);

}  // namespace f3r
