// Host-side plumbing shared by the single-system and the batched entry
// points: error propagation, owned device allocations and the device copy
// of one matrix (SELL-64 arrays, scaled level copies, M values, scaling).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <vector>

#include "f3r.h"
#include "ilu.h"
#include "kernels.h"

namespace f3r {

struct DevErr {
  hipError_t e;
};
struct StatusErr {
  f3r_status s;
};
#define HIPCHK(x)                                 \
  do {                                            \
    hipError_t _e = (x);                          \
    if (_e != hipSuccess) throw ::f3r::DevErr{_e}; \
  } while (0)

// Device allocations owned by one object; freed together.
struct DevAllocs {
  std::vector<void*> ptrs;
  void* get(size_t bytes) {
    void* p = nullptr;
    if (bytes == 0) bytes = 8;
    if (hipMalloc(&p, bytes) != hipSuccess) throw StatusErr{F3R_ERR_NOMEM};
    ptrs.push_back(p);
    return p;
  }
  void release(void* p) {
    auto it = std::find(ptrs.begin(), ptrs.end(), p);
    if (it == ptrs.end()) return;
    (void)hipFree(p);
    ptrs.erase(it);
  }
  void release_all() {
    for (void* p : ptrs) (void)hipFree(p);
    ptrs.clear();
  }
};

// One matrix on the device.
struct MatrixDev {
  int64_t n = 0, nnz = 0, padded = 0;
  SellDesc A{};
  int32_t* rp = nullptr;      // CSR row pointers (kept for read-back)
  double* a64 = nullptr;      // original values
  void* ah[4] = {};           // scaled values per precision tag (null when unused)
  void* mv[4] = {};           // M values when they differ from -ahat (alpha != 1)
  bool m_shared = true;       // M values are -ahat (alpha == 1)
  double gd[4] = {1, 1, 1, 1};  // diagonal of G: round_t(1 / alpha)
  double* s = nullptr;        // s_i = 1 / sqrt(|a_ii|)
  uint16_t* kd_true = nullptr;  // diagonal-aligned format: each row's own diagonal position
  int32_t* ci = nullptr;        // slice-offset format: CSR columns (for read-back)
  IluDesc ilu;                  // block-Jacobi ILU(0) schedule (blocks = 0: not used)
};

// Validates the CSR matrix (host checks first, then the device checks of
// the set-up kernels), scales it, builds the SELL-64 arrays and the level
// copies the parameters ask for.  need[t] forces the scaled copy of tag t.
// Returns F3R_OK or the status of the first failed check; throws DevErr on a
// HIP error and StatusErr on an allocation failure.
// allow_slice: the slice-offset format may be chosen (not for the batch
// kernel, which reads per-entry indices only).
f3r_status build_matrix(hipStream_t st, const f3r_csr* A, const f3r_params* p, const bool need[4],
                        DevAllocs& al, MatrixDev& m, bool allow_slice = true);

// Several systems solved in lockstep by the per-kernel path: one handle whose
// matrix holds the systems on its diagonal (each padded with identity rows
// to a multiple of 1024), every kernel covering all systems, reductions and
// level state per system.  b, x: host arrays of device pointers.
f3r_status stacked_setup(int32_t count, const f3r_csr* A, const f3r_params* p, void* hip_stream,
                         f3r_handle** out);
f3r_status stacked_solve(f3r_handle* h, const double* const* b, double* const* x, double tol,
                         f3r_info* infos);
f3r_status stacked_history(const f3r_handle* h, int32_t sys, double* buf, int64_t cap,
                           int64_t* len);

}  // namespace f3r
