// Device interface of the batched solver: one persistent launch in which
// every workgroup takes systems from a queue (largest first) and runs the
// whole F3R nest of Sec. 3/4.2 on each, with workgroup barriers in place of
// kernel boundaries and the stopping test of Sec. 5 taken on the device.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace f3r {

constexpr int kBatchThreads = 512;  // threads of a batch workgroup (8 waves)
constexpr int kBatchMaxM1 = 128;     // largest outermost restart length
constexpr int kBatchMaxInner = 16;   // largest m of the inner levels

// Per-system results, written by the system's workgroup.
struct BatchOut {
  int32_t status, outer, restarts, fallbacks, breakdowns, pad;
  int64_t r_calls, upd_calls;
  double relres_est, relres_true;
};

// One system.  The workspace `ws` holds, in this order (n = A.n):
//   V1 (m1+1) n doubles | Z1 m1 n floats | H1 (m1+1) m1 doubles |
//   V2 (m2+1) n floats  | Z2 m2 n floats | V3 m3 n floats |
//   Z3 m3 n narrow      | R 5 n narrow (r, t, y, z_a, z_b)
// where "narrow" is the fp16 or bf16 storage of the two inner levels.
struct BatchSys {
  SellDesc A;
  const double* a64;  // original values (outermost level)
  const float* a32;   // scaled values, fp32 (second level)
  const void* a16;    // scaled values, narrow (third level and Richardson)
  const void* m16;    // M values (a16 itself, negated, when alpha = 1)
  const double* s;    // diagonal scaling
  const double* b;
  double* x;
  char* ws;
  double* hist;       // max_outer residual estimates
  BatchOut* out;
};

struct BatchArgs {
  const BatchSys* sys;
  const int* order;  // processing order (indices into sys)
  int count;
  int* queue;        // next position in `order`; zero before the launch
  int m1, m2, m3, m4, c, max_outer, use_x0, neg, bf16, idx16;
  float omega_init;  // initial Richardson weight (fp32 value)
  float gd;          // diagonal of G, round(1 / alpha) in the narrow format
  double tol;
};

// bytes of the workspace of one system
size_t batch_ws_bytes(int64_t n, int m1, int m2, int m3);

hipError_t batch_launch(hipStream_t st, const BatchArgs& a, int grid);

}  // namespace f3r
