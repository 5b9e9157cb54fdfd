// Vector kernels of the fp64 comparison solvers (see krylov.h).  Rows are
// split as in the level kernels (kR rows per thread, 1024 rows per block,
// XCD-aware block order); every thread derives the same scalar from the
// device slots, so no extra kernel computes it.
#include "common.h"
#include "kernels.h"
#include "krylov.h"

namespace f3r {

namespace {

__device__ __forceinline__ int64_t row_of(int64_t lb, int r) {
  return lb * kRowsPerBlock + (int64_t)r * kBlock + threadIdx.x;
}

__global__ __launch_bounds__(kBlock) void k_dotp(int64_t n, const double* __restrict__ x,
                                                 const double* __restrict__ y,
                                                 double* __restrict__ part, int64_t nb) {
  __shared__ double lds[kBlock / kWave];
  const int64_t lb = logical_block(nb);
  if (lb >= nb) return;
  double v = 0.0;
#pragma unroll
  for (int r = 0; r < kR; r++) {
    const int64_t i = row_of(lb, r);
    if (i < n) v = v + x[i] * y[i];
  }
  const double s = block_sum(v, lds);
  if (threadIdx.x == 0) part[lb] = s;
}

__global__ __launch_bounds__(kBlock) void k_cg_xr(int64_t n, double* __restrict__ x,
                                                  double* __restrict__ r,
                                                  const double* __restrict__ p,
                                                  const double* __restrict__ q, const double* rz,
                                                  const double* pq, double* __restrict__ part,
                                                  int64_t nb) {
  __shared__ double lds[kBlock / kWave];
  const int64_t lb = logical_block(nb);
  if (lb >= nb) return;
  const double alpha = *rz / *pq;
  double sq = 0.0;
#pragma unroll
  for (int k = 0; k < kR; k++) {
    const int64_t i = row_of(lb, k);
    if (i < n) {
      x[i] = x[i] + alpha * p[i];
      const double ri = r[i] - alpha * q[i];
      r[i] = ri;
      sq = sq + ri * ri;
    }
  }
  const double s = block_sum(sq, lds);
  if (threadIdx.x == 0) part[lb] = s;
}

__global__ __launch_bounds__(kBlock) void k_cg_p(int64_t n, double* __restrict__ p,
                                                 const double* __restrict__ z, const double* rzn,
                                                 const double* rzo, int64_t nb) {
  const int64_t lb = logical_block(nb);
  if (lb >= nb) return;
  const double beta = *rzn / *rzo;
#pragma unroll
  for (int k = 0; k < kR; k++) {
    const int64_t i = row_of(lb, k);
    if (i < n) p[i] = z[i] + beta * p[i];
  }
}

__global__ __launch_bounds__(kBlock) void k_bicg_p(int64_t n, double* __restrict__ p,
                                                   const double* __restrict__ r,
                                                   const double* __restrict__ v, const double* rhon,
                                                   const double* rhoo, const double* alpha,
                                                   const double* omega, int64_t nb) {
  const int64_t lb = logical_block(nb);
  if (lb >= nb) return;
  const double om = *omega;
  const double beta = (*rhon / *rhoo) * (*alpha / om);
#pragma unroll
  for (int k = 0; k < kR; k++) {
    const int64_t i = row_of(lb, k);
    if (i < n) p[i] = r[i] + beta * (p[i] - om * v[i]);
  }
}

__global__ __launch_bounds__(kBlock) void k_bicg_s(int64_t n, double* __restrict__ s,
                                                   const double* __restrict__ r,
                                                   const double* __restrict__ v, const double* rho,
                                                   const double* rv, double* alpha_out,
                                                   double* __restrict__ part, int64_t nb) {
  __shared__ double lds[kBlock / kWave];
  const int64_t lb = logical_block(nb);
  if (lb >= nb) return;
  const double alpha = *rho / *rv;
  double sq = 0.0;
#pragma unroll
  for (int k = 0; k < kR; k++) {
    const int64_t i = row_of(lb, k);
    if (i < n) {
      const double si = r[i] - alpha * v[i];
      s[i] = si;
      sq = sq + si * si;
    }
  }
  const double t = block_sum(sq, lds);
  if (threadIdx.x == 0) {
    part[lb] = t;
    if (lb == 0) *alpha_out = alpha;
  }
}

__global__ __launch_bounds__(kBlock) void k_bicg_xr(int64_t n, double* __restrict__ x,
                                                    double* __restrict__ r,
                                                    const double* __restrict__ s,
                                                    const double* __restrict__ t,
                                                    const double* __restrict__ z,
                                                    const double* __restrict__ ps,
                                                    const double* alpha, const double* ts,
                                                    const double* tt, double* omega_out,
                                                    double* __restrict__ part, int64_t nb) {
  __shared__ double lds[kBlock / kWave];
  const int64_t lb = logical_block(nb);
  if (lb >= nb) return;
  const double a = *alpha;
  const double om = *ts / *tt;
  double sq = 0.0;
#pragma unroll
  for (int k = 0; k < kR; k++) {
    const int64_t i = row_of(lb, k);
    if (i < n) {
      x[i] = x[i] + a * z[i] + om * ps[i];
      const double ri = s[i] - om * t[i];
      r[i] = ri;
      sq = sq + ri * ri;
    }
  }
  const double u = block_sum(sq, lds);
  if (threadIdx.x == 0) {
    part[lb] = u;
    if (lb == 0) *omega_out = om;
  }
}

__global__ __launch_bounds__(kBlock) void k_axpy_dev(int64_t n, double* __restrict__ x,
                                                     const double* __restrict__ z,
                                                     const double* alpha, int64_t nb) {
  const int64_t lb = logical_block(nb);
  if (lb >= nb) return;
  const double a = *alpha;
#pragma unroll
  for (int k = 0; k < kR; k++) {
    const int64_t i = row_of(lb, k);
    if (i < n) x[i] = x[i] + a * z[i];
  }
}

dim3 grid_of(int64_t n) { return dim3((unsigned)physical_grid(n_blocks(n))); }

}  // namespace

hipError_t dot64_partials(hipStream_t st, int64_t n, const double* x, const double* y,
                          void* partials) {
  hipLaunchKernelGGL(k_dotp, grid_of(n), dim3(kBlock), 0, st, n, x, y, (double*)partials, n_blocks(n));
  return hipGetLastError();
}

hipError_t cg_update_xr(hipStream_t st, int64_t n, double* x, double* r, const double* p,
                        const double* q, const double* rz, const double* pq, void* partials) {
  hipLaunchKernelGGL(k_cg_xr, grid_of(n), dim3(kBlock), 0, st, n, x, r, p, q, rz, pq,
                     (double*)partials, n_blocks(n));
  return hipGetLastError();
}

hipError_t cg_update_p(hipStream_t st, int64_t n, double* p, const double* z,
                       const double* rz_new, const double* rz_old) {
  hipLaunchKernelGGL(k_cg_p, grid_of(n), dim3(kBlock), 0, st, n, p, z, rz_new, rz_old, n_blocks(n));
  return hipGetLastError();
}

hipError_t bicg_update_p(hipStream_t st, int64_t n, double* p, const double* r, const double* v,
                         const double* rho_new, const double* rho_old, const double* alpha,
                         const double* omega) {
  hipLaunchKernelGGL(k_bicg_p, grid_of(n), dim3(kBlock), 0, st, n, p, r, v, rho_new, rho_old, alpha,
                     omega, n_blocks(n));
  return hipGetLastError();
}

hipError_t bicg_update_s(hipStream_t st, int64_t n, double* s, const double* r, const double* v,
                         const double* rho, const double* rv, double* alpha_out, void* partials) {
  hipLaunchKernelGGL(k_bicg_s, grid_of(n), dim3(kBlock), 0, st, n, s, r, v, rho, rv, alpha_out,
                     (double*)partials, n_blocks(n));
  return hipGetLastError();
}

hipError_t bicg_update_xr(hipStream_t st, int64_t n, double* x, double* r, const double* s,
                          const double* t, const double* z, const double* ps, const double* alpha,
                          const double* ts, const double* tt, double* omega_out, void* partials) {
  hipLaunchKernelGGL(k_bicg_xr, grid_of(n), dim3(kBlock), 0, st, n, x, r, s, t, z, ps, alpha, ts, tt,
                     omega_out, (double*)partials, n_blocks(n));
  return hipGetLastError();
}

hipError_t axpy_dev(hipStream_t st, int64_t n, double* x, const double* z, const double* alpha) {
  hipLaunchKernelGGL(k_axpy_dev, grid_of(n), dim3(kBlock), 0, st, n, x, z, alpha, n_blocks(n));
  return hipGetLastError();
}

}  // namespace f3r
