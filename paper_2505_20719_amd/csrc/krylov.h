// Vector kernels of the comparison solvers of Sec. 5 (preconditioned CG and
// BiCGStab, all fp64).  Scalars live in device memory (named slots of one
// small array), so an iteration needs no host round trip except its
// convergence check.  Every sum is a per-block partial followed by a
// fixed-order final sum (finalize_sums), as in the level kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace f3r {

// partial sums of x_i y_i per block (n_blocks(n) of them)
hipError_t dot64_partials(hipStream_t st, int64_t n, const double* x, const double* y,
                          void* partials);
// CG: alpha = rz / pq; x += alpha p; r -= alpha q; partials of ||r||^2
hipError_t cg_update_xr(hipStream_t st, int64_t n, double* x, double* r, const double* p,
                        const double* q, const double* rz, const double* pq, void* partials);
// CG: p = z + (rz_new / rz_old) p
hipError_t cg_update_p(hipStream_t st, int64_t n, double* p, const double* z,
                       const double* rz_new, const double* rz_old);
// BiCGStab: p = r + beta (p - omega v), beta = (rho_new / rho_old) (alpha / omega)
hipError_t bicg_update_p(hipStream_t st, int64_t n, double* p, const double* r, const double* v,
                         const double* rho_new, const double* rho_old, const double* alpha,
                         const double* omega);
// BiCGStab: alpha = rho / rv (stored to *alpha_out by block 0); s = r - alpha v;
// partials of ||s||^2
hipError_t bicg_update_s(hipStream_t st, int64_t n, double* s, const double* r, const double* v,
                         const double* rho, const double* rv, double* alpha_out, void* partials);
// BiCGStab: omega = ts / tt (stored to *omega_out by block 0);
// x += alpha z + omega ps; r = s - omega t; partials of ||r||^2
hipError_t bicg_update_xr(hipStream_t st, int64_t n, double* x, double* r, const double* s,
                          const double* t, const double* z, const double* ps, const double* alpha,
                          const double* ts, const double* tt, double* omega_out, void* partials);
// BiCGStab half step: x += alpha z
hipError_t axpy_dev(hipStream_t st, int64_t n, double* x, const double* z, const double* alpha);

}  // namespace f3r
