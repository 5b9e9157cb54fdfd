/*
 * f3r.h -- C ABI of the MI355X (gfx950) F3R solver library, libf3r.so.
 *
 * F3R is the nested Krylov solver of "A Nested Krylov Method Using
 * Half-Precision Arithmetic" (arXiv 2505.20719): in the tuple notation of
 * Sec. 3, (F_m1, F_m2, F_m3, R_m4, M) with defaults (100, 8, 4, 2) (Sec. 4.2),
 * three FGMRES levels in fp64, fp32 and fp16-matrix/fp32-vector precision
 * around a fp16 Richardson level with adaptive weights (Alg. 1, Sec. 4.3)
 * and a primary preconditioner M (Table 1).  The problem is A x = b with a
 * square sparse A, x0 = 0, stopping when ||b - A x||_2 / ||b||_2 < tol
 * (Sec. 1 and Sec. 5).
 *
 * Conventions for every entry point:
 *   - status codes only; nothing is thrown across the ABI;
 *   - matrices are passed as host CSR (0-based, int32 row pointers and
 *     column indices, columns sorted and unique within a row, fp64 values);
 *     f3r_setup copies them, the caller may free its arrays on return;
 *   - vectors b, x (and the vectors of the f3r_debug_* calls) are DEVICE
 *     pointers to n doubles on the device that was current at set-up;
 *   - all work is enqueued on the hipStream_t given at set-up (NULL = the
 *     default stream); calls return after that stream has drained the work
 *     they enqueued, because the outermost level checks convergence on the
 *     host (Sec. 5.2);
 *   - a handle is not re-entrant: one call at a time per handle.
 */
#ifndef F3R_H
#define F3R_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
typedef int32_t f3r_status;
#define F3R_OK 0
#define F3R_NOT_CONVERGED 1   /* soft: x holds the best iterate */
#define F3R_ERR_ARG (-1)      /* bad argument or parameter */
#define F3R_ERR_MATRIX (-2)   /* not square, unsorted/duplicate columns,
                                 missing or zero diagonal, non-finite value */
#define F3R_ERR_RANGE (-3)    /* a scaled value overflows a narrow format */
#define F3R_ERR_NOMEM (-4)    /* device or pinned host allocation failed */
#define F3R_ERR_DEVICE (-5)   /* HIP runtime error; code in f3r_info.hip_error */
#define F3R_ERR_BREAKDOWN (-6) /* non-finite value in the outermost level */

/* ---- precisions and level kinds --------------------------------------- */
#define F3R_FP64 0
#define F3R_FP32 1
#define F3R_FP16 2
#define F3R_BF16 3
#define F3R_FGMRES 0
#define F3R_RICHARDSON 1

/* variants for f3r_params_default (Sec. 5 names) */
#define F3R_VARIANT_FP16 0     /* fp16-F3R, precisions of Table 1 */
#define F3R_VARIANT_FP32 1     /* fp32-F3R: every inner level fp32 */
#define F3R_VARIANT_FP64 2     /* fp64-F3R: every level fp64 */
#define F3R_VARIANT_FGMRES64 3 /* FGMRES(64)+M, all fp64 (comparison solver) */
#define F3R_VARIANT_BF16 4     /* fp16-F3R with bfloat16 in place of binary16 */

/* flags */
#define F3R_USE_X0 1u          /* x holds the initial guess on entry */
#define F3R_PERSIST_WEIGHTS 2u /* keep omega and c_ntr from the previous solve */
#define F3R_NO_GRAPH 4u        /* launch kernels one by one (the default; wins over
                                  F3R_USE_GRAPH) */
#define F3R_BATCH_LOCKSTEP 8u  /* batches: solve the systems in lockstep with
                                  the per-kernel path (see f3r_setup_batched) */
#define F3R_USE_GRAPH 16u      /* record each call of the second level (one per
                                  Richardson update pattern) as a hipGraph and
                                  replay it.  Off by default: the outermost
                                  level waits on the host after every
                                  iteration, so each replay starts on an idle
                                  GPU, and launching the kernels one by one
                                  measured as fast or faster (fp16-F3R on the
                                  128^3 Poisson system 15.1 ms against 15.6 ms) */

/* kernels that f3r_params.probe_kernel can time with HIP events */
#define F3R_PROBE_NONE 0
#define F3R_PROBE_M_LOWER 1    /* W sweep of M inside the Richardson level */
#define F3R_PROBE_M_UPPER 2    /* G sweep of M (with the Richardson update) */
#define F3R_PROBE_R_RESIDUAL 3 /* Richardson residual SpMV r = v - A z */
#define F3R_PROBE_SPMV_L2 4    /* SpMV + Gram-Schmidt dots of level 2 */
#define F3R_PROBE_SPMV_L1 5    /* SpMV + Gram-Schmidt dots of level 1 */
#define F3R_PROBE_SPMV_L0 6    /* SpMV + Gram-Schmidt dots of level 0 */

/* device matrix formats (f3r_params.layout) */
#define F3R_LAYOUT_AUTO 0      /* SLICE when it stores at most 25 % more entries than
                                  the better of SELL and DIAG (not with M_ILU, not
                                  in the persistent batch kernel), else DIAG when
                                  it stores at most 3 % more entries than SELL,
                                  else SELL */
#define F3R_LAYOUT_SELL 1      /* slices of 64 rows, each padded to its longest row */
#define F3R_LAYOUT_DIAG 2      /* slices of 64 rows of one common width with every
                                  row's diagonal at one common position: no
                                  per-slice offsets or bounds to load */
#define F3R_LAYOUT_SLICE 3     /* DIAG whose column offsets are stored once per
                                  slice: each slice's positions are the sorted
                                  union of its rows' offsets (a row without an
                                  entry there holds 0), so no per-entry index
                                  is read.  At most 64 offsets per slice;
                                  refused (F3R_ERR_ARG) with M_ILU, whose
                                  ILU(0) needs each row's own pattern, and by
                                  the persistent batch kernel (the lockstep
                                  batch mode supports it) */

/* primary preconditioner M (f3r_params.m_kind) */
#define F3R_M_SGS 0   /* two-SpMV truncated inverse of the alpha-shifted
                         symmetric Gauss-Seidel factors (Sec. 5.2) */
#define F3R_M_ILU 1   /* block-Jacobi ILU(0) (Sec. 5.1): the rows split into
                         ilu_blocks contiguous ranges of nearly equal size
                         (block b: rows [b n / B, (b + 1) n / B)), couplings
                         between ranges dropped, each diagonal block of the
                         scaled matrix with its diagonal multiplied by alpha
                         factored as L U with A's sparsity; applied by a
                         forward and a backward sweep per block.  Not for
                         batches; the M_UPPER probe is refused. */

#define F3R_MAX_LEVELS 8

typedef struct {
  int32_t kind;   /* F3R_FGMRES or F3R_RICHARDSON (innermost only) */
  int32_t m;      /* iterations per invocation (m1..m4 of Sec. 4.2) */
  int32_t prec_a; /* storage precision of the level's matrix */
  int32_t prec_v; /* storage precision of the level's vectors; arithmetic is
                     fp64 when this is fp64 and fp32 otherwise (Table 1) */
} f3r_level;

typedef struct {
  int32_t nlev;                  /* number of solver levels (1..8) */
  f3r_level lev[F3R_MAX_LEVELS]; /* lev[0] is the outermost FGMRES, fp64 */
  int32_t prec_m;                /* storage precision of M (Table 1) */
  int32_t m_identity;            /* must be 0 (M = I is not provided) */
  int32_t c;                     /* weight-update cycle of Alg. 1; 0 = never */
  double alpha;                  /* diagonal factor used to build M (Sec. 5.2) */
  double omega_init;             /* initial Richardson weights (Alg. 1: 1) */
  int32_t max_outer;             /* outermost iterations allowed in total */
  uint32_t flags;                /* F3R_USE_X0 | F3R_PERSIST_WEIGHTS | ... */
  int32_t poison_call;           /* >0: test hook, NaN in that R call's output */
  int32_t probe_kernel;          /* F3R_PROBE_*: time that kernel with HIP events
                                    on the solve's stream (each call repeated 4
                                    times between one event pair; the kernel
                                    rewrites the same output); the solve then
                                    launches without hipGraphs */
  int32_t rows_per_lane;         /* shape of the M sweeps and of the Richardson
                                    residual: 0 = picked from the row lengths
                                    (two rows per lane for at most four
                                    entries on a side of the diagonal, four
                                    with narrow vectors in the slice-offset
                                    layout, else one); -1 = picked by timing
                                    the candidate shapes at set-up; 1, 2 or
                                    4 = that many rows per lane.  Results do
                                    not depend on it. */
  int32_t entry_chunk;           /* with rows_per_lane != 0: entries per load
                                    chunk (0 = 8, 4, 4 for 1, 2, 4 rows; 3 is
                                    allowed with 2 or 4 rows and narrow vectors,
                                    or with layout F3R_LAYOUT_SLICE) */
  int32_t layout;                /* F3R_LAYOUT_*: device format of the matrix
                                    and M; results do not depend on it */
  int32_t m_kind;                /* F3R_M_SGS (default) or F3R_M_ILU */
  int32_t ilu_blocks;            /* F3R_M_ILU: number of row blocks (1 .. n;
                                    default 112, Sec. 5.1) */
  int32_t reserved[1];
} f3r_params;

typedef struct {
  int64_t n;              /* rows = columns */
  int64_t nnz;            /* stored entries */
  const int32_t* row_ptr; /* host, n+1 entries, row_ptr[0] = 0 */
  const int32_t* col_idx; /* host, nnz entries, sorted and unique per row */
  const double* val;      /* host, nnz entries */
} f3r_csr;

typedef struct {
  int32_t status;        /* same as the return value */
  int32_t outer_iters;   /* outermost iterations done */
  int32_t restarts;      /* outermost cycles that ended without convergence */
  int32_t hip_error;     /* hipError_t of the failing call, for F3R_ERR_DEVICE */
  int64_t m_calls;       /* applications of M */
  int64_t r_calls;       /* Richardson invocations scheduled */
  int64_t spmv[F3R_MAX_LEVELS]; /* SpMVs with each level's matrix */
  int64_t fallbacks;     /* inner outputs replaced by the input (non-finite) */
  int64_t breakdowns;    /* exact zero subdiagonal met in a level */
  double relres_est;     /* last Givens estimate |g_{j+1}| / ||b|| */
  double relres_true;    /* ||b - A x|| / ||b|| at exit, fp64 */
  double setup_ms;       /* wall time of f3r_setup */
  double solve_ms;       /* wall time of the solve */
  int64_t graph_launches; /* F2-call graphs replayed (F3R_USE_GRAPH) */
  int32_t idx_bits;      /* 16 or 32: column index width of the device format
                            (0: offsets per slice, no per-entry index) */
  int32_t sell_c;        /* rows per slice of the device format */
  double probe_ms;       /* summed duration of the probed kernel's launches */
  int64_t probe_launches; /* launches of the probed kernel (each probed call is
                             made 4 times in a row between one event pair) */
  int64_t padded_nnz;    /* stored entries of the device format incl. padding */
  int32_t rows_per_lane[3]; /* shapes in use: W sweep, G sweep, Richardson residual */
  int32_t entry_chunk[3];   /* entries per load chunk of the same three sweeps
                               (the residual's rule also picks 7, one chunk
                               over rows of seven entries, for narrow vectors
                               in the slice-offset layout) */
  double tune_ms;        /* set-up time spent timing the candidate shapes */
  int32_t layout;        /* F3R_LAYOUT_SELL, _DIAG or _SLICE: format in use */
  int32_t ilu_sweep;     /* F3R_M_ILU: forms of the triangular sweeps launched
                            since set-up, a bit mask: 1 = level windows staged
                            in LDS, 2 = block vector in LDS without windows,
                            4 = vector in global memory (0 otherwise) */
} f3r_info;

typedef struct f3r_handle f3r_handle;

/* Parameters of a named variant (Sec. 5): fills every field. */
void f3r_params_default(f3r_params* p, int32_t variant);

/* Copies A to the device, applies symmetric diagonal scaling
   Ahat = D^-1/2 A D^-1/2 (Sec. 5), rounds the per-level value copies of
   Table 1 directly from fp64, builds the two factors of M in fp64 and casts
   them (Secs. 5 and 5.2), converts everything to the device format and
   allocates every workspace.  hip_stream: a hipStream_t or NULL.
   Errors: F3R_ERR_ARG (NULL pointers, bad parameters), F3R_ERR_MATRIX,
   F3R_ERR_RANGE (a narrow copy of Ahat or M would overflow),
   F3R_ERR_NOMEM, F3R_ERR_DEVICE.  *out is NULL on error. */
f3r_status f3r_setup(const f3r_csr* A, const f3r_params* p, void* hip_stream,
                     f3r_handle** out);

/* Solves A x = b with the nest given at set-up (Sec. 4.2): FGMRES(m1) in
   fp64 on the original A, calling the inner nest as S F2(S v) on the scaled
   system; convergence is checked on the host after each outermost iteration
   from the Givens estimate and confirmed with the fp64 true residual at the
   end of each cycle; the whole nest restarts after m1 iterations (Sec. 4.2).
   b, x: device pointers (n doubles); x is overwritten (or read first with
   F3R_USE_X0).  level_override: NULL, or parameters whose nlev, m, c,
   omega_init, max_outer and flags replace the set-up ones for this call
   (precisions must equal the set-up ones).  info may be NULL.
   Returns F3R_OK, F3R_NOT_CONVERGED (x is the last iterate), or an error. */
f3r_status f3r_solve(f3r_handle* h, const double* b, double* x, double tol,
                     const f3r_params* level_override, f3r_info* info);

/* Restarted FGMRES(m) in fp64 preconditioned by S M (S v): the comparison
   solver of Sec. 5.  prec_m is the storage of M's values (F3R_FP64 for
   "fp64-FGMRES(64)", or a precision the handle holds -- its prec_m, and any
   level precision when alpha = 1 -- for the fp32/fp16 variants; arithmetic
   stays fp64); others give F3R_ERR_ARG.  Same conventions as f3r_solve;
   max_iter counts iterations over all restarts, m <= the set-up m1. */
f3r_status f3r_fgmres_solve(f3r_handle* h, const double* b, double* x,
                            double tol, int32_t m, int32_t max_iter,
                            int32_t prec_m, f3r_info* info);

/* The other comparison solvers of Sec. 5: preconditioned CG (method F3R_CG,
   for symmetric positive definite A) or right-preconditioned BiCGStab
   (F3R_BICGSTAB), every vector and operation in fp64, preconditioned by
   S M (S v) with M's factors stored in prec_m (F3R_FP64, or a precision the
   handle holds: its prec_m, and any level precision when alpha = 1).
   Convergence is tested on the recursive residual and confirmed with the
   fp64 true residual (the iteration continues from it otherwise); max_iter
   bounds the iterations.  info->outer_iters counts iterations, m_calls the
   applications of M.  Same conventions as f3r_solve; F3R_ERR_ARG for an
   unknown method, a precision the handle does not hold, tol <= 0 or
   max_iter < 1, and on a batched (stacked) handle. */
#define F3R_CG 0
#define F3R_BICGSTAB 1
f3r_status f3r_krylov_solve(f3r_handle* h, int32_t method, int32_t prec_m, const double* b,
                            double* x, double tol, int32_t max_iter, f3r_info* info);

/* Residual history of the last solve (Sec. 4.2: each FGMRES level's Givens
   estimate).  level 0: the relative residual estimate |g_{j+1}| / ||b||
   after every outermost iteration.  level d >= 1 (an FGMRES level): the
   estimate |g_{j+1}| / beta of that level after every iteration of every
   call, in order (beta = the norm of the call's input; a call that ends in
   a breakdown records the iterations it made; calls skipped because an
   outer level stopped record nothing); at most 1,000 outermost iterations'
   worth are kept, and none for batched handles (*len = 0).  Copies
   min(cap, available) values to buf (host), *len = available.
   Errors: F3R_ERR_ARG (bad level, a Richardson level), F3R_ERR_DEVICE. */
f3r_status f3r_get_history(const f3r_handle* h, int32_t level, double* buf,
                           int64_t cap, int64_t* len);

/* Richardson state of Alg. 1 for the Richardson level `level`: the weights
   omega_1..omega_m (host array of m doubles) and the call counter c_ntr.
   Errors: F3R_ERR_ARG when `level` is not a Richardson level. */
f3r_status f3r_get_weights(f3r_handle* h, int32_t level, double* omega,
                           int64_t* c_ntr);
f3r_status f3r_set_weights(f3r_handle* h, int32_t level, const double* omega,
                           int64_t c_ntr);

/* Frees every device and host resource of the handle. NULL is allowed. */
void f3r_destroy(f3r_handle* h);

/* Static English text of a status code. */
const char* f3r_status_str(f3r_status s);

/* ---- batches of independent systems -------------------------------------
   Many systems of different sizes solved by one persistent kernel launch:
   each workgroup of the launch takes the next system from a queue ordered
   by decreasing size and runs the whole nest of Sec. 4.2 on it, with the
   per-iteration stopping test of Sec. 5 taken on the device.  The
   arithmetic of every stored value is that of Table 1, as in f3r_solve;
   only the summation order of dot products and norms differs. */
typedef struct f3r_batch f3r_batch;

/* Sets up `count` systems (A: host array of count CSR matrices, each copied
   and scaled as by f3r_setup).  Two execution modes:
   - default: one persistent launch, one workgroup per system (above).  The
     parameters must describe the narrow F3R nest: nlev = 4; levels FGMRES
     (fp64, fp64), FGMRES (fp32, fp32), FGMRES (narrow matrix, fp32
     vectors), Richardson (narrow, narrow), with prec_m = narrow, where
     narrow is F3R_FP16 or F3R_BF16 (the defaults of F3R_VARIANT_FP16 and
     F3R_VARIANT_BF16); m1 <= 128 and m2, m3, m4 <= 16.  Flags: only
     F3R_USE_X0.
   - F3R_BATCH_LOCKSTEP in p->flags: the systems become the diagonal blocks
     of one matrix (each padded with identity rows to a multiple of 1024
     rows) solved by the per-kernel path of f3r_solve: every kernel covers
     all systems, sums and level state are per system, and each system stops
     at its own tolerance (its rows are then skipped).  Any nest f3r_setup
     accepts; the Richardson call counter c_ntr is shared by the systems.
   Weights and c_ntr restart for every solve (Alg. 1).  Errors as f3r_setup;
   F3R_ERR_ARG also for parameters outside the mode's set.  *out is NULL on
   error. */
f3r_status f3r_setup_batched(int32_t count, const f3r_csr* A, const f3r_params* p,
                             void* hip_stream, f3r_batch** out);

/* Solves every system: b[i], x[i] are device pointers (n_i doubles) held in
   host arrays of `count` entries; x[i] is overwritten (or read first with
   F3R_USE_X0).  infos: NULL or a host array of `count` records (solve_ms is
   the wall time of the whole batch).  Returns F3R_OK when every system
   converged, F3R_NOT_CONVERGED when some did not, else the most severe
   error of any system; the call returns after the launch has finished. */
f3r_status f3r_solve_batched(f3r_batch* bt, const double* const* b, double* const* x,
                             double tol, f3r_info* infos);

/* Residual estimates after every outermost iteration of system `sys` in the
   last batched solve; conventions of f3r_get_history. */
f3r_status f3r_batch_get_history(const f3r_batch* bt, int32_t sys, double* buf,
                                 int64_t cap, int64_t* len);

/* Frees every resource of the batch. NULL is allowed. */
void f3r_batch_destroy(f3r_batch* bt);

/* ---- single steps, for lockstep checks against a reference ------------
   Every vector is a device array of n doubles holding values representable
   in the precision named; results are widened exactly to fp64. */

/* y = A_d x: level 0 uses the original A in fp64; level d >= 1 the scaled
   matrix stored in the level's prec_a, with the level's arithmetic, the
   result rounded to the level's prec_v (Table 1; mixed inputs use the wider
   arithmetic, Sec. 4.2). */
f3r_status f3r_debug_spmv(f3r_handle* h, int32_t level, const double* x,
                          double* y);

/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid allocation): y = M r
   as f3r_debug_apply_m computes it (same kernels, same results bit for
   bit), with its two intermediate vectors (the input cast to prec and
   t = W r) in a fixed 64 MiB device array of the library instead of the
   handle's workspace, so the call allocates nothing.  Each device keeps
   its own copy of the array until the process ends; its address is looked
   up when a handle is set up on that device.  Calls on one device share
   that array: calls that overlap on one device (several host threads or
   streams) race, and must be serialised by the caller.  r, y: device
   arrays of n doubles; prec as for f3r_debug_apply_m.
   Errors: F3R_ERR_ARG (bad arguments, or 2 n (bytes of prec) rounded up to
   256 each above 64 MiB: n > 4,194,304 in fp64, 8,388,608 in fp32,
   16,777,216 in fp16/bf16), F3R_ERR_DEVICE. */
f3r_status f3r_apply_m_static(f3r_handle* h, int32_t prec, const double* r, double* y);

/* Measurement of the level SpMV of Sec. 4.2 on its own: `reps` launches of
   level `level`'s SpMV (an FGMRES level: level 0 is the fp64 matrix with
   fp64 vectors, deeper levels their Table 1 storage) on the handle's own
   buffers, each bracketed by its own pair of HIP events on the handle's
   stream.  With scrub_bytes > 0, a device buffer `scrub` (caller-owned,
   16-byte aligned, larger than the last-level cache, zero-filled by the
   caller) is read once before every launch, so that the matrix comes from
   HBM and not from the caches and no dirty lines are written back during
   the timed launch.  *avg_ms = mean launch time.  Overwrites the level's first
   Z slot and second V slot (solve state), nothing else.  F3R_ERR_ARG for a
   Richardson level or bad sizes. */
f3r_status f3r_time_spmv(f3r_handle* h, int32_t level, int32_t reps, void* scrub,
                         int64_t scrub_bytes, double* avg_ms);

/* The reference that the SpMV rates above are read against (Sec. 5.2 counts
   the sliced-ELLPACK SpMV as bandwidth-bound): `reps` plain reads of the
   first bytes / 16 x 16 bytes of the device buffer `buf` (caller-owned,
   16-byte aligned, zero-filled by the caller, not written), each workgroup
   reading one contiguous range with 16-byte non-temporal loads, each read
   bracketed by its own pair of HIP events on the handle's stream.
   *avg_ms = mean time of one read.  F3R_ERR_ARG for a null or unaligned
   buffer, bytes < 16 or reps outside [1, 10000]. */
f3r_status f3r_time_read(f3r_handle* h, const void* buf, int64_t bytes, int32_t reps,
                         double* avg_ms);

/* y = M r with vectors stored in prec (the two-SpMV application of
   Sec. 5.2; fp32 arithmetic for narrow prec, fp64 for fp64). prec must be
   the precision of M or wider. */
f3r_status f3r_debug_apply_m(f3r_handle* h, int32_t prec, const double* r,
                             double* y);

/* z = level d (1 <= d < nlev) applied to v on the scaled system, with the
   handle's Richardson state (which it advances). */
f3r_status f3r_debug_apply_level(f3r_handle* h, int32_t level, const double* v,
                                 double* z);

/* out_i = in_i rounded to prec with the library's conversion (round to
   nearest, ties to even, directly from fp64; Table 1 casts) and widened back
   exactly.  in, out: device arrays of n doubles.  No handle is needed. */
f3r_status f3r_debug_round(int32_t prec, const double* in, double* out, int64_t n,
                           void* hip_stream);

/* Host copies of the set-up results in CSR order: the scaling s (n doubles)
   and the scaled values rounded to prec (nnz doubles). */
f3r_status f3r_debug_scaling(f3r_handle* h, double* s_host);
f3r_status f3r_debug_level_values(f3r_handle* h, int32_t prec,
                                  double* vals_host);
/* M's stored values in CSR order of A (nnz doubles) in storage prec, when M
   has its own values (alpha != 1 or block-Jacobi ILU(0): the factors, L left
   of the diagonal, U on and right of it, zero across blocks); else
   F3R_ERR_ARG. */
f3r_status f3r_debug_m_values(f3r_handle* h, int32_t prec, double* vals_host);

#ifdef __cplusplus
}
#endif
#endif
