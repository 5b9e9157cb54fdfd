/*
 * f3r_oracle.h -- CPU oracle for the F3R nested Krylov solver.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, single-threaded C
 * implementation of what the GPU library computes, written step by step
 * from the paper ("A Nested Krylov Method Using Half-Precision Arithmetic",
 * arXiv 2505.20719).  Only the test-suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or helper with the GPU library and never
 * calls it.
 *
 * Every floating-point value is held in a C double.  A value "in precision
 * p" is a double that is exactly representable in p; every arithmetic
 * operation carried out "in precision q" is done in double and then rounded
 * to q with round-to-nearest-even.  For q in {fp32, fp16, bf16} that is
 * exactly IEEE arithmetic in q, because double has more than 2q+2 bits of
 * significand (the classical innocuous-double-rounding result for + - * / sqrt).
 *
 * Parity pins: see the header comment of f3r_oracle.c.
 */
#ifndef F3R_ORACLE_H
#define F3R_ORACLE_H
#include <stdint.h>

/* precision tags */
enum { OR_F64 = 0, OR_F32 = 1, OR_F16 = 2, OR_BF16 = 3 };
/* level kinds (Sec. 3 notation: F_m = FGMRES(m), R_m = Richardson(m)) */
enum { OR_FGMRES = 0, OR_RICH = 1 };
/* status codes */
enum {
  OR_OK = 0,
  OR_NOT_CONVERGED = 1,
  OR_ERR_ARG = -1,
  OR_ERR_MATRIX = -2,
  OR_ERR_RANGE = -3,
  OR_ERR_NOMEM = -4,
  OR_ERR_BREAKDOWN = -6
};

#define OR_MAX_LEV 8

typedef struct {
  int32_t kind;  /* OR_FGMRES or OR_RICH */
  int32_t m;     /* iterations per invocation */
  int32_t pA;    /* storage precision of the matrix at this level */
  int32_t pv;    /* storage precision of the level's vectors */
  int32_t pacc;  /* arithmetic precision (fp64 when pv is fp64, else fp32) */
} or_level;

typedef struct {
  int32_t nlev;            /* number of solver levels; level 0 is outermost */
  or_level lev[OR_MAX_LEV];
  int32_t pM;              /* storage precision of the primary preconditioner */
  int32_t m_identity;      /* 1: M = I */
  int32_t c;               /* weight-update cycle of Alg. 1; 0 = never update */
  double alpha;            /* diagonal factor used while building M */
  double omega_init;       /* initial Richardson weights (Alg. 1 uses 1) */
  int32_t max_outer;       /* total outermost iterations allowed */
  int32_t use_x0;          /* 1: x holds the initial guess */
  int32_t persist_weights; /* 1: keep omega and c_ntr from the previous solve */
  int32_t poison_call;     /* >0: inject NaN into the output of that R call */
  int32_t m_kind;          /* OR_M_SGS (two-SpMV truncated inverse) or OR_M_ILU */
  int32_t ilu_blocks;      /* block-Jacobi ILU(0): number of row blocks */
  int32_t dot_order;       /* summation order of the level dots and norms:
                              0 left to right (default), 1 right to left,
                              2, 4, 5, 6 blocks of 1024, 64, 256, 4096,
                              3, 7 pairwise with runs of 8, 32 */
} or_params;

#define OR_M_SGS 0
#define OR_M_ILU 1

typedef struct {
  int32_t status;
  int32_t outer_iters;   /* outermost iterations done */
  int32_t restarts;      /* completed outermost cycles that did not converge */
  int64_t m_calls;       /* applications of M */
  int64_t r_calls;       /* Richardson invocations actually executed */
  int64_t spmv[OR_MAX_LEV]; /* SpMVs with the level matrix, per level */
  int64_t fallbacks;     /* non-finite inner outputs replaced by the input */
  int64_t breakdowns;    /* exact zero subdiagonals met in any level */
  double relres_est;     /* last Givens estimate |g_{j+1}|/||b|| */
  double relres_true;    /* ||b - A x|| / ||b|| at exit, in fp64 */
} or_info;

typedef struct or_handle or_handle;

/* ---- soft floating point (IEEE 754 binary16 / bfloat16, RNE) ---- */
uint16_t or_f64_to_f16(double x);
double   or_f16_to_f64(uint16_t h);
uint16_t or_f64_to_bf16(double x);
double   or_bf16_to_f64(uint16_t h);
double   or_round(int32_t p, double x);
void     or_round_array(int32_t p, int64_t n, const double* in, double* out);
void     or_encode_f16_array(int64_t n, const double* in, uint16_t* out);
void     or_encode_bf16_array(int64_t n, const double* in, uint16_t* out);
void     or_decode_f16_array(int64_t n, const uint16_t* in, double* out);
void     or_decode_bf16_array(int64_t n, const uint16_t* in, double* out);

/* ---- set-up and solve ---- */
void or_params_default(or_params* p, int32_t variant);
int32_t or_setup(int64_t n, int64_t nnz, const int32_t* row_ptr,
                 const int32_t* col_idx, const double* val,
                 const or_params* p, or_handle** out);
void or_destroy(or_handle* h);
int32_t or_solve(or_handle* h, const double* b, double* x, double tol,
                 or_info* info);
/* comparison solvers (Sec. 5), fp64 vectors and arithmetic, preconditioner
   S M (S v) with M's factors in fp64 (m64 = 1) or in the handle's pM (0):
   restarted FGMRES(m), and method 0 = preconditioned CG, 1 = right-
   preconditioned BiCGStab. */
int32_t or_fgmres_solve(or_handle* h, const double* b, double* x, double tol,
                        int32_t m, int32_t max_iter, int32_t m64, or_info* info);
int32_t or_krylov_solve(or_handle* h, int32_t method, int32_t m64, const double* b,
                        double* x, double tol, int32_t max_iter, or_info* info);

/* ---- pieces, for lockstep comparisons and pins ---- */
int64_t or_n(const or_handle* h);
/* threads the library's parallel loops use (1 for the plain build) */
int32_t or_threads(void);
void or_get_scaling(const or_handle* h, double* s);
void or_get_level_values(const or_handle* h, int32_t p, double* vals);
void or_get_m_factors(const or_handle* h, int32_t* wrp, int32_t* wci,
                      double* wv, int32_t* grp, int32_t* gci, double* gv);
/* block-Jacobi ILU(0) factors in CSR order of A (L strictly below the
   diagonal, unit diagonal implied; U on and above it; couplings across
   blocks 0): fp64 (use64 = 1) or rounded to pM */
void or_get_ilu_values(const or_handle* h, int32_t use64, double* vals);
/* first row of block b (b = 0 .. blocks) */
int64_t or_ilu_block_start(const or_handle* h, int64_t b);
int64_t or_m_nnz_lower(const or_handle* h);
int64_t or_m_nnz_upper(const or_handle* h);
/* y = A_p x with A's values stored in pA, products and sums in pacc, result
   rounded to pout.  scaled = 1 uses the scaled matrix, 0 the original. */
void or_spmv(const or_handle* h, int32_t scaled, int32_t pA, int32_t pacc,
             int32_t pout, const double* x, double* y);
/* y = M r with vectors in pv, arithmetic in pacc */
void or_apply_m(or_handle* h, int32_t pv, int32_t pacc, const double* r,
                double* y);
/* z = level d applied to v (d >= 1; the level's own precisions) */
void or_apply_level(or_handle* h, int32_t d, const double* v, double* z);
/* Richardson state of level d (Alg. 1): weights omega_1..omega_m and c_ntr */
void or_get_weights(const or_handle* h, int32_t d, double* omega, int64_t* cntr);
void or_set_weights(or_handle* h, int32_t d, const double* omega, int64_t cntr);
/* outermost history: relative residual estimate per outermost iteration */
int64_t or_history(const or_handle* h, double* buf, int64_t cap);
/* level d's history: d = 0 as or_history; d >= 1 (FGMRES) the Givens
   estimate |g_{j+1}| / beta after every iteration of every invocation of
   the last solve, in order */
int64_t or_level_history(const or_handle* h, int32_t d, double* buf, int64_t cap);
/* Pins of the narrow arithmetic: or_trace(h, d, 1) makes every later
   invocation of the Richardson level d record its stored intermediates;
   or_rich_trace copies those of the last invocation (k steps: v (n), then
   r, tw, y, z, ta as k x n row-major, sc as k x 8) and returns k.
   or_level_cycle copies the last invocation of the FGMRES level d: V
   ((m+1) x n), Z (m x n), the Hessenberg matrix before rotations ((m+1) x m,
   column-major), the rotated g (m+1), y (m) and beta; returns m, or -1. */
int32_t or_trace(or_handle* h, int32_t d, int32_t on);
int32_t or_rich_trace(const or_handle* h, double* v, double* r, double* tw,
                      double* y, double* z, double* ta, double* sc);
int32_t or_level_cycle(const or_handle* h, int32_t d, double* V, double* Z,
                       double* H, double* g, double* y, double* beta);
/* the last outermost cycle's basis, for the Arnoldi-relation pin */
int32_t or_last_cycle(const or_handle* h, double* V, double* Z, double* H,
                      int32_t cap_m);

#endif
