/*
 * f3r_oracle.c -- CPU oracle for F3R (arXiv 2505.20719).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test-suite, the smoke check and
 * the CPU-baseline leg of the benchmark; never by the GPU library.
 *
 * What it computes, and where the paper defines it:
 *   - the nested solver (S1, ..., SD, M) of Sec. 3, instantiated as F3R =
 *     (F_m1, F_m2, F_m3, R_m4, M) of Sec. 4.2, precisions per Table 1;
 *   - the variants of Sec. 5 (fp64-, fp32-, fp16-F3R), the depth variants of
 *     Table 4, and restarted FGMRES(m) + M used as the comparison solver;
 *   - FGMRES levels with classical Gram-Schmidt and Givens rotations
 *     (Sec. 4.2), inner initial guess zero, convergence checked only by the
 *     outermost level, whole-nest restart after m1 outermost iterations;
 *   - Richardson with adaptive weights, Alg. 1 and Eqs. (4)-(5) of Sec. 4.3;
 *     the locally optimal weight is computed in fp32 (end of Sec. 4.3);
 *   - symmetric diagonal scaling of A (Sec. 5);
 *   - the primary preconditioner M: the paper's GPU preconditioner costs two
 *     SpMVs per application and scales the diagonal of A by alpha while it is
 *     built (Sec. 5.2), but its construction is not given.  This oracle uses
 *     M = G W with W = I - L/alpha and G = (1/alpha)(I - U/alpha), where
 *     Ahat = I + L + U (unit diagonal after scaling): the first-order
 *     truncation of the inverse of the alpha-shifted symmetric Gauss-Seidel
 *     factors.  Built in fp64, then cast (Sec. 5: preconditioners are built
 *     in fp64 and their values cast to the lower precision).
 *
 * Readings where the paper is silent (each is also listed in the design
 * notes of the repository):
 *   - a single classical Gram-Schmidt pass; h_{j+1,j} is the norm of the
 *     updated w;
 *   - an exact zero h_{j+1,j} truncates the level at that iteration; Richardson
 *     calls that the skipped iterations would have made still advance c_ntr,
 *     so c_ntr is a function of the position in the nest schedule only;
 *   - a non-finite output of an inner level is replaced by that level's
 *     input (identity fallback) and counted;
 *   - l in Eq. (5) is taken literally as c_ntr / c (integer division), so
 *     the initial weight counts as one sample of the running mean;
 *   - omega and c_ntr are reset at the start of every solve (unless
 *     persist_weights is set) and kept across outermost restarts;
 *   - when (t, t) is zero or omega' is not finite the update is skipped and
 *     the current omega_k is used for that step;
 *   - the outermost level runs on the original A in fp64 and calls the inner
 *     nest as P(v) = S F2(S v) with S = diag(s); the inner levels run on
 *     Ahat = S A S, whose value copies are rounded directly from fp64 (RNE);
 *   - inner-level arithmetic is fp32 whenever its vectors are narrower than
 *     fp64 (products and sums rounded to fp32, one rounding to the storage
 *     precision per stored element).
 *
 * Parity pins (tests marked "not gpu"): soft binary16/bfloat16 against
 * numpy/torch conversions over all codes; SpMV against exact sums within the
 * unit-roundoff bound; M against its dense product; Richardson closed forms
 * and the GMRES(1) special case; FGMRES against dense LU and the flexible
 * Arnoldi relation; nest reductions (fp64-F3R with m2=m3=m4=1 equals
 * FGMRES(m1)+M); M-call counts; end-to-end residual certificates; every
 * stored intermediate of the narrow levels (Richardson in fp16/bf16, the
 * fp32 FGMRES levels) within the rounding bound of its stage, recorded
 * through or_trace / or_rich_trace / or_level_cycle (recording only).
 *
 * Threads: built with -fopenmp (the CPU-baseline build), the loops whose
 * iterations write separate elements (SpMV rows, vector updates) and the
 * blocks of the blocked dot orders are shared among threads; every value is computed
 * by the same operations as in the plain build, so both builds give the
 * same results bit for bit.  The plain build (-fno-openmp) is what the pins
 * exercise.
 */
#include "f3r_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
/* the next loop's iterations are independent: share them among threads */
#define OR_PAR_FOR _Pragma("omp parallel for schedule(static)")
#else
#define OR_PAR_FOR
#endif

int32_t or_threads(void) {
#ifdef _OPENMP
  return (int32_t)omp_get_max_threads();
#else
  return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* soft floating point                                                       */
/* ------------------------------------------------------------------------ */

/* binary16: 1 sign bit, 5 exponent bits (bias 15), 10 fraction bits.
   Normal numbers 2^-14 <= |x| <= 65504, subnormals k * 2^-24.
   Round to nearest, ties to even (nearbyint in the default rounding mode).
   Scaling by powers of two with ldexp is exact. */
uint16_t or_f64_to_f16(double x) {
  uint16_t sign = signbit(x) ? 0x8000u : 0u;
  if (isnan(x)) return (uint16_t)(sign | 0x7E00u);
  double a = fabs(x);
  if (isinf(a)) return (uint16_t)(sign | 0x7C00u);
  if (a < 0x1p-14) {
    double k = nearbyint(a * 0x1p24); /* 0..1024; 1024 encodes 2^-14 */
    return (uint16_t)(sign | (uint16_t)k);
  }
  int e;
  frexp(a, &e); /* a = f 2^e with f in [0.5, 1) */
  int E = e - 1; /* a in [2^E, 2^(E+1)) */
  double k = nearbyint(ldexp(a, 10 - E)); /* in [1024, 2048] */
  if (k == 2048.0) {
    k = 1024.0;
    E += 1;
  }
  if (E > 15) return (uint16_t)(sign | 0x7C00u);
  return (uint16_t)(sign | (uint16_t)(((E + 15) << 10) | ((int)k - 1024)));
}

double or_f16_to_f64(uint16_t h) {
  int s = h >> 15, E = (h >> 10) & 31, f = h & 1023;
  double v;
  if (E == 0)
    v = ldexp((double)f, -24);
  else if (E == 31)
    v = f ? NAN : INFINITY;
  else
    v = ldexp((double)(1024 + f), E - 25);
  return s ? -v : v;
}

/* bfloat16: 1 sign bit, 8 exponent bits (bias 127), 7 fraction bits.
   Normal numbers 2^-126 <= |x| < 2^128, subnormals k * 2^-133. */
uint16_t or_f64_to_bf16(double x) {
  uint16_t sign = signbit(x) ? 0x8000u : 0u;
  if (isnan(x)) return (uint16_t)(sign | 0x7FC0u);
  double a = fabs(x);
  if (isinf(a)) return (uint16_t)(sign | 0x7F80u);
  if (a < 0x1p-126) {
    double k = nearbyint(a * 0x1p133); /* 0..128; 128 encodes 2^-126 */
    return (uint16_t)(sign | (uint16_t)k);
  }
  int e;
  frexp(a, &e);
  int E = e - 1;
  double k = nearbyint(ldexp(a, 7 - E)); /* in [128, 256] */
  if (k == 256.0) {
    k = 128.0;
    E += 1;
  }
  if (E > 127) return (uint16_t)(sign | 0x7F80u);
  return (uint16_t)(sign | (uint16_t)(((E + 127) << 7) | ((int)k - 128)));
}

double or_bf16_to_f64(uint16_t h) {
  int s = h >> 15, E = (h >> 7) & 255, f = h & 127;
  double v;
  if (E == 0)
    v = ldexp((double)f, -133);
  else if (E == 255)
    v = f ? NAN : INFINITY;
  else
    v = ldexp((double)(128 + f), E - 134);
  return s ? -v : v;
}

double or_round(int32_t p, double x) {
  switch (p) {
    case OR_F32:
      return (double)(float)x;
    case OR_F16:
      return or_f16_to_f64(or_f64_to_f16(x));
    case OR_BF16:
      return or_bf16_to_f64(or_f64_to_bf16(x));
    default:
      return x;
  }
}

/* rounding helper used by all arithmetic below */
#define RND(p, x) or_round((p), (x))

void or_round_array(int32_t p, int64_t n, const double* in, double* out) {
  for (int64_t i = 0; i < n; i++) out[i] = RND(p, in[i]);
}
void or_encode_f16_array(int64_t n, const double* in, uint16_t* out) {
  for (int64_t i = 0; i < n; i++) out[i] = or_f64_to_f16(in[i]);
}
void or_encode_bf16_array(int64_t n, const double* in, uint16_t* out) {
  for (int64_t i = 0; i < n; i++) out[i] = or_f64_to_bf16(in[i]);
}
void or_decode_f16_array(int64_t n, const uint16_t* in, double* out) {
  for (int64_t i = 0; i < n; i++) out[i] = or_f16_to_f64(in[i]);
}
void or_decode_bf16_array(int64_t n, const uint16_t* in, double* out) {
  for (int64_t i = 0; i < n; i++) out[i] = or_bf16_to_f64(in[i]);
}

/* ------------------------------------------------------------------------ */
/* handle                                                                    */
/* ------------------------------------------------------------------------ */

typedef struct {
  int32_t m;
  double *V, *Z, *H, *Hraw, *cs, *sn, *g, *y, *w;
  double *tmp0, *tmp1, *tmp2, *tmp3, *tmp4; /* Richardson / scaling scratch */
  double beta;   /* ||v|| of the level's last invocation (FGMRES) */
  int32_t meff;  /* iterations of that invocation */
} level_ws;

/* Copies of every stored intermediate of one Richardson invocation, kept
   only when tracing is switched on (or_trace); recording changes nothing
   in the arithmetic. */
typedef struct {
  int32_t on, d, m, steps;
  double* v;    /* the input rounded to the level's storage */
  double* r;    /* m x n: r_{k-1} */
  double* tw;   /* m x n: W r_{k-1} (the first of the two SpMVs of M) */
  double* y;    /* m x n: M r_{k-1} */
  double* z;    /* m x n: z_k */
  double* ta;   /* m x n: A y on update steps (kept in the arithmetic precision) */
  double sc[64][8]; /* per step: updated, num, den, omega', omega before,
                       omega after, l, weight used */
} rich_trace;

struct or_handle {
  or_params p;
  int64_t n, nnz;
  int32_t *rp, *ci;
  double* a;           /* original values */
  double* s;           /* s_i = 1 / sqrt(|a_ii|) */
  double* ahat;        /* scaled values in fp64 */
  double* alev[4];     /* ahat rounded to each precision tag, when used */
  int64_t wnnz, gnnz;  /* M factors: W lower (unit diagonal), G upper */
  int32_t *wrp, *wci, *grp, *gci;
  double *wv64, *gv64; /* fp64 factors */
  double *wv, *gv;     /* factors rounded to pM */
  double* mtmp;        /* intermediate of the two-SpMV application */
  double *iv64, *iv;   /* block-Jacobi ILU(0) factors (CSR order of A), fp64 and pM */
  int32_t* idiag;      /* position of each row's diagonal in its CSR row */
  level_ws ws[OR_MAX_LEV];
  double omega[OR_MAX_LEV][64];
  int64_t cntr[OR_MAX_LEV];
  or_info st;
  int32_t baseline; /* 1 while running the comparison FGMRES(m) */
  int32_t base_m64; /* its M: fp64 factors (1) or the pM ones (0) */
  double* hist;
  int64_t hist_len, hist_cap;
  int32_t last_m;
  rich_trace tr;
  double* lhist[OR_MAX_LEV]; /* inner levels: |g_{j+1}| / beta per iteration */
  int64_t lhist_len[OR_MAX_LEV], lhist_cap[OR_MAX_LEV];
};

int64_t or_n(const or_handle* h) { return h->n; }

static void* xcalloc(int64_t count, size_t sz) {
  if (count <= 0) count = 1;
  return calloc((size_t)count, sz);
}

void or_params_default(or_params* p, int32_t variant) {
  memset(p, 0, sizeof(*p));
  p->pM = OR_F16;
  p->c = 64;
  p->alpha = 1.0;
  p->omega_init = 1.0;
  p->max_outer = 300;
  /* F3R = (F100, F8, F4, R2, M), Sec. 4.2 */
  p->nlev = 4;
  int ms[4] = {100, 8, 4, 2};
  for (int d = 0; d < 4; d++) {
    p->lev[d].kind = d == 3 ? OR_RICH : OR_FGMRES;
    p->lev[d].m = ms[d];
  }
  /* variant 0: fp16-F3R, Table 1 */
  int pA[4] = {OR_F64, OR_F32, OR_F16, OR_F16};
  int pv[4] = {OR_F64, OR_F32, OR_F32, OR_F16};
  if (variant == 1) { /* fp32-F3R: every inner level fp32 (Sec. 5) */
    int a2[4] = {OR_F64, OR_F32, OR_F32, OR_F32};
    int v2[4] = {OR_F64, OR_F32, OR_F32, OR_F32};
    memcpy(pA, a2, sizeof a2);
    memcpy(pv, v2, sizeof v2);
    p->pM = OR_F32;
  } else if (variant == 2) { /* fp64-F3R */
    for (int d = 0; d < 4; d++) pA[d] = pv[d] = OR_F64;
    p->pM = OR_F64;
  } else if (variant == 3) { /* FGMRES(64) + M in fp64, the comparison solver */
    p->nlev = 1;
    p->lev[0].m = 64;
    p->pM = OR_F64;
    p->max_outer = 19200;
  } else if (variant == 4) { /* fp16-F3R with bfloat16 in place of binary16 */
    pA[2] = pA[3] = OR_BF16;
    pv[3] = OR_BF16;
    p->pM = OR_BF16;
  }
  for (int d = 0; d < 4; d++) {
    p->lev[d].pA = pA[d];
    p->lev[d].pv = pv[d];
    p->lev[d].pacc = pv[d] == OR_F64 ? OR_F64 : OR_F32;
  }
}

void or_destroy(or_handle* h) {
  if (!h) return;
  free(h->rp);
  free(h->ci);
  free(h->a);
  free(h->s);
  free(h->ahat);
  for (int i = 0; i < 4; i++) free(h->alev[i]);
  free(h->wrp);
  free(h->wci);
  free(h->grp);
  free(h->gci);
  free(h->wv64);
  free(h->gv64);
  free(h->iv64);
  free(h->iv);
  free(h->idiag);
  free(h->wv);
  free(h->gv);
  free(h->mtmp);
  for (int d = 0; d < OR_MAX_LEV; d++) {
    level_ws* w = &h->ws[d];
    free(w->V);
    free(w->Z);
    free(w->H);
    free(w->Hraw);
    free(w->cs);
    free(w->sn);
    free(w->g);
    free(w->y);
    free(w->w);
    free(w->tmp0);
    free(w->tmp1);
    free(w->tmp2);
    free(w->tmp3);
    free(w->tmp4);
  }
  free(h->hist);
  for (int d = 0; d < OR_MAX_LEV; d++) free(h->lhist[d]);
  free(h->tr.v);
  free(h->tr.r);
  free(h->tr.tw);
  free(h->tr.y);
  free(h->tr.z);
  free(h->tr.ta);
  free(h);
}

static int alloc_level(or_handle* h, int d, int32_t m) {
  level_ws* w = &h->ws[d];
  int64_t n = h->n;
  free(w->V);
  free(w->Z);
  free(w->H);
  free(w->Hraw);
  free(w->cs);
  free(w->sn);
  free(w->g);
  free(w->y);
  w->m = m;
  w->V = xcalloc((int64_t)(m + 1) * n, sizeof(double));
  w->Z = xcalloc((int64_t)m * n, sizeof(double));
  w->H = xcalloc((int64_t)(m + 1) * m, sizeof(double));
  w->Hraw = xcalloc((int64_t)(m + 1) * m, sizeof(double));
  w->cs = xcalloc(m + 1, sizeof(double));
  w->sn = xcalloc(m + 1, sizeof(double));
  w->g = xcalloc(m + 2, sizeof(double));
  w->y = xcalloc(m + 1, sizeof(double));
  if (!w->w) w->w = xcalloc(n, sizeof(double));
  if (!w->tmp0) w->tmp0 = xcalloc(n, sizeof(double));
  if (!w->tmp1) w->tmp1 = xcalloc(n, sizeof(double));
  if (!w->tmp2) w->tmp2 = xcalloc(n, sizeof(double));
  if (!w->tmp3) w->tmp3 = xcalloc(n, sizeof(double));
  if (!w->tmp4) w->tmp4 = xcalloc(n, sizeof(double));
  return w->V && w->Z && w->H && w->Hraw && w->cs && w->sn && w->g && w->y &&
         w->w && w->tmp0 && w->tmp1 && w->tmp2 && w->tmp3 && w->tmp4;
}

static int validate(int64_t n, int64_t nnz, const int32_t* rp,
                    const int32_t* ci, const double* v) {
  if (n <= 0 || nnz < n || !rp || !ci || !v) return OR_ERR_ARG;
  if (rp[0] != 0 || rp[n] != nnz) return OR_ERR_MATRIX;
  for (int64_t i = 0; i < n; i++) {
    if (rp[i + 1] < rp[i]) return OR_ERR_MATRIX;
    int has_diag = 0;
    for (int64_t k = rp[i]; k < rp[i + 1]; k++) {
      if (ci[k] < 0 || ci[k] >= n) return OR_ERR_MATRIX;
      if (k > rp[i] && ci[k] <= ci[k - 1]) return OR_ERR_MATRIX;
      if (!isfinite(v[k])) return OR_ERR_MATRIX;
      if (ci[k] == i) {
        has_diag = 1;
        if (v[k] == 0.0) return OR_ERR_MATRIX;
      }
    }
    if (!has_diag) return OR_ERR_MATRIX;
  }
  return OR_OK;
}

/* M factors of the scaled matrix, built in fp64 (see the file header) */
static int build_m(or_handle* h) {
  int64_t n = h->n;
  double al = h->p.alpha;
  int64_t nl = 0, nu = 0;
  for (int64_t i = 0; i < n; i++)
    for (int64_t k = h->rp[i]; k < h->rp[i + 1]; k++) {
      if (h->ci[k] < i) nl++;
      if (h->ci[k] > i) nu++;
    }
  h->wnnz = nl + n;
  h->gnnz = nu + n;
  h->wrp = xcalloc(n + 1, sizeof(int32_t));
  h->grp = xcalloc(n + 1, sizeof(int32_t));
  h->wci = xcalloc(h->wnnz, sizeof(int32_t));
  h->gci = xcalloc(h->gnnz, sizeof(int32_t));
  h->wv64 = xcalloc(h->wnnz, sizeof(double));
  h->gv64 = xcalloc(h->gnnz, sizeof(double));
  h->wv = xcalloc(h->wnnz, sizeof(double));
  h->gv = xcalloc(h->gnnz, sizeof(double));
  h->mtmp = xcalloc(n, sizeof(double));
  if (!h->wrp || !h->grp || !h->wci || !h->gci || !h->wv64 || !h->gv64 ||
      !h->wv || !h->gv || !h->mtmp)
    return OR_ERR_NOMEM;
  int64_t pw = 0, pg = 0;
  for (int64_t i = 0; i < n; i++) {
    h->wrp[i] = (int32_t)pw;
    h->grp[i] = (int32_t)pg;
    /* W row i: strictly lower entries -ahat/alpha, then the unit diagonal */
    for (int64_t k = h->rp[i]; k < h->rp[i + 1]; k++)
      if (h->ci[k] < i) {
        h->wci[pw] = h->ci[k];
        h->wv64[pw++] = -h->ahat[k] / al;
      }
    h->wci[pw] = (int32_t)i;
    h->wv64[pw++] = 1.0;
    /* G row i: diagonal 1/alpha, then strictly upper entries (-ahat/alpha)/alpha */
    h->gci[pg] = (int32_t)i;
    h->gv64[pg++] = 1.0 / al;
    for (int64_t k = h->rp[i]; k < h->rp[i + 1]; k++)
      if (h->ci[k] > i) {
        h->gci[pg] = h->ci[k];
        h->gv64[pg++] = (-h->ahat[k] / al) / al;
      }
  }
  h->wrp[n] = (int32_t)pw;
  h->grp[n] = (int32_t)pg;
  for (int64_t k = 0; k < h->wnnz; k++) h->wv[k] = RND(h->p.pM, h->wv64[k]);
  for (int64_t k = 0; k < h->gnnz; k++) h->gv[k] = RND(h->p.pM, h->gv64[k]);
  return OR_OK;
}

/* Block-Jacobi ILU(0) (Sec. 5.1, the CPU experiments' primary
   preconditioner): rows split into `blocks` contiguous ranges of nearly equal
   size, the couplings between ranges dropped; each diagonal block of the
   scaled matrix, with its diagonal multiplied by alpha, is factored as
   L U keeping the sparsity of A (ILU(0)): for every row i in order, for each
   k < i of its pattern in increasing order, l_ik = a_ik / u_kk and then
   a_ij -= l_ik u_kj for every j > k of row i's pattern that row k also
   holds.  Built in fp64, then cast to pM. */
int64_t or_ilu_block_start(const or_handle* h, int64_t b) {
  return (b * h->n) / h->p.ilu_blocks;
}

static int64_t block_of(const or_handle* h, int64_t i) {
  /* largest b with start(b) <= i */
  int64_t b = (i * h->p.ilu_blocks) / h->n;
  while (b + 1 <= h->p.ilu_blocks && or_ilu_block_start(h, b + 1) <= i) b++;
  while (b > 0 && or_ilu_block_start(h, b) > i) b--;
  return b;
}

static int build_ilu(or_handle* h) {
  const int64_t n = h->n;
  h->iv64 = xcalloc(h->nnz, sizeof(double));
  h->iv = xcalloc(h->nnz, sizeof(double));
  h->idiag = xcalloc(n, sizeof(int32_t));
  if (!h->iv64 || !h->iv || !h->idiag) return OR_ERR_NOMEM;
  for (int64_t i = 0; i < n; i++) {
    const int64_t b = block_of(h, i);
    const int64_t r0 = or_ilu_block_start(h, b), r1 = or_ilu_block_start(h, b + 1);
    for (int64_t k = h->rp[i]; k < h->rp[i + 1]; k++) {
      const int64_t c = h->ci[k];
      if (c == i) {
        h->idiag[i] = (int32_t)(k - h->rp[i]);
        h->iv64[k] = h->p.alpha * h->ahat[k];
      } else {
        h->iv64[k] = (c >= r0 && c < r1) ? h->ahat[k] : 0.0;
      }
    }
  }
  double* v = h->iv64;
  for (int64_t i = 0; i < n; i++) {
    const int64_t b = block_of(h, i);
    const int64_t r0 = or_ilu_block_start(h, b);
    const int64_t lo = h->rp[i], hi = h->rp[i + 1];
    for (int64_t p = lo; p < hi; p++) {
      const int64_t k = h->ci[p];
      if (k >= i) break;
      if (k < r0) continue;  /* dropped coupling */
      const double ukk = v[h->rp[k] + h->idiag[k]];
      v[p] = v[p] / ukk;
      /* row i's entries right of k against row k's upper entries */
      int64_t q = h->rp[k] + h->idiag[k] + 1;
      for (int64_t pj = p + 1; pj < hi; pj++) {
        const int64_t j = h->ci[pj];
        while (q < h->rp[k + 1] && h->ci[q] < j) q++;
        if (q < h->rp[k + 1] && h->ci[q] == j) v[pj] = v[pj] - v[p] * v[q];
      }
    }
  }
  for (int64_t k = 0; k < h->nnz; k++) {
    if (!isfinite(v[k])) return OR_ERR_MATRIX;
    h->iv[k] = RND(h->p.pM, v[k]);
  }
  return OR_OK;
}

/* y = U^-1 L^-1 r per block, vectors stored in pv, arithmetic in q: the
   forward sweep forms t_i = r_i - sum_k l_ik t_k, the backward sweep
   y_i = (t_i - sum_j u_ij y_j) / u_ii, terms in column order, each product
   and difference rounded to q, t and y stored in pv. */
static void apply_ilu(or_handle* h, int32_t pv, int32_t q, int use64, const double* r,
                      double* y) {
  const int64_t n = h->n;
  const double* v = use64 ? h->iv64 : h->iv;
  double* t = h->mtmp;
  for (int64_t i = 0; i < n; i++) {
    const int64_t r0 = or_ilu_block_start(h, block_of(h, i));
    double acc = r[i];
    for (int64_t p = h->rp[i]; p < h->rp[i + 1] && h->ci[p] < i; p++)
      if (h->ci[p] >= r0) acc = RND(q, acc - RND(q, v[p] * t[h->ci[p]]));
    t[i] = RND(pv, acc);
  }
  for (int64_t i = n - 1; i >= 0; i--) {
    const int64_t r1 = or_ilu_block_start(h, block_of(h, i) + 1);
    const int64_t pd = h->rp[i] + h->idiag[i];
    double acc = t[i];
    for (int64_t p = pd + 1; p < h->rp[i + 1]; p++)
      if (h->ci[p] < r1) acc = RND(q, acc - RND(q, v[p] * y[h->ci[p]]));
    y[i] = RND(pv, RND(q, acc / v[pd]));
  }
}

void or_get_ilu_values(const or_handle* h, int32_t use64, double* vals) {
  if (!h->iv64) return;
  memcpy(vals, use64 ? h->iv64 : h->iv, (size_t)h->nnz * sizeof(double));
}

int32_t or_setup(int64_t n, int64_t nnz, const int32_t* rp, const int32_t* ci,
                 const double* val, const or_params* p, or_handle** out) {
  *out = NULL;
  if (!p || p->nlev < 1 || p->nlev > OR_MAX_LEV) return OR_ERR_ARG;
  if (p->lev[0].kind != OR_FGMRES) return OR_ERR_ARG;
  for (int d = 0; d < p->nlev; d++)
    if (p->lev[d].m < 1 || p->lev[d].m > (d == 0 ? 100000 : 64))
      return OR_ERR_ARG;
  if (!(p->alpha > 0.0)) return OR_ERR_ARG;
  if (p->m_kind != OR_M_SGS && p->m_kind != OR_M_ILU) return OR_ERR_ARG;
  if (p->m_kind == OR_M_ILU && (p->ilu_blocks < 1 || p->ilu_blocks > n)) return OR_ERR_ARG;
  int st = validate(n, nnz, rp, ci, val);
  if (st != OR_OK) return st;
  or_handle* h = calloc(1, sizeof(*h));
  if (!h) return OR_ERR_NOMEM;
  h->p = *p;
  h->n = n;
  h->nnz = nnz;
  h->rp = xcalloc(n + 1, sizeof(int32_t));
  h->ci = xcalloc(nnz, sizeof(int32_t));
  h->a = xcalloc(nnz, sizeof(double));
  h->s = xcalloc(n, sizeof(double));
  h->ahat = xcalloc(nnz, sizeof(double));
  if (!h->rp || !h->ci || !h->a || !h->s || !h->ahat) {
    or_destroy(h);
    return OR_ERR_NOMEM;
  }
  memcpy(h->rp, rp, (size_t)(n + 1) * sizeof(int32_t));
  memcpy(h->ci, ci, (size_t)nnz * sizeof(int32_t));
  memcpy(h->a, val, (size_t)nnz * sizeof(double));
  /* symmetric diagonal scaling (Sec. 5): s_i = 1/sqrt(|a_ii|),
     ahat_ij = (s_i a_ij) s_j */
  for (int64_t i = 0; i < n; i++)
    for (int64_t k = rp[i]; k < rp[i + 1]; k++)
      if (ci[k] == i) h->s[i] = 1.0 / sqrt(fabs(val[k]));
  for (int64_t i = 0; i < n; i++)
    for (int64_t k = rp[i]; k < rp[i + 1]; k++)
      h->ahat[k] = (h->s[i] * val[k]) * h->s[ci[k]];
  /* per-precision copies of Ahat, each rounded directly from fp64 (Table 1);
     only the precisions the nest uses are range-checked */
  int need[4] = {1, 0, 0, 0};
  for (int d = 0; d < p->nlev; d++) need[p->lev[d].pA] = 1;
  for (int q = 0; q < 4; q++) {
    h->alev[q] = xcalloc(nnz, sizeof(double));
    if (!h->alev[q]) {
      or_destroy(h);
      return OR_ERR_NOMEM;
    }
    for (int64_t k = 0; k < nnz; k++) {
      h->alev[q][k] = RND(q, h->ahat[k]);
      if (need[q] && !isfinite(h->alev[q][k])) {
        or_destroy(h);
        return OR_ERR_RANGE;
      }
    }
  }
  st = build_m(h);
  if (st == OR_OK && p->m_kind == OR_M_ILU) st = build_ilu(h);
  if (st != OR_OK) {
    or_destroy(h);
    return st;
  }
  for (int64_t k = 0; k < h->wnnz; k++)
    if (!isfinite(h->wv[k])) st = OR_ERR_RANGE;
  for (int64_t k = 0; k < h->gnnz; k++)
    if (!isfinite(h->gv[k])) st = OR_ERR_RANGE;
  if (st != OR_OK) {
    or_destroy(h);
    return st;
  }
  for (int d = 0; d < p->nlev; d++)
    if (!alloc_level(h, d, p->lev[d].m)) {
      or_destroy(h);
      return OR_ERR_NOMEM;
    }
  for (int d = 0; d < OR_MAX_LEV; d++) {
    h->cntr[d] = 1;
    for (int k = 0; k < 64; k++) h->omega[d][k] = p->omega_init;
  }
  h->hist_cap = 1024;
  h->hist = xcalloc(h->hist_cap, sizeof(double));
  *out = h;
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* basic operations                                                          */
/* ------------------------------------------------------------------------ */

/* y_i = round_pout( sum_k round_q(v_k x_{c_k}) ), summed left to right in q */
static void csr_mv(int64_t n, const int32_t* rp, const int32_t* ci,
                   const double* v, int32_t q, int32_t pout, const double* x,
                   double* y) {
  OR_PAR_FOR
  for (int64_t i = 0; i < n; i++) {
    double acc = 0.0;
    for (int64_t k = rp[i]; k < rp[i + 1]; k++)
      acc = RND(q, acc + RND(q, v[k] * x[ci[k]]));
    y[i] = RND(pout, acc);
  }
}

static double dot(int32_t q, int64_t n, const double* x, const double* y) {
  double acc = 0.0;
  for (int64_t i = 0; i < n; i++) acc = RND(q, acc + RND(q, x[i] * y[i]));
  return acc;
}

static double nrm2(int32_t q, int64_t n, const double* x) {
  return RND(q, sqrt(dot(q, n, x, x)));
}

/* Sum of round_q(x_i y_i) over i = lo .. hi-1 in precision q, in the order
   `order` (or_params.dot_order; the paper fixes no order for the dot
   products of the Gram-Schmidt step or of the weight, Secs. 4.2-4.3):
   0 left to right, 1 right to left, 2 / 4 / 5 / 6 blocks of 1024 / 64 /
   256 / 4096 elements each summed left to right and then the block sums
   left to right, 3 / 7 pairwise (halves summed recursively, runs of at
   most 8 / 32 left to right). */
static int64_t block_len(int32_t order) {
  return order == 4 ? 64 : order == 5 ? 256 : order == 6 ? 4096 : 1024;
}
static double dot_range(int32_t q, int32_t order, int64_t lo, int64_t hi,
                        const double* x, const double* y) {
  double acc = 0.0;
  if (order == 1) {
    for (int64_t i = hi - 1; i >= lo; i--) acc = RND(q, acc + RND(q, x[i] * y[i]));
  } else if (order == 2 || order == 4 || order == 5 || order == 6) {
    /* each block's sum alone (the blocks are independent), then the block
       sums in block order */
    int64_t bl = block_len(order);
    int64_t nblk = (hi - lo + bl - 1) / bl;
    double* bs = malloc((size_t)(nblk > 0 ? nblk : 1) * sizeof(double));
    if (!bs) return NAN;
    OR_PAR_FOR
    for (int64_t t = 0; t < nblk; t++) {
      int64_t b = lo + t * bl;
      int64_t e = b + bl < hi ? b + bl : hi;
      bs[t] = dot_range(q, 0, b, e, x, y);
    }
    for (int64_t t = 0; t < nblk; t++) acc = RND(q, acc + bs[t]);
    free(bs);
  } else if ((order == 3 && hi - lo > 8) || (order == 7 && hi - lo > 32)) {
    int64_t mid = lo + (hi - lo) / 2;
    acc = RND(q, dot_range(q, order, lo, mid, x, y) + dot_range(q, order, mid, hi, x, y));
  } else {
    for (int64_t i = lo; i < hi; i++) acc = RND(q, acc + RND(q, x[i] * y[i]));
  }
  return acc;
}
/* the dot products and norms of the level arithmetic, in the handle's order */
static double ldot(const or_handle* h, int32_t q, int64_t n, const double* x, const double* y) {
  return dot_range(q, h->p.dot_order, 0, n, x, y);
}
static double lnrm2(const or_handle* h, int32_t q, int64_t n, const double* x) {
  return RND(q, sqrt(ldot(h, q, n, x, x)));
}

static int all_finite(int64_t n, const double* x) {
  for (int64_t i = 0; i < n; i++)
    if (!isfinite(x[i])) return 0;
  return 1;
}

void or_spmv(const or_handle* h, int32_t scaled, int32_t pA, int32_t pacc,
             int32_t pout, const double* x, double* y) {
  const double* v = scaled ? h->alev[pA] : h->a;
  csr_mv(h->n, h->rp, h->ci, v, pacc, pout, x, y);
}

static void apply_m_impl(or_handle* h, int32_t pv, int32_t q, int use64,
                         const double* r, double* y) {
  h->st.m_calls++;
  if (h->p.m_identity) {
    for (int64_t i = 0; i < h->n; i++) y[i] = RND(pv, r[i]);
    return;
  }
  if (h->p.m_kind == OR_M_ILU) {
    apply_ilu(h, pv, q, use64, r, y);
    return;
  }
  const double* wv = use64 ? h->wv64 : h->wv;
  const double* gv = use64 ? h->gv64 : h->gv;
  /* t = W r, stored in pv; y = G t, stored in pv (two SpMVs, Sec. 5.2) */
  csr_mv(h->n, h->wrp, h->wci, wv, q, pv, r, h->mtmp);
  csr_mv(h->n, h->grp, h->gci, gv, q, pv, h->mtmp, y);
}

void or_apply_m(or_handle* h, int32_t pv, int32_t pacc, const double* r,
                double* y) {
  apply_m_impl(h, pv, pacc, 0, r, y);
}

/* number of invocations of level r made by one invocation of level e */
static int64_t calls_between(const or_handle* h, int e, int r) {
  int64_t c = 1;
  for (int k = e; k < r; k++) c *= h->p.lev[k].m;
  return c;
}

/* advance c_ntr of every Richardson level below d as if `iters` iterations
   of level d had run (see the breakdown reading in the file header) */
static void skip_calls(or_handle* h, int d, int64_t iters) {
  for (int r = d + 1; r < h->p.nlev; r++)
    if (h->p.lev[r].kind == OR_RICH)
      h->cntr[r] += iters * calls_between(h, d + 1, r);
}

static void apply_level_impl(or_handle* h, int d, const double* v, double* z);

/* preconditioner of level d applied to v (v and z in level d's precision) */
static void apply_prec(or_handle* h, int d, const double* v, double* z) {
  int64_t n = h->n;
  if (d == 0) {
    /* outermost: the inner nest runs on the scaled system, P(v) = S F2(S v) */
    double* t0 = h->ws[0].tmp0;
    double* t1 = h->ws[0].tmp1;
    OR_PAR_FOR
    for (int64_t i = 0; i < n; i++) t0[i] = h->s[i] * v[i];
    if (h->baseline || h->p.nlev == 1)
      apply_m_impl(h, OR_F64, OR_F64, h->baseline && h->base_m64, t0, t1);
    else
      apply_level_impl(h, 1, t0, t1);
    OR_PAR_FOR
    for (int64_t i = 0; i < n; i++) z[i] = h->s[i] * t1[i];
    return;
  }
  if (d + 1 < h->p.nlev)
    apply_level_impl(h, d + 1, v, z);
  else
    apply_m_impl(h, h->p.lev[d].pv, h->p.lev[d].pacc, 0, v, z);
}

static void lhist_push(or_handle* h, int d, double v) {
  if (h->lhist_len[d] == h->lhist_cap[d]) {
    int64_t cap = h->lhist_cap[d] ? 2 * h->lhist_cap[d] : 1024;
    double* nh = realloc(h->lhist[d], (size_t)cap * sizeof(double));
    if (!nh) return;
    h->lhist[d] = nh;
    h->lhist_cap[d] = cap;
  }
  h->lhist[d][h->lhist_len[d]++] = v;
}

/* ------------------------------------------------------------------------ */
/* FGMRES level (Sec. 4.2: classical Gram-Schmidt, Givens rotations)        */
/* ------------------------------------------------------------------------ */

/* One cycle of right-preconditioned FGMRES at level d on the system
   A_d u = vin with u0 = 0.  Writes u = sum_j y_j z_j to out.
   m: iterations; tolabs > 0 enables the outermost stopping test
   |g_{j+1}| < tolabs (with ||b|| folded into tolabs).  Returns iterations
   done; *bad is set when a non-finite value appears in the outermost
   level's own scalars. */
static int fgmres_cycle(or_handle* h, int d, const double* vin, int m,
                        double tolabs, double bnorm, double* out, int* bad) {
  int64_t n = h->n;
  level_ws* W = &h->ws[d];
  const or_level* L = &h->p.lev[d];
  int32_t p = L->pv, q = L->pacc;
  int M1 = W->m; /* leading dimension of H */
  double* w = W->w;
#define Vc(i) (W->V + (int64_t)(i) * n)
#define Zc(i) (W->Z + (int64_t)(i) * n)
#define Hh(i, j) (W->H[(i) + (int64_t)(j) * (M1 + 1)])
#define Hr(i, j) (W->Hraw[(i) + (int64_t)(j) * (M1 + 1)])
  *bad = 0;
  OR_PAR_FOR
  for (int64_t i = 0; i < n; i++) Vc(0)[i] = RND(p, vin[i]);
  double beta = lnrm2(h, q, n, Vc(0));
  W->beta = beta;
  W->meff = 0;
  if (beta == 0.0) {
    for (int64_t i = 0; i < n; i++) out[i] = 0.0;
    skip_calls(h, d, m);
    return 0;
  }
  OR_PAR_FOR
  for (int64_t i = 0; i < n; i++) Vc(0)[i] = RND(p, RND(q, Vc(0)[i] / beta));
  for (int j = 0; j <= m; j++) W->g[j] = 0.0;
  W->g[0] = beta;
  int meff = m;
  int done = 0;
  for (int j = 0; j < m; j++) {
    /* z_j = P(v_j) */
    apply_prec(h, d, Vc(j), Zc(j));
    if (!all_finite(n, Zc(j))) { /* identity fallback for a bad inner output */
      OR_PAR_FOR
      for (int64_t i = 0; i < n; i++) Zc(j)[i] = Vc(j)[i];
      h->st.fallbacks++;
    }
    /* w = A_d z_j */
    if (d == 0)
      csr_mv(n, h->rp, h->ci, h->a, OR_F64, OR_F64, Zc(j), w);
    else
      csr_mv(n, h->rp, h->ci, h->alev[L->pA], q, p, Zc(j), w);
    h->st.spmv[d]++;
    /* classical Gram-Schmidt: all h_ij from the same w */
    for (int i = 0; i <= j; i++) Hh(i, j) = ldot(h, q, n, w, Vc(i));
    OR_PAR_FOR
    for (int64_t k = 0; k < n; k++) {
      double acc = w[k];
      for (int i = 0; i <= j; i++) acc = RND(q, acc - RND(q, Hh(i, j) * Vc(i)[k]));
      w[k] = RND(p, acc);
    }
    double hn = lnrm2(h, q, n, w);
    for (int i = 0; i <= j; i++) Hr(i, j) = Hh(i, j);
    Hr(j + 1, j) = hn;
    /* apply the previous rotations to column j */
    for (int i = 0; i < j; i++) {
      double a0 = Hh(i, j), a1 = Hh(i + 1, j);
      Hh(i, j) = RND(q, RND(q, W->cs[i] * a0) + RND(q, W->sn[i] * a1));
      Hh(i + 1, j) = RND(q, RND(q, -W->sn[i] * a0) + RND(q, W->cs[i] * a1));
    }
    double rho = RND(q, hypot(Hh(j, j), hn));
    if (rho == 0.0 || !isfinite(rho)) {
      if (!isfinite(rho)) *bad = 1;
      meff = j;
      h->st.breakdowns++;
      skip_calls(h, d, m - j - 1);
      done = 1;
      break;
    }
    W->cs[j] = RND(q, Hh(j, j) / rho);
    W->sn[j] = RND(q, hn / rho);
    Hh(j, j) = rho;
    Hh(j + 1, j) = 0.0;
    W->g[j + 1] = RND(q, -W->sn[j] * W->g[j]);
    W->g[j] = RND(q, W->cs[j] * W->g[j]);
    if (d == 0) {
      double est = fabs(W->g[j + 1]) / bnorm;
      h->st.relres_est = est;
      if (h->hist_len == h->hist_cap) {
        double* nh = realloc(h->hist, (size_t)(2 * h->hist_cap) * sizeof(double));
        if (nh) {
          h->hist = nh;
          h->hist_cap *= 2;
        }
      }
      if (h->hist_len < h->hist_cap) h->hist[h->hist_len++] = est;
    } else {
      /* inner levels: the estimate relative to the invocation's input norm */
      lhist_push(h, d, fabs(W->g[j + 1]) / beta);
    }
    if (hn == 0.0) { /* exact breakdown: the subspace holds the solution */
      meff = j + 1;
      h->st.breakdowns++;
      skip_calls(h, d, m - j - 1);
      done = 1;
      break;
    }
    OR_PAR_FOR
    for (int64_t k = 0; k < n; k++) Vc(j + 1)[k] = RND(p, RND(q, w[k] / hn));
    if (tolabs > 0.0 && fabs(W->g[j + 1]) < tolabs) {
      meff = j + 1;
      done = 1;
      break;
    }
  }
  (void)done;
  /* back substitution R y = g */
  for (int i = meff - 1; i >= 0; i--) {
    double acc = W->g[i];
    for (int k = i + 1; k < meff; k++) acc = RND(q, acc - RND(q, Hh(i, k) * W->y[k]));
    W->y[i] = RND(q, acc / Hh(i, i));
  }
  /* u = Z y */
  OR_PAR_FOR
  for (int64_t k = 0; k < n; k++) {
    double acc = 0.0;
    for (int j = 0; j < meff; j++) acc = RND(q, acc + RND(q, W->y[j] * Zc(j)[k]));
    out[k] = RND(p, acc);
  }
  W->meff = meff;
  if (d == 0) h->last_m = meff;
  return meff;
#undef Vc
#undef Zc
#undef Hh
#undef Hr
}

/* ------------------------------------------------------------------------ */
/* Richardson with adaptive weights (Alg. 1, Eqs. (4)-(5))                   */
/* ------------------------------------------------------------------------ */

static void richardson(or_handle* h, int d, const double* vin, double* out) {
  int64_t n = h->n;
  const or_level* L = &h->p.lev[d];
  int32_t p = L->pv, q = L->pacc;
  level_ws* W = &h->ws[d];
  double* v = W->tmp0;
  double* z = W->tmp1;
  double* r = W->tmp2;
  double* y = W->tmp3;
  double* t = W->tmp4;
  double* om = h->omega[d];
  int64_t cn = h->cntr[d];
  int32_t c = h->p.c;
  if (cn == 1) /* the first call: omega_1 = ... = omega_m = 1 */
    for (int k = 0; k < L->m; k++) om[k] = RND(q, h->p.omega_init);
  OR_PAR_FOR
  for (int64_t i = 0; i < n; i++) v[i] = RND(p, vin[i]);
  OR_PAR_FOR
  for (int64_t i = 0; i < n; i++) z[i] = 0.0; /* z_0 = 0 */
  rich_trace* T = (h->tr.on && h->tr.d == d) ? &h->tr : NULL;
  if (T) {
    memcpy(T->v, v, (size_t)n * sizeof(double));
    T->steps = 0;
  }
  for (int k = 0; k < L->m; k++) {
    /* r_{k-1} = v - A z_{k-1}; r_0 = v without computation */
    if (k == 0) {
      OR_PAR_FOR
      for (int64_t i = 0; i < n; i++) r[i] = v[i];
    } else {
      csr_mv(n, h->rp, h->ci, h->alev[L->pA], q, q, z, t);
      h->st.spmv[d]++;
      OR_PAR_FOR
      for (int64_t i = 0; i < n; i++) r[i] = RND(p, RND(q, v[i] - t[i]));
    }
    /* y = M r_{k-1} (or the next level when R is not innermost) */
    apply_prec(h, d, r, y);
    int updated = 0;
    double om_before = om[k], wp_used = 0.0, num_k = 0.0, den_k = 0.0;
    int64_t l_k = 0;
    if (c > 0 && cn % c == 0) {
      /* omega'_k = (r, A M r) / (A M r, A M r), in fp32 (Sec. 4.3) */
      csr_mv(n, h->rp, h->ci, h->alev[L->pA], q, q, y, t);
      h->st.spmv[d]++;
      double num = ldot(h, q, n, r, t);
      double den = ldot(h, q, n, t, t);
      double wp = RND(q, num / den);
      num_k = num;
      den_k = den;
      if (T) memcpy(T->ta + (int64_t)k * n, t, (size_t)n * sizeof(double));
      if (den > 0.0 && isfinite(wp)) {
        OR_PAR_FOR
        for (int64_t i = 0; i < n; i++) z[i] = RND(p, RND(q, z[i] + RND(q, wp * y[i])));
        int64_t l = cn / c;
        om[k] = RND(q, RND(q, RND(q, (double)l * om[k]) + wp) / (double)(l + 1));
        updated = 1;
        wp_used = wp;
        l_k = l;
      }
    }
    if (!updated) {
      OR_PAR_FOR
      for (int64_t i = 0; i < n; i++) z[i] = RND(p, RND(q, z[i] + RND(q, om[k] * y[i])));
      wp_used = om[k];
    }
    if (T && k < 64) {
      memcpy(T->r + (int64_t)k * n, r, (size_t)n * sizeof(double));
      memcpy(T->tw + (int64_t)k * n, h->mtmp, (size_t)n * sizeof(double));
      memcpy(T->y + (int64_t)k * n, y, (size_t)n * sizeof(double));
      memcpy(T->z + (int64_t)k * n, z, (size_t)n * sizeof(double));
      double* sc = T->sc[k];
      sc[0] = updated;
      sc[1] = num_k;
      sc[2] = den_k;
      sc[3] = updated ? wp_used : 0.0;
      sc[4] = om_before;
      sc[5] = om[k];
      sc[6] = (double)l_k;
      sc[7] = wp_used;
      T->steps = k + 1;
    }
  }
  h->cntr[d] = cn + 1;
  h->st.r_calls++;
  OR_PAR_FOR
  for (int64_t i = 0; i < n; i++) out[i] = z[i];
  if (h->p.poison_call > 0 && h->st.r_calls == h->p.poison_call) out[0] = NAN;
}

static void apply_level_impl(or_handle* h, int d, const double* v, double* z) {
  const or_level* L = &h->p.lev[d];
  if (L->kind == OR_RICH) {
    richardson(h, d, v, z);
  } else {
    int bad = 0;
    fgmres_cycle(h, d, v, L->m, 0.0, 1.0, z, &bad);
  }
}

void or_apply_level(or_handle* h, int32_t d, const double* v, double* z) {
  if (d < 1 || d >= h->p.nlev) return;
  apply_level_impl(h, d, v, z);
}

/* ------------------------------------------------------------------------ */
/* outermost level with restarts                                              */
/* ------------------------------------------------------------------------ */

static void residual64(const or_handle* h, const double* b, const double* x,
                       double* r) {
  csr_mv(h->n, h->rp, h->ci, h->a, OR_F64, OR_F64, x, r);
  OR_PAR_FOR
  for (int64_t i = 0; i < h->n; i++) r[i] = b[i] - r[i];
}

static int32_t outer_solve(or_handle* h, const double* b, double* x,
                           double tol, int32_t m1, int32_t max_outer,
                           or_info* info) {
  int64_t n = h->n;
  memset(&h->st, 0, sizeof(h->st));
  h->hist_len = 0;
  for (int d = 0; d < OR_MAX_LEV; d++) h->lhist_len[d] = 0;
  if (!h->p.persist_weights)
    for (int d = 0; d < OR_MAX_LEV; d++) h->cntr[d] = 1;
  double* r = xcalloc(n, sizeof(double));
  double* u = xcalloc(n, sizeof(double));
  if (!r || !u) {
    free(r);
    free(u);
    return OR_ERR_NOMEM;
  }
  if (!h->p.use_x0)
    for (int64_t i = 0; i < n; i++) x[i] = 0.0;
  double bnorm = nrm2(OR_F64, n, b);
  int32_t status = OR_NOT_CONVERGED;
  if (bnorm == 0.0) {
    for (int64_t i = 0; i < n; i++) x[i] = 0.0;
    h->st.relres_true = 0.0;
    status = OR_OK;
  } else {
    residual64(h, b, x, r);
    double rel = nrm2(OR_F64, n, r) / bnorm;
    h->st.relres_true = rel;
    if (rel < tol) status = OR_OK;
    int outer = 0;
    while (status != OR_OK && outer < max_outer) {
      int len = m1 < max_outer - outer ? m1 : max_outer - outer;
      if (h->ws[0].m < len && !alloc_level(h, 0, len)) {
        status = OR_ERR_NOMEM;
        break;
      }
      int bad = 0;
      int it = fgmres_cycle(h, 0, r, len, tol * bnorm, bnorm, u, &bad);
      outer += it;
      if (bad || !all_finite(n, u)) {
        status = OR_ERR_BREAKDOWN;
        break;
      }
      OR_PAR_FOR
      for (int64_t i = 0; i < n; i++) x[i] = x[i] + u[i];
      residual64(h, b, x, r);
      rel = nrm2(OR_F64, n, r) / bnorm;
      h->st.relres_true = rel;
      if (rel < tol) {
        status = OR_OK;
        break;
      }
      h->st.restarts++;
      if (it == 0) break; /* zero residual direction: nothing more to do */
    }
    h->st.outer_iters = outer;
  }
  free(r);
  free(u);
  h->st.status = status;
  if (info) *info = h->st;
  return status;
}

int32_t or_solve(or_handle* h, const double* b, double* x, double tol,
                 or_info* info) {
  if (!h || !b || !x || !(tol > 0.0)) return OR_ERR_ARG;
  h->baseline = 0;
  return outer_solve(h, b, x, tol, h->p.lev[0].m, h->p.max_outer, info);
}

int32_t or_fgmres_solve(or_handle* h, const double* b, double* x, double tol,
                        int32_t m, int32_t max_iter, int32_t m64, or_info* info) {
  if (!h || !b || !x || !(tol > 0.0) || m < 1 || max_iter < 1)
    return OR_ERR_ARG;
  h->baseline = 1;
  h->base_m64 = m64 != 0;
  int32_t st = outer_solve(h, b, x, tol, m, max_iter, info);
  h->baseline = 0;
  return st;
}

/* ------------------------------------------------------------------------ */
/* comparison solvers of Sec. 5: preconditioned CG (symmetric matrices) and  */
/* BiCGStab (nonsymmetric), every value fp64, with the preconditioner        */
/* P(v) = S M (S v) -- the diagonal scaling of Sec. 5 around the primary     */
/* preconditioner, whose factors are stored in the handle's pM (or fp64).    */
/* ------------------------------------------------------------------------ */

static void hist_push(or_handle* h, double v) {
  if (h->hist_len == h->hist_cap) {
    double* nh = realloc(h->hist, (size_t)(2 * h->hist_cap) * sizeof(double));
    if (nh) {
      h->hist = nh;
      h->hist_cap *= 2;
    }
  }
  if (h->hist_len < h->hist_cap) h->hist[h->hist_len++] = v;
}

/* z = S M (S r), fp64 arithmetic, M factors in fp64 (m64) or in pM */
static void apply_p64(or_handle* h, int m64, const double* r, double* z, double* tmp) {
  for (int64_t i = 0; i < h->n; i++) tmp[i] = h->s[i] * r[i];
  apply_m_impl(h, OR_F64, OR_F64, m64, tmp, z);
  for (int64_t i = 0; i < h->n; i++) z[i] = h->s[i] * z[i];
}

static double relres_of(or_handle* h, const double* b, const double* x, double* r, double bn) {
  csr_mv(h->n, h->rp, h->ci, h->a, OR_F64, OR_F64, x, r);
  for (int64_t i = 0; i < h->n; i++) r[i] = b[i] - r[i];
  return nrm2(OR_F64, h->n, r) / bn;
}

int32_t or_krylov_solve(or_handle* h, int32_t method, int32_t m64, const double* b, double* x,
                        double tol, int32_t max_iter, or_info* info) {
  if (!h || !b || !x || !(tol > 0.0) || max_iter < 1 || (method != 0 && method != 1))
    return OR_ERR_ARG;
  const int64_t n = h->n;
  memset(info, 0, sizeof(*info));
  memset(&h->st, 0, sizeof(h->st));
  h->hist_len = 0;
  for (int d = 0; d < OR_MAX_LEV; d++) h->lhist_len[d] = 0;
  enum { NW = 10 };
  double* w[NW];
  for (int k = 0; k < NW; k++) w[k] = xcalloc((size_t)n, sizeof(double));
  double *r = w[0], *z = w[1], *p = w[2], *q = w[3], *tmp = w[4];
  double *rh = w[5], *v = w[6], *t = w[7], *ps = w[8], *sv = w[9];
  if (!h->p.use_x0) memset(x, 0, (size_t)n * sizeof(double));
  const double bn = nrm2(OR_F64, n, b);
  int32_t status = OR_NOT_CONVERGED;
  int it = 0;
  double rel = 0.0;
  if (bn == 0.0) {
    memset(x, 0, (size_t)n * sizeof(double));
    status = OR_OK;
  } else if (method == 0) {
    /* preconditioned conjugate gradients */
    rel = relres_of(h, b, x, r, bn);
    apply_p64(h, m64, r, z, tmp);
    memcpy(p, z, (size_t)n * sizeof(double));
    double rz = dot(OR_F64, n, r, z);
    while (rel >= tol && it < max_iter) {
      csr_mv(n, h->rp, h->ci, h->a, OR_F64, OR_F64, p, q);
      const double alpha = rz / dot(OR_F64, n, p, q);
      for (int64_t i = 0; i < n; i++) {
        x[i] = x[i] + alpha * p[i];
        r[i] = r[i] - alpha * q[i];
      }
      it++;
      rel = nrm2(OR_F64, n, r) / bn;
      hist_push(h, rel);
      if (!isfinite(rel)) break;
      if (rel < tol) {
        /* confirm with the true residual; continue from it otherwise */
        rel = relres_of(h, b, x, r, bn);
        if (rel < tol) break;
      }
      apply_p64(h, m64, r, z, tmp);
      const double rz1 = dot(OR_F64, n, r, z);
      const double beta = rz1 / rz;
      rz = rz1;
      for (int64_t i = 0; i < n; i++) p[i] = z[i] + beta * p[i];
    }
  } else {
    /* right-preconditioned BiCGStab; the preconditioned vectors P p and
       P s are the ones added to x */
    rel = relres_of(h, b, x, r, bn);
    memcpy(rh, r, (size_t)n * sizeof(double));
    double rho = 1.0, alpha = 1.0, omega = 1.0;
    while (rel >= tol && it < max_iter) {
      const double rho1 = dot(OR_F64, n, rh, r);
      const double beta = (rho1 / rho) * (alpha / omega);
      rho = rho1;
      for (int64_t i = 0; i < n; i++) p[i] = r[i] + beta * (p[i] - omega * v[i]);
      apply_p64(h, m64, p, z, tmp); /* z = P p */
      csr_mv(n, h->rp, h->ci, h->a, OR_F64, OR_F64, z, v);
      alpha = rho / dot(OR_F64, n, rh, v);
      for (int64_t i = 0; i < n; i++) sv[i] = r[i] - alpha * v[i];
      it++;
      const double srel = nrm2(OR_F64, n, sv) / bn;
      if (srel < tol) {
        /* the half step already meets the tolerance */
        for (int64_t i = 0; i < n; i++) x[i] = x[i] + alpha * z[i];
        rel = relres_of(h, b, x, r, bn);
        hist_push(h, rel);
        if (rel < tol || !isfinite(rel)) break;
        continue;
      }
      apply_p64(h, m64, sv, ps, tmp); /* P s */
      csr_mv(n, h->rp, h->ci, h->a, OR_F64, OR_F64, ps, t);
      omega = dot(OR_F64, n, t, sv) / dot(OR_F64, n, t, t);
      for (int64_t i = 0; i < n; i++) {
        x[i] = x[i] + alpha * z[i] + omega * ps[i];
        r[i] = sv[i] - omega * t[i];
      }
      rel = nrm2(OR_F64, n, r) / bn;
      hist_push(h, rel);
      if (!isfinite(rel)) break;
      if (rel < tol) {
        rel = relres_of(h, b, x, r, bn);
        if (rel < tol) break;
      }
    }
  }
  if (bn != 0.0) {
    rel = relres_of(h, b, x, r, bn);
    if (!isfinite(rel)) status = OR_ERR_BREAKDOWN;
    else if (rel < tol) status = OR_OK;
  }
  for (int k = 0; k < NW; k++) free(w[k]);
  info->status = status;
  info->outer_iters = it;
  info->m_calls = h->st.m_calls;
  info->relres_true = rel;
  info->relres_est = h->hist_len ? h->hist[h->hist_len - 1] : rel;
  return status;
}

/* ------------------------------------------------------------------------ */
/* accessors                                                                 */
/* ------------------------------------------------------------------------ */

void or_get_scaling(const or_handle* h, double* s) {
  memcpy(s, h->s, (size_t)h->n * sizeof(double));
}
void or_get_level_values(const or_handle* h, int32_t p, double* vals) {
  if (p < 0 || p > 3) return;
  memcpy(vals, h->alev[p], (size_t)h->nnz * sizeof(double));
}
int64_t or_m_nnz_lower(const or_handle* h) { return h->wnnz; }
int64_t or_m_nnz_upper(const or_handle* h) { return h->gnnz; }
void or_get_m_factors(const or_handle* h, int32_t* wrp, int32_t* wci,
                      double* wv, int32_t* grp, int32_t* gci, double* gv) {
  memcpy(wrp, h->wrp, (size_t)(h->n + 1) * sizeof(int32_t));
  memcpy(grp, h->grp, (size_t)(h->n + 1) * sizeof(int32_t));
  memcpy(wci, h->wci, (size_t)h->wnnz * sizeof(int32_t));
  memcpy(gci, h->gci, (size_t)h->gnnz * sizeof(int32_t));
  memcpy(wv, h->wv, (size_t)h->wnnz * sizeof(double));
  memcpy(gv, h->gv, (size_t)h->gnnz * sizeof(double));
}
void or_get_weights(const or_handle* h, int32_t d, double* omega,
                    int64_t* cntr) {
  if (d < 0 || d >= OR_MAX_LEV) return;
  for (int k = 0; k < h->p.lev[d].m && k < 64; k++) omega[k] = h->omega[d][k];
  *cntr = h->cntr[d];
}
void or_set_weights(or_handle* h, int32_t d, const double* omega,
                    int64_t cntr) {
  if (d < 0 || d >= OR_MAX_LEV) return;
  /* the weights are quantities of the level arithmetic (fp32 for narrow
     levels, Sec. 4.3) */
  for (int k = 0; k < h->p.lev[d].m && k < 64; k++)
    h->omega[d][k] = RND(h->p.lev[d].pacc, omega[k]);
  h->cntr[d] = cntr;
}
int64_t or_history(const or_handle* h, double* buf, int64_t cap) {
  int64_t k = h->hist_len < cap ? h->hist_len : cap;
  if (buf) memcpy(buf, h->hist, (size_t)k * sizeof(double));
  return h->hist_len;
}
int64_t or_level_history(const or_handle* h, int32_t d, double* buf, int64_t cap) {
  if (d == 0) return or_history(h, buf, cap);
  if (d < 0 || d >= OR_MAX_LEV) return 0;
  int64_t k = h->lhist_len[d] < cap ? h->lhist_len[d] : cap;
  if (buf && k > 0) memcpy(buf, h->lhist[d], (size_t)k * sizeof(double));
  return h->lhist_len[d];
}
int32_t or_trace(or_handle* h, int32_t d, int32_t on) {
  rich_trace* T = &h->tr;
  free(T->v);
  free(T->r);
  free(T->tw);
  free(T->y);
  free(T->z);
  free(T->ta);
  memset(T, 0, sizeof(*T));
  if (!on || d < 1 || d >= h->p.nlev || h->p.lev[d].kind != OR_RICH) return OR_OK;
  int64_t n = h->n, m = h->p.lev[d].m;
  if (m > 64) return OR_ERR_ARG;
  T->v = xcalloc(n, sizeof(double));
  T->r = xcalloc(m * n, sizeof(double));
  T->tw = xcalloc(m * n, sizeof(double));
  T->y = xcalloc(m * n, sizeof(double));
  T->z = xcalloc(m * n, sizeof(double));
  T->ta = xcalloc(m * n, sizeof(double));
  if (!T->v || !T->r || !T->tw || !T->y || !T->z || !T->ta) return OR_ERR_NOMEM;
  T->on = 1;
  T->d = d;
  T->m = (int32_t)m;
  return OR_OK;
}
int32_t or_rich_trace(const or_handle* h, double* v, double* r, double* tw,
                      double* y, double* z, double* ta, double* sc) {
  const rich_trace* T = &h->tr;
  if (!T->on) return 0;
  int64_t n = h->n, k = T->steps;
  memcpy(v, T->v, (size_t)n * sizeof(double));
  memcpy(r, T->r, (size_t)(k * n) * sizeof(double));
  memcpy(tw, T->tw, (size_t)(k * n) * sizeof(double));
  memcpy(y, T->y, (size_t)(k * n) * sizeof(double));
  memcpy(z, T->z, (size_t)(k * n) * sizeof(double));
  memcpy(ta, T->ta, (size_t)(k * n) * sizeof(double));
  memcpy(sc, T->sc, (size_t)k * 8 * sizeof(double));
  return (int32_t)k;
}
int32_t or_level_cycle(const or_handle* h, int32_t d, double* V, double* Z,
                       double* H, double* g, double* y, double* beta) {
  if (d < 0 || d >= h->p.nlev || h->p.lev[d].kind != OR_FGMRES) return -1;
  const level_ws* W = &h->ws[d];
  int32_t m = W->meff;
  int64_t n = h->n;
  memcpy(V, W->V, (size_t)(m + 1) * (size_t)n * sizeof(double));
  memcpy(Z, W->Z, (size_t)m * (size_t)n * sizeof(double));
  for (int j = 0; j < m; j++)
    for (int i = 0; i <= m; i++)
      H[i + (int64_t)j * (m + 1)] = W->Hraw[i + (int64_t)j * (W->m + 1)];
  memcpy(g, W->g, (size_t)(m + 1) * sizeof(double));
  memcpy(y, W->y, (size_t)m * sizeof(double));
  *beta = W->beta;
  return m;
}
int32_t or_last_cycle(const or_handle* h, double* V, double* Z, double* H,
                      int32_t cap_m) {
  int32_t m = h->last_m < cap_m ? h->last_m : cap_m;
  const level_ws* W = &h->ws[0];
  int64_t n = h->n;
  memcpy(V, W->V, (size_t)(m + 1) * (size_t)n * sizeof(double));
  memcpy(Z, W->Z, (size_t)m * (size_t)n * sizeof(double));
  for (int j = 0; j < m; j++)
    for (int i = 0; i <= m; i++)
      H[i + (int64_t)j * (m + 1)] = W->Hraw[i + (int64_t)j * (W->m + 1)];
  return m;
}
