// Host-side declarations of the kernel launchers of libf3r (gfx950).
// Every launcher enqueues work on `st` and returns the hipError_t of the
// launch.  Vector arguments are device pointers; "type" tags say how a
// vector is stored.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace f3r {

enum TypeTag { T64 = 0, T32 = 1, T16 = 2, TB16 = 3 };
inline size_t type_size(int t) { return t == T64 ? 8 : t == T32 ? 4 : 2; }
// arithmetic of a level whose vectors are stored in `t` (Table 1 policy)
inline int q_of(int t) { return t == T64 ? T64 : T32; }

// SELL-64 sparse structure shared by every value array of one matrix:
// slice s holds rows [64 s, 64 s + 64); entry k of its row r is stored at
// off[s] + 64 k + (r mod 64) (column-major inside the slice, so a wave
// reads 64 consecutive elements per k).  Entries are in CSR column order;
// rows are padded to the slice width with value 0 and the row's own column.
// idx holds int16 offsets col - row when every offset fits, else int32
// columns.  kd[r] is the position of the diagonal inside row r; kdr[s] packs
// the smallest (low 16 bits) and largest (high 16 bits) kd of slice s.
// Several independent systems can share one descriptor as the diagonal
// blocks of one matrix: system s owns the rows of the 1024-row blocks
// [b0[s], b0[s+1]) (its rows padded with identity rows to a multiple of
// 1024), and its device state (level scalars, flags, weights) sits at
// s * dS doubles and s * dI ints from system 0's.  Every kernel offsets the
// state pointers it is given by the system of its rows; reductions are
// summed per system.  One system: blk = b0 = nullptr.
constexpr int kSysAlign = 1024;  // rows of one reduction block; systems start at multiples

struct SysLayout {
  const int* blk = nullptr;  // system of each 1024-row block
  const int* b0 = nullptr;   // first 1024-row block of each system, nsys + 1 entries
  int nsys = 1;
  int64_t dS = 0, dI = 0;
};

struct IluDesc;  // block-Jacobi ILU(0) schedule (ilu.h)

// Diagonal-aligned variant (dell_w > 0): every slice has width dell_w and
// entry j of row r sits at position dell_kd - (lower entries of r) + j, so
// the diagonal of every row is at position dell_kd; the positions before a
// row's first entry and after its last are padding (value 0, the row's own
// column).  off, kd (= dell_kd) and kdr (= dell_kd | dell_kd << 16) are
// filled consistently, so code that reads them computes the same sums; the
// kernels take the widths and bounds from dell_w/dell_kd instead, which
// removes the dependent loads before the first entry load of a wave.
//
// Slice-offset variant (idx16 = 2, also diagonal-aligned): position k of
// every row of slice s has the same column offset, idx[s * dell_w + k]
// (int32), the sorted offsets of the slice's rows below the diagonal ending
// at dell_kd - 1 and those above it starting at dell_kd + 1; a row without
// an entry at an offset holds value 0 there (its column, when outside the
// matrix, replaced by the row's own).  No per-entry index is stored.
struct SellDesc {
  int64_t n = 0, ns = 0;
  const uint32_t* off = nullptr;
  const void* idx = nullptr;
  int idx16 = 0;  // 0: int32 columns, 1: int16 offsets, 2: offsets per slice
  const uint16_t* kd = nullptr;
  const uint32_t* kdr = nullptr;
  SysLayout sys;
  int dell_w = 0, dell_kd = 0;
  // host pointer: when set, M is block-Jacobi ILU(0) and the M launchers run
  // its triangular sweeps (never read on the device)
  const IluDesc* ilu = nullptr;
};

__host__ __device__ inline int64_t n_slices(int64_t n) { return (n + 63) / 64; }
// blocks of a row-parallel kernel: 16 slices (1024 rows) per block
__host__ __device__ inline int64_t n_blocks(int64_t n) { return (n_slices(n) + 15) / 16; }
// blocks of a sweep with kr rows per lane: 4 kr slices per block
__host__ __device__ inline int64_t n_blocks_kr(int64_t n, int kr) {
  return (n_slices(n) + 4 * kr - 1) / (4 * kr);
}

// A basis vector held lazily normalised: value_i = raw_i * (*scale) (times
// s_i when s != nullptr), rounded to the consumer's storage type.
struct Basis {
  const void* raw = nullptr;
  int type = T64;
  const double* scale = nullptr;
  const double* s = nullptr;
  const int* cur = nullptr;  // when set: raw/scale are bases indexed by *cur
  int64_t stride = 0;        // elements between consecutive basis vectors
};

// ---- level SpMV + classical Gram-Schmidt dots ----------------------------
// y = A x (values `av` of type ta, x of type tx, y of type ty, arithmetic
// q = q_of(ty)); then partial sums of (y, V_l) for l < nv where V_0 = v0 and
// V_l = vb + (l-1) n.  Partials (type q) at partials[l * nb + block].
// When fb && *fb, the input x is replaced by the basis `alt`.
hipError_t spmv_dots(hipStream_t st, const SellDesc& A, const void* av, int ta,
                     const void* x, int tx, const Basis* alt, const int* fb,
                     void* y, int ty, const void* v0, const void* vb, int nv,
                     void* partials, const int* stop);

// dst[l] = round_q(sum_b partials[l nb + b] * (scales ? scales[l] : 1)),
// one block per l; dst entries are doubles holding q values.
hipError_t finalize_sums(hipStream_t st, const SysLayout& sl, int q, const void* partials,
                         int64_t nb, int count, const double* scales, double* dst,
                         const int* stop);

// w_i <- round(w_i - sum_l round(h_l * round(raw_l,i * scale_l))) and partial
// sums of w_i^2 at partials[b].
hipError_t axpy_norm(hipStream_t st, const SysLayout& sl, int64_t n, void* w, int tw,
                     const void* v0, const void* vb, int nv, const double* h,
                     const double* scales, void* partials, const int* stop);

// The dot finalisation and the update in one kernel, for one system and
// 1 <= nv <= 16: hcol[l] = round_q(sum_b dot_partials[l dnb + b] * scales[l])
// (summed in the order finalize_sums uses, so bit for bit its result), then
// the update and squared norm of axpy_norm, whose *nnb partials (one per
// 8,192 rows) go to norm_partials, which must not overlap the dot partials.
hipError_t axpy_norm_fin(hipStream_t st, int64_t n, void* w, int tw, const void* v0, const void* vb,
                         int nv, const void* dot_partials, int64_t dnb, const double* scales,
                         double* hcol, void* norm_partials, int64_t* nnb, const int* stop);

// Layout of the device scalars of one FGMRES level (doubles).
struct LevelLayout {
  int m = 0;
  int64_t H = 0, Hraw = 0, cs = 0, sn = 0, g = 0, y = 0, scale = 0, beta = 0,
          cbeta = 0, total = 0;
  void init(int mm) {
    m = mm;
    int64_t o = 0;
    H = o; o += (int64_t)(m + 1) * m;
    Hraw = o; o += (int64_t)(m + 1) * m;
    cs = o; o += m;
    sn = o; o += m;
    g = o; o += m + 1;
    y = o; o += m;
    scale = o; o += m + 1;
    beta = o; o += 1;
    cbeta = o; o += 1;
    total = o;
  }
};
// ints of one FGMRES level
// I_HOLD (outermost level): the system has finished and its rows are skipped
// I_HLEN (inner levels): residual estimates recorded in the level's history
enum { I_MEFF = 0, I_STOP = 1, I_CUR = 2, I_BAD = 3, I_FALLBACKS = 4, I_BREAKDOWNS = 5, I_HOLD = 6,
       I_HLEN = 7, I_FB = 8 };
inline int level_ints(int m) { return I_FB + m + 8; }

struct ChildInit {  // state of a child FGMRES level reset by its parent
  double* S = nullptr;
  int* I = nullptr;
  int m = 0;
  int64_t g = 0, scale = 0;
  int64_t beta = -1;  // slot keeping the input norm of the call (-1: none)
};

// Residual history of an inner FGMRES level: after each Givens step,
// |g_{j+1}| / beta (beta = the norm of the call's input) is appended at
// p[I[I_HLEN]++] while I_HLEN < cap.
struct HistOut {
  double* p = nullptr;
  int64_t cap = 0;
};

// Givens step j of a level whose arithmetic is q (one block):
// h_{j+1,j} = sqrt(sum partials); rotations; g; scale_{j+1} = 1/h_{j+1,j};
// breakdown/stop handling; when solve_y, back-substitution R y = g.
// host_out (pinned host, outermost only; 4 words per system): [0] =
// |g_{j+1}| / ||b|| with inv_bnorm[s] = 1 / ||b_s||, [1] flags; with tol > 0
// a system whose estimate is below tol stops.  One block per system.
hipError_t givens(hipStream_t st, const SysLayout& sl, int q, const void* partials, int64_t nb,
                  double* S, int* I, const LevelLayout& L, int j, int solve_y,
                  const double* inv_bnorm, double* host_out, const ChildInit* child,
                  double tol = 0.0, HistOut hist = HistOut{});

hipError_t backsolve(hipStream_t st, const SysLayout& sl, int q, double* S, int* I,
                     const LevelLayout& L);

// The basis of one FGMRES level: V_0 = v0, V_j = vb + (j-1) n, each held
// lazily normalised by scales[j].
struct LevelBasis {
  const void* v0 = nullptr;
  const void* vb = nullptr;
  int type = T64;
  const double* scales = nullptr;
};

// Output of a level with vectors stored in tv:
// u_i = round_tv(sum_{j < meff} round(y_j Z_j,i)).  With s: out_i = s_i u_i
// in fp64; with accumulate: out_i += u_i; otherwise out_i = u_i (type tv).
// When `cur` is set the output vector is out + (*cur) n.  fb: per-column
// flags; a flagged column uses the basis vector V_j instead of Z_j.
// Rows of systems whose pstop flag is set are left alone.  m: the level's
// restart length (Z holds m columns, y m entries; meff <= m).
hipError_t combine(hipStream_t st, const SysLayout& sl, int64_t n, const void* Z, int tz,
                   int tv, const double* y, const int* meff, int m, void* out, const double* s,
                   const int* cur, int accumulate, const LevelBasis* alt,
                   const int* fb, int* out_fb, const int* pstop);

// Entry of an FGMRES level: out = round_to(to, basis value) and partial
// sums of out^2 (arithmetic q_of(to)); then the level state is reset with
// beta = ||out||.
hipError_t entry_cast(hipStream_t st, const SysLayout& sl, int64_t n, const Basis& in,
                      void* out, int to, void* partials, const int* parent_stop);
hipError_t entry_finalize(hipStream_t st, const SysLayout& sl, int q, const void* partials,
                          int64_t nb, const ChildInit& lev, const ChildInit* child,
                          const int* parent_stop);
// state of an aliased child for its first call: scale_0 and beta of the
// level's own V_0, stop flag copied
hipError_t child_init0(hipStream_t st, const SysLayout& sl, double* S, int* I,
                       const LevelLayout& L, const ChildInit& child);

// outermost: r = b - A x (fp64) into r, partial sums of r^2
hipError_t residual64(hipStream_t st, const SellDesc& A, const double* a64,
                      const double* x, const double* b, double* r, void* partials);
// per system: beta = ||r||; S.scale[0], S.g, I (meff, stop, cur, bad) reset;
// host_out[4 s] = beta * inv_bnorm[s], host_out[4 s + 2] = beta.  A held
// system (I[I_HOLD]) stays stopped.
hipError_t residual_finalize(hipStream_t st, const SysLayout& sl, const void* partials,
                             int64_t nb, double* S, int* I, const LevelLayout& L,
                             const double* inv_bnorm, double* host_out);
// partial sums of x_i y_i (fp64), then the sum of system s into host_out[4 s]
hipError_t dot64_to_host(hipStream_t st, const SysLayout& sl, int64_t n, const double* x,
                         const double* y, void* partials, double* host_out);

// ---- primary preconditioner M = G W (two SpMVs) and Richardson ------------
// t = round(u_i + sum_{k < kd} w_k u_c): W = I - L/alpha; `mv` (type tm) are
// the W values, or the scaled matrix negated when neg = 1.  The input u is
// a stored vector (`in.raw`, type in.type == tt, scale == nullptr) or a basis.
// cntr_inc (nullable): the Richardson call counter, advanced by one even when
// the call is skipped.  kr: sweep shape 10 KR + U (KR rows per lane, entry
// chunks of U: 18, 24, 44, and 23, 43 for narrow vectors); the result does
// not depend on it.
hipError_t m_apply_w(hipStream_t st, const SellDesc& A, const void* mv, int tm, int neg,
                     const Basis& in, void* t, int tt, const int* stop, int64_t* cntr_inc,
                     int kr = 44);

// With A.ilu set, m_apply_w is the forward sweep t = L^-1 r and m_apply_g
// the backward sweep y = U^-1 t, which overwrites t with y.
// y = round(gd t_i + sum_{k > kd} g_k t_c): G = (1/alpha)(I - U/alpha).
// mode 0: out = y; 1: out = round(w y); 2: out = round(zprev + w y) with
// w = *omega; 3: out = s_i y (fp64 output, s scaling of the comparison solver).
// fbflag (nullable): set to 1 when an output value is not finite.
hipError_t m_apply_g(hipStream_t st, const SellDesc& A, const void* mv, int tm, int neg,
                     double gd, const void* t, int tt, int mode, const double* omega,
                     const void* zprev, void* out, int tout, const double* s,
                     int* fbflag, const int* stop, const int* cur = nullptr, int kr = 44);

// r = round(u_i - sum_k a_k z_c) with u given by `in` (basis) and z stored.
hipError_t rich_residual(hipStream_t st, const SellDesc& A, const void* av, int ta,
                         const Basis& in, const void* z, void* r, int tr, const int* stop,
                         int kr = 44);
// t = A y kept in q; partials [0] = sum r_i t_i, [1] = sum t_i t_i; r given
// by `rin` (a basis, or a stored vector with scale == nullptr).
hipError_t rich_tdots(hipStream_t st, const SellDesc& A, const void* av, int ta,
                      const void* y, int ty, const Basis& rin, void* partials,
                      const int* stop);
// omega' = num / den; running mean of Eq. (5) with l = c_ntr / c, where the
// device counter holds c_ntr + 1 during the call
hipError_t rich_omega(hipStream_t st, const SysLayout& sl, int q, const void* partials,
                      int64_t nb, double* omega_k, double* wcur, const int64_t* cntr, int c,
                      const int* stop);
// advances a Richardson level's call counter by one (a level whose
// preconditioner is the next level; the innermost level's W sweep does it)
hipError_t cntr_advance(hipStream_t st, int64_t* cntr);
// z = round(zprev + w y) (zprev may be null), w = *wcur
hipError_t rich_zupdate(hipStream_t st, const SysLayout& sl, int64_t n, const void* zprev,
                        const void* y, int tr, const double* wcur, void* z, int* fbflag,
                        const int* stop);

// ---- stacked systems: caller vectors <-> the stacked vector ---------------
struct StackIo {
  SysLayout sl;
  const int64_t* row0 = nullptr;   // first row of each system (device)
  const int64_t* nrows = nullptr;  // rows of each system (device)
  double* const* ptrs = nullptr;   // the caller's vector of each system (device array)
  int64_t n = 0;                   // stacked rows
};
// cat_i = ptrs[s][i - row0[s]] on the rows of system s, 0 on its padding
hipError_t stack_gather(hipStream_t st, const StackIo& io, double* cat);
// ptrs[s][i - row0[s]] = cat_i
hipError_t stack_scatter(hipStream_t st, const StackIo& io, const double* cat);

// ---- small utilities -------------------------------------------------------
hipError_t convert(hipStream_t st, int64_t n, const void* in, int ti, void* out, int to);
hipError_t fill_nan(hipStream_t st, void* p, int t, int64_t count, int* flag);
hipError_t set_omega(hipStream_t st, const SysLayout& sl, double* omega, int m, double v);
// I[I_HOLD] = I[I_STOP] = 1 for the systems s with mask[s] != 0 (mask:
// device, nsys ints; I: the outermost level's flags)
hipError_t sys_hold(hipStream_t st, const SysLayout& sl, int* I, const int* mask);

}  // namespace f3r
