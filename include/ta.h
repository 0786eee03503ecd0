/*
 * ta.h -- C ABI of libta.so: elementwise piecewise trigonometric
 * approximations (Goyal & Arora, arXiv 2502.10831) on AMD Instinct MI355X
 * (gfx950) device arrays.
 *
 * The method (Section 2 of the paper, derived in Appendix A): an angle is
 * folded to rho in [0, pi/2] with a sign (Section 3); rho selects one of six
 * pieces of width pi/12; on piece k, with t = rho in degrees,
 *     N = a_k t + b_k,   D = c_k t + d_k       (Appendix A, eqs. 5-10)
 *     tan = N / D,   sin = N / sqrt(N^2 + D^2),   cos = D / sqrt(N^2 + D^2)
 * (Appendix A.4).  Arithmetic: argument reduction and the two linear forms
 * in FP64, everything after (the quadratic, inverse square root, quotient)
 * in FP32.  Results agree with a plain FP64 evaluation of the same formulas
 * to within 4 FP32 ulp.
 *
 * Conventions for every entry point:
 *  - Buffers are device pointers owned by the caller, contiguous, all of the
 *    same storage dtype `dt`.  The library never allocates, frees or
 *    synchronises.  Work is enqueued on `stream` (NULL = default stream);
 *    results are valid once the caller synchronises that stream.
 *  - `n` is the element count.  n == 0 returns TA_OK without a launch.
 *  - Errors detected before any HIP call (so also testable without a GPU):
 *      TA_EINVAL   n < 0, a required pointer NULL while n > 0, a bad `terms`
 *                  or unknown flag bits;
 *      TA_EDTYPE   `dt` is not one of ta_dtype;
 *      TA_EOVERLAP an output partially overlaps an input or another output
 *                  (an output may alias an input exactly: in-place).
 *    TA_EHIP: the kernel launch failed; ta_last_hip_error() returns the
 *    hipError_t of the calling thread's last failure.
 *  - Any alignment is accepted.  When every buffer has the same address
 *    modulo 16 the body runs with 16-byte vector accesses after a scalar
 *    head and before a scalar tail; otherwise a scalar path runs.
 *  - Calls are reentrant and thread-safe: there is no mutable global state.
 *  - Inputs: any value.  NaN and +-Inf give NaN; sin and tan keep the sign of
 *    a zero input; cos(+-0) = 1.  Every finite input is reduced exactly
 *    enough for the 4-ulp agreement (FP64 Cody-Waite below 2^29 in magnitude,
 *    a 2/pi bit-table reduction above).
 */
#ifndef TA_H_
#define TA_H_

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* TA_F64: FP64 storage, and every stage of the method in FP64 (the paper's
 * own functions take and return double).  Results agree with an exact
 * evaluation of the same formulas to within 6 FP64 ulp. */
/* The last enumerator of each enum only widens its range to every 32-bit
 * value, so that any int a caller passes is a valid value of the type (an
 * unknown dtype is then an error status, not undefined behaviour in the
 * library's C++); it is not a dtype or a status. */
typedef enum {
  TA_F32 = 0,
  TA_F16 = 1,
  TA_BF16 = 2,
  TA_F64 = 3,
  TA_DTYPE_RANGE_ = 0x7fffffff
} ta_dtype;

typedef enum {
  TA_OK = 0,
  TA_EINVAL = 1,
  TA_EDTYPE = 2,
  TA_EOVERLAP = 3,
  TA_EHIP = 4,
  TA_STATUS_RANGE_ = 0x7fffffff
} ta_status;

/* Flag bits for the *_ex forward calls. */
enum {
  /* The pseudocode of proposed_tan (Section 3) returns +infinity, before the
   * sign is applied, when the folded angle is within 1e-3 of pi/2.  Off by
   * default (the formula is then used all the way to the pole). */
  TA_FLAG_TAN_GUARD = 1u,
  /* Reduce the argument in FP64 (Cody-Waite below 2^29, a 2/pi bit-table
   * reduction above).  This is the default for FP32 and FP64 storage, so
   * the flag changes nothing there; it is accepted by every call that takes
   * flags.  16-bit storage always evaluates in FP32 (below). */
  TA_FLAG_FORCE_FP64_REDUCTION = 2u,
  /* Forward *_ex calls on FP32 storage: reduce and evaluate in FP32, FP64
   * only for |x| >= 2^20 (and +-Inf, NaN).  Below 2^20: a three-word FP32
   * Cody-Waite reduction whose rounding error is carried as a second word,
   * the angle in degrees split into a high part on a 2^-12 grid (so that the
   * slope times it plus the intercept is exact) and a low part, each linear
   * form one exact FMA plus one rounding FMA, then the refined inverse
   * square root and reciprocal.  FP32 results stay within 4 FP32 ulp of the
   * formula (3.16 measured over every FP32 below 2^20, against 2.53 for the
   * default FP64 forms).  No effect for 16-bit storage (always evaluated in
   * FP32); TA_EINVAL with TA_F64 or with TA_FLAG_FORCE_FP64_REDUCTION. */
  TA_FLAG_FORCE_FP32_REDUCTION = 4u,
  /* ta_paper_sincos only: index the pieces by floor(rho / 0.261) as the
   * pseudocode of proposed_sin / proposed_tan does (clamped to the last
   * piece) instead of the pi/12 intervals of Section 2. */
  TA_FLAG_LITERAL_DIVISOR = 8u
};

/* ---- forward: the proposed functions (Section 2 formulas, Section 3 fold) */

/* y[i] = sin_a(x[i]).  Section 2, sine cases. */
ta_status ta_sin(const void *x, void *y, int64_t n, ta_dtype dt,
                 hipStream_t stream);
/* y[i] = cos_a(x[i]).  Section 2, cosine cases. */
ta_status ta_cos(const void *x, void *y, int64_t n, ta_dtype dt,
                 hipStream_t stream);
/* The same with flag bits (TA_FLAG_FORCE_FP64_REDUCTION,
 * TA_FLAG_FORCE_FP32_REDUCTION; TA_FLAG_TAN_GUARD is accepted and affects
 * tan outputs only). */
ta_status ta_sin_ex(const void *x, void *y, int64_t n, ta_dtype dt,
                    hipStream_t stream, uint32_t flags);
ta_status ta_cos_ex(const void *x, void *y, int64_t n, ta_dtype dt,
                    hipStream_t stream, uint32_t flags);
/* y[i] = tan_a(x[i]).  Section 2, tangent cases; finite up to the
 * pole (the last piece's D vanishes only at exactly pi/2). */
ta_status ta_tan(const void *x, void *y, int64_t n, ta_dtype dt,
                 hipStream_t stream);
/* Fused: one reduction per element, ys = sin_a, yc = cos_a and, when `yt` is
 * not NULL, yt = tan_a.  `ys` and `yc` are required. */
ta_status ta_sincos(const void *x, void *ys, void *yc, void *yt, int64_t n,
                    ta_dtype dt, hipStream_t stream);
/* Same as above with flag bits (TA_FLAG_TAN_GUARD affects tan outputs;
 * TA_FLAG_FORCE_FP64_REDUCTION, TA_FLAG_FORCE_FP32_REDUCTION). */
ta_status ta_tan_ex(const void *x, void *y, int64_t n, ta_dtype dt,
                    hipStream_t stream, uint32_t flags);
ta_status ta_sincos_ex(const void *x, void *ys, void *yc, void *yt, int64_t n,
                       ta_dtype dt, hipStream_t stream, uint32_t flags);

/* ---- Taylor baseline (Section 3, Taylor comparison; Tables 1-3 columns) ----
 * The first `terms` (5, 7 or 9) non-zero Maclaurin terms of sin, cos or tan,
 * in FP32 Horner form, evaluated on the same folded angle rho in [0, pi/2]
 * with the same signs.  terms outside {5, 7, 9} -> TA_EINVAL. */
ta_status ta_taylor_sin(const void *x, void *y, int64_t n, int terms,
                        ta_dtype dt, hipStream_t stream);
ta_status ta_taylor_cos(const void *x, void *y, int64_t n, int terms,
                        ta_dtype dt, hipStream_t stream);
ta_status ta_taylor_tan(const void *x, void *y, int64_t n, int terms,
                        ta_dtype dt, hipStream_t stream);

/* ---- backward: analytic derivative of the selected piece ----------------
 * Differentiating Appendix A.4 on piece k gives, with
 * omega = (180/pi) (a_k d_k - b_k c_k) / (N^2 + D^2):
 *   d sin_a/dx = omega cos_a(x),  d cos_a/dx = -omega sin_a(x),
 *   d tan_a/dx = omega (1 + tan_a(x)^2)        in every quadrant.
 * The approximation jumps at 15, 30, 60 and 75 degrees and has a kink at 45;
 * there the derivative of the piece selected by the forward is returned.
 * gx[i] = gy[i] * d f/dx (x[i]).  x, gy, gx share the dtype. */
ta_status ta_sin_bwd(const void *x, const void *gy, void *gx, int64_t n,
                     ta_dtype dt, hipStream_t stream);
ta_status ta_cos_bwd(const void *x, const void *gy, void *gx, int64_t n,
                     ta_dtype dt, hipStream_t stream);
ta_status ta_tan_bwd(const void *x, const void *gy, void *gx, int64_t n,
                     ta_dtype dt, hipStream_t stream);
/* gx = gs * d sin_a/dx + gc * d cos_a/dx.  Either gs or gc may be NULL
 * (treated as zero); not both. */
ta_status ta_sincos_bwd(const void *x, const void *gs, const void *gc,
                        void *gx, int64_t n, ta_dtype dt, hipStream_t stream);

/* ---- fused forward + backward in one pass (reads x, gy; writes y, gx) --- */
ta_status ta_sin_fwdbwd(const void *x, const void *gy, void *y, void *gx,
                        int64_t n, ta_dtype dt, hipStream_t stream);
ta_status ta_cos_fwdbwd(const void *x, const void *gy, void *y, void *gx,
                        int64_t n, ta_dtype dt, hipStream_t stream);
ta_status ta_tan_fwdbwd(const void *x, const void *gy, void *y, void *gx,
                        int64_t n, ta_dtype dt, hipStream_t stream);

/* ---- the paper's literal arithmetic (Section 3, Algorithms 1-4) ---------
 * Same fold and signs, then in FP64: radian coefficients a_k*180/pi,
 * c_k*180/pi (b_k, d_k unchanged), piece index floor(rho / (pi/12)),
 * sin = (a rho + b) * FISR(x rho^2 + y rho + z), cos likewise with
 * (c rho + d), tan = (a rho + b) * FISR(c rho + d)^2, where FISR is
 * Algorithm 1 (magic constant 0x5fe6eb50c7b537a9, one Newton step).  Results
 * are rounded to the storage dtype.  This reproduces the error statistics of
 * Tables 1-3 (maximum sin/cos error 1.532e-3); it is ~3x less accurate than
 * ta_sincos.  Any non-empty subset of ys/yc/yt; flags: TA_FLAG_TAN_GUARD,
 * TA_FLAG_LITERAL_DIVISOR, TA_FLAG_FORCE_FP64_REDUCTION. */
ta_status ta_paper_sincos(const void *x, void *ys, void *yc, void *yt,
                          int64_t n, ta_dtype dt, hipStream_t stream,
                          uint32_t flags);

/* ---- multi-frequency encoding (an application of the fused core) --------
 * For j = 0 .. nfreq-1 (1 <= nfreq <= 16), with y holding 2*nfreq planes of n
 * elements each (plane-major):
 *   y[(2j) n + i] = sin_a(2^j x[i]),   y[(2j+1) n + i] = cos_a(2^j x[i]).
 * One read of x, one reduction and one pair of linear forms per frequency,
 * same accuracy as ta_sincos on the argument 2^j x (exact in FP32; it
 * overflows to +-Inf, giving NaN, only for |x| >= 2^(128-j)).  y must not
 * overlap x.  16-byte accesses when x and y share their address modulo 16 and
 * n * sizeof(dtype) is a multiple of 16; a scalar kernel otherwise. */
ta_status ta_sincos_encode(const void *x, void *y, int64_t n, int nfreq,
                           ta_dtype dt, hipStream_t stream);

/* ---- measurement comparators (not part of the method) -------------------
 * The same load/store skeleton around the GPU's built-in functions:
 *   kind 0: sinf / cosf / tanf (accurate device library)
 *   kind 1: __sinf / __cosf / __tanf (hardware approximations)
 *   kind 2: sincosf + tanf
 * Outputs: ys alone, ys and yc, or ys, yc and yt (any other choice of NULLs
 * is TA_EINVAL).  FP32, and FP16/BF16 storage (the FP32 function of the
 * widened input, rounded to nearest even); FP64: the device library's double
 * functions, kinds 0 and 2 (kind 1 is TA_EDTYPE). */
ta_status ta_builtin_sincos(const void *x, void *ys, void *yc, void *yt,
                            int64_t n, int kind, ta_dtype dt,
                            hipStream_t stream);
/* The sine activation's fused forward and backward with the built-in
 * functions: y = sin x, gx = gy cos x, by sincosf (kind 0) or __sinf and
 * __cosf (kind 1); FP64 storage: sincos (kind 0 only).  Same conventions as
 * ta_sin_fwdbwd. */
ta_status ta_builtin_sin_fwdbwd(const void *x, const void *gy, void *y,
                                void *gx, int64_t n, int kind, ta_dtype dt,
                                hipStream_t stream);
/* Plain streaming copy with the same access pattern as the kernels: reads
 * n_in input arrays (1..3) and writes n_out outputs (1..3), out[j][i] =
 * in[j % n_in][i].  The achievable HBM ceiling for that byte mix. */
ta_status ta_copy(const void *const *in, int n_in, void *const *out,
                  int n_out, int64_t n, ta_dtype dt, hipStream_t stream);

/* Bandwidth probes: plain 16-byte streams over FP32 arrays of n elements
 * (n a multiple of 4; every buffer 16-byte aligned; otherwise TA_EINVAL),
 * one access per stream per thread, to measure what HBM delivers for a
 * byte mix.
 *   kind 0: read x (n_out = 1: out[0] is a sink of 1024 words, written at
 *           most a few times);
 *   kind 1: write n_out (1..3) arrays, x unused;
 *   kind 2: copy x into n_out (1..3) arrays.
 * flags: TA_PROBE_NT_LOAD / TA_PROBE_NT_STORE (nontemporal accesses),
 * TA_PROBE_BLOCK256 (256-thread workgroups; 64 otherwise),
 * TA_PROBE_DEVICE_SCOPE (with TA_PROBE_NT_STORE only: nontemporal stores at
 * device scope, the store the kernels' vector bodies issue).  Overlapping
 * buffers are TA_EOVERLAP. */
enum {
  TA_PROBE_NT_LOAD = 1u,
  TA_PROBE_NT_STORE = 2u,
  TA_PROBE_BLOCK256 = 4u,
  TA_PROBE_DEVICE_SCOPE = 8u
};
ta_status ta_stream_probe(int kind, const void *x, void *const *out,
                          int n_out, int64_t n, uint32_t flags,
                          hipStream_t stream);

/* ---- utilities ---------------------------------------------------------- */
const char *ta_status_str(ta_status s);
/* hipError_t of the calling thread's last TA_EHIP (0 if none). */
int ta_last_hip_error(void);
const char *ta_version(void);

#ifdef __cplusplus
}
#endif

#endif /* TA_H_ */
