// ta_kernels.hip -- gfx950 kernels and the C ABI of libta.so.
//
// Every entry point is an elementwise map: NIN input streams, NOUT output
// streams, one functor per element.  The streaming skeleton issues 16-byte
// global loads and stores (4 FP32, 8 FP16/BF16 or 2 FP64 elements per
// access; 8-byte accesses of 4 FP16/BF16 elements for one input and several
// outputs), with a launch shape per kernel category (see shape_for) and
// 64-bit indexing.  The
// per-piece coefficients live in LDS (one copy of 176-360 bytes per
// workgroup, by kernel family), never in HBM.
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <stdint.h>
#include <string.h>

#include <type_traits>

#include "ta.h"
#include "ta_math.hpp"

namespace ta {

// ---------------------------------------------------------------------------
// Storage formats.  `val` is the arithmetic type of the element functors:
// FP32 for the FP32 and 16-bit formats (loads widen exactly, stores round
// to nearest even), FP64 for FP64.  unpack/pack convert one 16-byte access
// (unpack copies the bytes out: reading lanes of a vector that is only
// loaded under a branch makes the compiler zero it first).
// ---------------------------------------------------------------------------
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

struct F32 {
  using raw = uint32_t;
  using val = float;
  using vec = u32x4;
  static constexpr int kVec = 4;
  static __device__ val load(raw v) { return __uint_as_float(v); }
  static __device__ raw store(val f) { return __float_as_uint(f); }
  static __device__ void unpack(const u32x4 &w, val *v) {
    __builtin_memcpy(v, &w, 16);
  }
  static __device__ u32x4 pack(const val *v) {
    u32x4 w;
#pragma unroll
    for (int e = 0; e < 4; ++e) w[e] = __float_as_uint(v[e]);
    return w;
  }
};

// 16-bit formats round pairs: a <2 x float> -> <2 x half|bfloat>
// conversion is one v_cvt_pk_{f16,bf16}_f32.  Accesses of NV elements: 8
// (16 bytes, 44-50 VGPRs for the method with the FP32 evaluation) or 4 (8
// bytes; the one-input, several-output kernels, below).
template <class Derived, int NV>
struct Half16 {
  using raw = uint16_t;
  using val = float;
  static constexpr int kVec = NV;
  using vec = typename std::conditional<NV == 8, u32x4, u32x2>::type;
  static __device__ void unpack(const vec &w, val *v) {
    raw h[kVec];
    __builtin_memcpy(h, &w, sizeof(vec));
#pragma unroll
    for (int e = 0; e < kVec; ++e) v[e] = Derived::load(h[e]);
  }
  static __device__ vec pack(const val *v) {
    vec w;
#pragma unroll
    for (int j = 0; j < kVec / 2; ++j)
      w[j] = Derived::store2(v[2 * j], v[2 * j + 1]);
    return w;
  }
};
template <int NV>
struct F16T : Half16<F16T<NV>, NV> {
  using raw = uint16_t;
  static __device__ float load(raw v) {
    return float(__builtin_bit_cast(_Float16, v));
  }
  static __device__ raw store(float f) {
    return __builtin_bit_cast(raw, _Float16(f));
  }
  static __device__ uint32_t store2(float lo, float hi) {
    const f32x2 v = {lo, hi};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, f16x2));
  }
};
template <int NV>
struct BF16T : Half16<BF16T<NV>, NV> {
  using raw = uint16_t;
  static __device__ float load(raw v) { return __uint_as_float(uint32_t(v) << 16); }
  static __device__ raw store(float f) {
    return __builtin_bit_cast(raw, __bf16(f));
  }
  static __device__ uint32_t store2(float lo, float hi) {
    const f32x2 v = {lo, hi};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
  }
};

using F16 = F16T<8>;
using BF16 = BF16T<8>;
// One input and several outputs of 16-bit storage take 8-byte accesses, two
// per thread in 256-thread groups: BF16 sin+cos+tan over 16 array placements
// in two processes 6.43 against 6.17 TB/s for one 16-byte access per thread
// (ahead on 15), sin+cos 6.42 against 6.36; one 8-byte access 6.26 and
// 5.89, two in 128-thread groups 6.22 and 6.39.  The fused forward and
// backward (two inputs, two outputs) takes one 8-byte access per thread in
// its 256-thread shape above 256 MiB of input: BF16 at 2^29 elements 6.48
// against 6.29 TB/s over 12 placements (ahead on 12); two accesses in
// 128-thread groups 6.55.
using F16x4 = F16T<4>;
using BF16x4 = BF16T<4>;

struct F64 {
  using raw = uint64_t;
  using val = double;
  using vec = u32x4;
  static constexpr int kVec = 2;
  static __device__ val load(raw v) { return __longlong_as_double(int64_t(v)); }
  static __device__ raw store(val f) { return raw(__double_as_longlong(f)); }
  static __device__ void unpack(const u32x4 &w, val *v) {
    __builtin_memcpy(v, &w, 16);
  }
  static __device__ u32x4 pack(const val *v) {
    u32x4 w;
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const raw b = store(v[e]);
      w[2 * e] = uint32_t(b);
      w[2 * e + 1] = uint32_t(b >> 32);
    }
    return w;
  }
};

// ---------------------------------------------------------------------------
// Element functors.  in[]/out[] are FP32 values; `tb` is the LDS table.
// ---------------------------------------------------------------------------
enum : int { kSin = 1, kCos = 2, kTan = 4 };

// The output sign: from the quadrant masks for the FP64 folds (8-row
// tables), already in N and D for the FP32 evaluation (the signed 32-row
// FP16 table, FoldedL).
template <class F, class V>
__device__ inline V sgn_sin(const F &f, V v) {
  if constexpr (std::is_same<F, FoldedL>::value) return v;
  else return flip_sign(v, sin_mask(f));
}
template <class F, class V>
__device__ inline V sgn_cos(const F &f, V v) {
  if constexpr (std::is_same<F, FoldedL>::value) return v;
  else return flip_sign(v, cos_mask(f));
}
template <class F, class V>
__device__ inline V sgn_tan(const F &f, V v) {
  if constexpr (std::is_same<F, FoldedL>::value) return v;
  else return flip_sign(v, tan_mask(f));
}

// LOW: the variant for 16-bit storage.  Its outputs keep 8 (BF16) or 11
// (FP16) significant bits, so the whole evaluation runs in FP32
// (fold_forms_f32) and the hardware inverse square root and reciprocal (each
// within about one FP32 ulp) are used without the Newton refinement.
// Every op names the instances the 16-bit formats launch: Low for BF16,
// LowH for FP16, whose finite values all lie below 2^16 (SMALL: no test for
// the FP64 fold; +-Inf and NaN come out NaN through the FP32 fold too).
// F32RED (forward, FP32 storage, TA_FLAG_FORCE_FP32_REDUCTION): the FP32
// evaluation with the reduction residual carried (fold_forms_f32, CARRY) and
// the refined inverse square root and reciprocal.
template <int MASK, bool GUARD, bool LOW = false, bool F32RED = false,
          bool SMALL = false>
struct FwdOp {
  static constexpr int NIN = 1;
  static constexpr int NOUT = ((MASK & kSin) ? 1 : 0) + ((MASK & kCos) ? 1 : 0) +
                              ((MASK & kTan) ? 1 : 0);
  static constexpr bool kFp32Fold = LOW || F32RED;
  // the tan guard keeps |r| live to the end: more than 64 VGPRs
  static constexpr bool kWideSingle = GUARD;
  using Table = typename std::conditional<kFp32Fold, Tables16, TablesFwd>::type;
  using Low = FwdOp<MASK, GUARD, true>;
  using LowH = FwdOp<MASK, GUARD, true, false, true>;
  __device__ static void apply(const float *in, float *out, const Table &tb,
                                  uint32_t) {
    if constexpr (kFp32Fold) {
      FoldedL f;
      const Forms v = fold_forms_f32<!SMALL, F32RED>(in[0], tb, f);
      finish(f, v, out);
    } else {
      const Folded f = fold(in[0], tb.magic);
      finish(f, forms(f, tb), out);
    }
  }
  template <class F>
  __device__ static void finish(const F &f, const Forms &v, float *out) {
    int o = 0;
    if constexpr ((MASK & (kSin | kCos)) != 0) {
      const float y = LOW ? rsqrt_est(v.q) : rsqrt_refined(v.q);
      if constexpr (MASK & kSin) out[o++] = sgn_sin(f, v.n * y);
      if constexpr (MASK & kCos) out[o++] = sgn_cos(f, v.d * y);
    }
    if constexpr (MASK & kTan) {
      float t = sgn_tan(f, LOW ? div_est(v.n, v.d) : div_refined(v.n, v.d));
      if constexpr (GUARD) {
        // Section 3 proposed_tan: +inf within 1e-3 of pi/2, before the sign.
        if ((f.q & 1u) && f.abs_r() < 1e-3) t = __builtin_inff();
      }
      out[o++] = t;
    }
  }
  __device__ static void apply(const double *in, double *out, const Table &tb,
                               uint32_t) {
    static_assert(!kFp32Fold, "FP64 storage uses the FP64 table");
    const Folded64 f = fold64(in[0], tb.magic);
    const Forms64 v = forms64(f, tb);
    int o = 0;
    if constexpr ((MASK & (kSin | kCos)) != 0) {
      const double y = rsqrt64_refined(v.q);
      if constexpr (MASK & kSin) out[o++] = sgn_sin(f, v.n * y);
      if constexpr (MASK & kCos) out[o++] = sgn_cos(f, v.d * y);
    }
    if constexpr (MASK & kTan) {
      double t = sgn_tan(f, div64_refined(v.n, v.d));
      if constexpr (GUARD) {
        if ((f.q & 1u) && f.abs_r() < 1e-3) t = __builtin_inf();
      }
      out[o++] = t;
    }
  }
};

template <int MASK, int TERMS>
struct TaylorOp {
  static constexpr int NIN = 1;
  static constexpr int NOUT = 1;
  using Table = NoTable;
  using Low = TaylorOp;
  using LowH = TaylorOp;
  __device__ static void apply(const float *in, float *out, const Table &,
                                  uint32_t) {
    const Folded f = fold(in[0]);
    const float rho = fold_rho(f);
    if constexpr (MASK == kSin)
      out[0] = flip_sign(taylor_sin_unsigned<TERMS>(rho), sin_mask(f));
    if constexpr (MASK == kCos)
      out[0] = flip_sign(taylor_cos_unsigned<TERMS>(rho), cos_mask(f));
    if constexpr (MASK == kTan)
      out[0] = flip_sign(taylor_tan_unsigned<TERMS>(rho), tan_mask(f));
  }
  __device__ static void apply(const double *in, double *out, const Table &,
                               uint32_t) {
    const Folded64 f = fold64(in[0]);
    const double rho = fold_rho64(f);
    if constexpr (MASK == kSin)
      out[0] = flip_sign(taylor_sin_unsigned<TERMS>(rho), sin_mask(f));
    if constexpr (MASK == kCos)
      out[0] = flip_sign(taylor_cos_unsigned<TERMS>(rho), cos_mask(f));
    if constexpr (MASK == kTan)
      out[0] = flip_sign(taylor_tan_unsigned<TERMS>(rho), tan_mask(f));
  }
};

// d/dx of the selected piece times the upstream gradient(s).
//   sin: gx = gy * omega * cos_a     cos: gx = -gy * omega * sin_a
//   tan: gx = gy * (180/pi) det / D^2
// WITH_Y also writes the forward value (the fused forward+backward).
template <int WHICH, bool WITH_Y, bool LOW = false, bool SMALL = false>
struct BwdOp {
  static constexpr int NIN = 2;  // x, gy
  static constexpr int NOUT = WITH_Y ? 2 : 1;
  using Table = typename std::conditional<LOW, Tables16Bwd, TablesBwd>::type;
  using Low = BwdOp<WHICH, WITH_Y, true>;
  using LowH = BwdOp<WHICH, WITH_Y, true, true>;
  __device__ static void apply(const float *in, float *out, const Table &tb,
                                  uint32_t) {
    if constexpr (LOW) {
      FoldedL f;
      const Forms v = fold_forms_f32<!SMALL>(in[0], tb, f);
      finish(f, v, in, out, tb);
    } else {
      const Folded f = fold(in[0], tb.magic);
      finish(f, forms(f, tb), in, out, tb);
    }
  }
  template <class F>
  __device__ static void finish(const F &f, const Forms &v, const float *in,
                                float *out, const Table &tb) {
    const float kdet = tb.kdet[f.row];
    if constexpr (WHICH == kTan) {
      const float r = LOW ? rcp_est(v.d) : rcp_refined(v.d);
      const float dt = kdet * r * r;
      if constexpr (WITH_Y)
        out[0] = sgn_tan(f, LOW ? v.n * r : div_refined(v.n, v.d));
      out[WITH_Y ? 1 : 0] = in[1] * dt;
    } else {
      const float y = LOW ? rsqrt_est(v.q) : rsqrt_refined(v.q);
      const float s = sgn_sin(f, v.n * y);
      const float c = sgn_cos(f, v.d * y);
      const float omega = kdet * y * y;
      if constexpr (WHICH == kSin) {
        if constexpr (WITH_Y) out[0] = s;
        out[WITH_Y ? 1 : 0] = in[1] * (omega * c);
      } else {
        if constexpr (WITH_Y) out[0] = c;
        out[WITH_Y ? 1 : 0] = -(in[1] * (omega * s));
      }
    }
  }
  __device__ static void apply(const double *in, double *out, const Table &tb,
                               uint32_t) {
    const Folded64 f = fold64(in[0], tb.magic);
    const Forms64 v = forms64(f, tb);
    const double kdet = tb.kdet64[f.row];
    if constexpr (WHICH == kTan) {
      const double r = rcp64_refined(v.d);
      const double dt = kdet * r * r;
      if constexpr (WITH_Y)
        out[0] = flip_sign(__builtin_fma(__builtin_fma(-v.d, v.n * r, v.n), r,
                                         v.n * r),
                           tan_mask(f));
      out[WITH_Y ? 1 : 0] = in[1] * dt;
    } else {
      const double y = rsqrt64_refined(v.q);
      const double s = sgn_sin(f, v.n * y);
      const double c = sgn_cos(f, v.d * y);
      const double omega = kdet * y * y;
      if constexpr (WHICH == kSin) {
        if constexpr (WITH_Y) out[0] = s;
        out[WITH_Y ? 1 : 0] = in[1] * (omega * c);
      } else {
        if constexpr (WITH_Y) out[0] = c;
        out[WITH_Y ? 1 : 0] = -(in[1] * (omega * s));
      }
    }
  }
};

// gx = gs * d sin_a/dx + gc * d cos_a/dx = omega (gs cos_a - gc sin_a).
template <bool HAS_GS, bool HAS_GC, bool LOW = false, bool SMALL = false>
struct SinCosBwdOp {
  static constexpr int NIN = 1 + (HAS_GS ? 1 : 0) + (HAS_GC ? 1 : 0);
  static constexpr int NOUT = 1;
  using Table = typename std::conditional<LOW, Tables16Bwd, TablesBwd>::type;
  using Low = SinCosBwdOp<HAS_GS, HAS_GC, true>;
  using LowH = SinCosBwdOp<HAS_GS, HAS_GC, true, true>;
  __device__ static void apply(const float *in, float *out, const Table &tb,
                                  uint32_t) {
    if constexpr (LOW) {
      FoldedL f;
      const Forms v = fold_forms_f32<!SMALL>(in[0], tb, f);
      finish(f, v, in, out, tb);
    } else {
      const Folded f = fold(in[0], tb.magic);
      finish(f, forms(f, tb), in, out, tb);
    }
  }
  template <class F>
  __device__ static void finish(const F &f, const Forms &v, const float *in,
                                float *out, const Table &tb) {
    const float y = LOW ? rsqrt_est(v.q) : rsqrt_refined(v.q);
    const float omega = tb.kdet[f.row] * y * y;
    float acc = 0.0f;
    if constexpr (HAS_GS) acc = in[1] * sgn_cos(f, v.d * y);
    if constexpr (HAS_GC)
      acc = __builtin_fmaf(-in[HAS_GS ? 2 : 1], sgn_sin(f, v.n * y),
                           acc);
    out[0] = omega * acc;
  }
  __device__ static void apply(const double *in, double *out, const Table &tb,
                               uint32_t) {
    const Folded64 f = fold64(in[0], tb.magic);
    const Forms64 v = forms64(f, tb);
    const double y = rsqrt64_refined(v.q);
    const double omega = tb.kdet64[f.row] * y * y;
    double acc = 0.0;
    if constexpr (HAS_GS) acc = in[1] * sgn_cos(f, v.d * y);
    if constexpr (HAS_GC)
      acc = __builtin_fma(-in[HAS_GS ? 2 : 1], sgn_sin(f, v.n * y),
                          acc);
    out[0] = omega * acc;
  }
};

// The paper's literal arithmetic (Algorithms 1-4 in FP64) on the same fold
// and signs; flags: TA_FLAG_TAN_GUARD, TA_FLAG_LITERAL_DIVISOR.
template <int MASK>
struct PaperOp {
  static constexpr int NIN = 1;
  static constexpr int NOUT = ((MASK & kSin) ? 1 : 0) + ((MASK & kCos) ? 1 : 0) +
                              ((MASK & kTan) ? 1 : 0);
  using Table = PaperTables;
  using Low = PaperOp;
  using LowH = PaperOp;
  __device__ static void apply(const float *in, float *out, const Table &tb,
                               uint32_t flags) {
    const Folded f = fold(in[0]);
    const double ang =
        (f.q & 1u) ? (kPio2Hi - f.abs_r()) + kPio2Lo : f.abs_r();
    const double divisor =
        (flags & TA_FLAG_LITERAL_DIVISOR) ? kLiteralDivisor : kPi12;
    double s, c, t;
    paper_eval(ang, divisor, tb, s, c, t);
    int o = 0;
    if constexpr (MASK & kSin) out[o++] = flip_sign(float(s), sin_mask(f));
    if constexpr (MASK & kCos) out[o++] = flip_sign(float(c), cos_mask(f));
    if constexpr (MASK & kTan) {
      float tt = flip_sign(float(t), tan_mask(f));
      // proposed_tan: +inf within 1e-3 of pi/2, before the sign
      if ((flags & TA_FLAG_TAN_GUARD) && (f.q & 1u) && f.abs_r() < 1e-3)
        tt = __builtin_inff();
      out[o++] = tt;
    }
  }
  __device__ static void apply(const double *in, double *out, const Table &tb,
                               uint32_t flags) {
    const Folded64 f = fold64(in[0]);
    const double ang = fold_rho64(f);
    const double divisor =
        (flags & TA_FLAG_LITERAL_DIVISOR) ? kLiteralDivisor : kPi12;
    double s, c, t;
    paper_eval(ang, divisor, tb, s, c, t);
    int o = 0;
    if constexpr (MASK & kSin) out[o++] = flip_sign(s, sin_mask(f));
    if constexpr (MASK & kCos) out[o++] = flip_sign(c, cos_mask(f));
    if constexpr (MASK & kTan) {
      double tt = flip_sign(t, tan_mask(f));
      if ((flags & TA_FLAG_TAN_GUARD) && (f.q & 1u) && f.abs_r() < 1e-3)
        tt = __builtin_inf();
      out[o++] = tt;
    }
  }
};

// Comparators: the GPU's built-in functions in the same skeleton.  NO
// outputs: sin (1), sin and cos (2), sin, cos and tan (3).  16-bit storage
// evaluates the FP32 function on the widened input and rounds the result.
template <int KIND, int NO>
struct BuiltinOp {
  static constexpr int NIN = 1;
  static constexpr int NOUT = NO;
  using Table = NoTable;
  using Low = BuiltinOp;
  using LowH = BuiltinOp;
  __device__ static void apply(const float *in, float *out, const Table &,
                                  uint32_t) {
    const float x = in[0];
    if constexpr (KIND == 0) {
      out[0] = sinf(x);
      if constexpr (NO >= 2) out[1] = cosf(x);
      if constexpr (NO >= 3) out[2] = tanf(x);
    } else if constexpr (KIND == 1) {
      out[0] = __sinf(x);
      if constexpr (NO >= 2) out[1] = __cosf(x);
      if constexpr (NO >= 3) out[2] = __tanf(x);
    } else {
      if constexpr (NO >= 2) {
        float s, c;
        sincosf(x, &s, &c);
        out[0] = s;
        out[1] = c;
      } else {
        out[0] = sinf(x);
      }
      if constexpr (NO >= 3) out[2] = tanf(x);
    }
  }
  // FP64: the device library's sin/cos/tan (kind 0) or sincos + tan (kind
  // 2); there are no FP64 hardware approximations (kind 1).
  __device__ static void apply(const double *in, double *out, const Table &,
                               uint32_t) {
    const double x = in[0];
    if constexpr (KIND == 2 && NO >= 2) {
      double s, c;
      sincos(x, &s, &c);
      out[0] = s;
      out[1] = c;
    } else {
      out[0] = sin(x);
      if constexpr (NO >= 2) out[1] = cos(x);
    }
    if constexpr (NO >= 3) out[2] = tan(x);
  }
};

// The fused forward+backward of the sine activation with the built-in
// functions: y = sin x, gx = gy cos x, by sincosf (kind 0) or __sinf and
// __cosf (kind 1); FP64: sincos.
template <int KIND>
struct BuiltinFwdBwdOp {
  static constexpr int NIN = 2;
  static constexpr int NOUT = 2;
  using Table = NoTable;
  using Low = BuiltinFwdBwdOp;
  using LowH = BuiltinFwdBwdOp;
  __device__ static void apply(const float *in, float *out, const Table &,
                               uint32_t) {
    float s, c;
    if constexpr (KIND == 0) {
      sincosf(in[0], &s, &c);
    } else {
      s = __sinf(in[0]);
      c = __cosf(in[0]);
    }
    out[0] = s;
    out[1] = in[1] * c;
  }
  __device__ static void apply(const double *in, double *out, const Table &,
                               uint32_t) {
    double s, c;
    sincos(in[0], &s, &c);
    out[0] = s;
    out[1] = in[1] * c;
  }
};

template <int NI, int NO>
struct CopyOp {
  static constexpr int NIN = NI;
  static constexpr int NOUT = NO;
  static constexpr bool kIsCopy = true;  // launched with the copy shape
  using Table = NoTable;
  using Low = CopyOp;
  using LowH = CopyOp;
  template <class V>
  __device__ static void apply(const V *in, V *out, const Table &, uint32_t) {
#pragma unroll
    for (int j = 0; j < NO; ++j) out[j] = in[j % NI];
  }
};

// ---------------------------------------------------------------------------
// Streaming skeleton
// ---------------------------------------------------------------------------
struct IoPtrs {
  const char *in[3];
  char *out[3];
  uint32_t flags;  // runtime flag bits for the element functor
};

// Launch shape of the vector body, per kernel category, chosen by timing on
// MI355X (2^27-2^29 elements):
//   one input, several outputs: plain loads and device-scope nontemporal
//     stores; FP32 sin, cos and tan of the method: 64 threads, four
//     accesses per thread, every output computed before the stores, then
//     each output array's four stores together (240 VGPRs, two waves per
//     SIMD; over 16 array placements in two processes it beat 256 threads
//     with one access on every one, mean 6.41 against 6.11 TB/s, worst 6.18
//     against 5.75; the same shape storing per access 5.67, 128 threads
//     grouped 6.30), the loads issued before the table fill (below); for
//     FP32 sin and cos grouping measured +2 % over 16 placements of one
//     probe but equal (6.36 against 6.37 TB/s, ahead on 4 of 8) after the
//     launches the benchmark times before it, and below the one-access
//     shape in the benchmark itself (513-517 against 520-535 Gelem/s), so
//     it keeps one access; for 16-bit storage and FP64 grouping was no
//     faster; the other FP32 multi-output kernels one access per stream per
//     thread and 256 threads (7 % above 128); FP64 128 threads (3 % above 256 in one
//     sweep, 12 % below it in another: where the arrays lie in memory
//     decides);
//   one FP32 output, the method (LDS table): 128 threads, two accesses per
//     thread, nontemporal loads and stores, at most 64 VGPRs (eight waves per
//     SIMD; the registers spilled are those of the rare large-argument
//     branch), the loads issued before the table fill (below): 819 Gelem/s
//     against 789 for 256 threads with the fill first; 64 threads 763, four
//     accesses 766, 72 VGPRs (seven waves) 804-808;
//     one FP64 output, and one FP32 output with the tan guard or the
//     paper-literal arithmetic (more than 64 VGPRs): 128 threads, two
//     accesses, loads before the fill, no occupancy bound (FP64 sin 400
//     Gelem/s against 374 for 256 threads with four accesses, FP64 tan 414
//     against 385, FP32 guarded tan 788 against 752; one access 356-361 for
//     FP64 sin);
//   one FP32/FP64 output, light functors (Taylor, the built-ins; no table):
//     one access, 128 threads (2 % above 256), nontemporal loads (sinf 860
//     Gelem/s against 827 with plain loads);
//   two FP32/FP64 inputs, one output (backward): 128 threads, two accesses,
//     nontemporal loads and stores; two outputs (fused forward+backward):
//     one access;
//   16-bit storage: one input and one output, 128 threads and two accesses
//     per thread with nontemporal loads, loads before the fill (BF16 sin
//     1663 Gelem/s against 1634 with the fill first and 1495 with four
//     8-byte accesses); one input and several outputs 8-byte accesses (the
//     F16x4/BF16x4 storage), two per thread in 256-thread groups, plain
//     loads (BF16 sin+cos+tan 6.28 against 6.19 TB/s with nontemporal loads
//     at one 16-byte access); two or more inputs one access per thread in
//     256-thread groups (8 bytes for two outputs above 256 MiB of input, 16
//     otherwise), nontemporal loads.
// loads_first: the kernel issues its loads, then fills the LDS table and
// waits at the barrier, so the fill overlaps the loads' latency.  That pays
// for one input and one output (FP32 sin +2.5-3.8 %, BF16 sin +1.7-2.2 %,
// FP16 sin +0.6 %) and for the grouped FP32 sin+cos+tan (+1.2 %, ahead on
// 14 of 16 placements); the other several-output kernels fill first
// (issuing their loads earlier measured sin+cos+tan in 256-thread groups
// -4.2 %, sin+cos -3.6 %, BF16 sin+cos+tan -0.3 %, FP64 sin+cos+tan
// -0.7 %), and the backward kernels
// showed no difference either way (FP64 single output: +3.6 % at 128
// threads with two accesses, none at 256 threads with four).
struct Shape {
  int block, unroll;
  bool nt_load, nt_store;
  int min_waves = 1;  // __launch_bounds__ minimum waves per SIMD
  bool loads_first = false;
  bool grouped = false;  // all outputs computed, then each array's stores
};
constexpr Shape kShapeMulti{256, 1, false, true};
constexpr Shape kShapeMulti3{64, 4, false, true, 1, true, true};
constexpr Shape kShapeSingle{128, 2, true, true, 8, true};
constexpr Shape kShapeSingleWide{128, 2, true, true, 1, true};
constexpr Shape kShapeMulti64{128, 1, false, true};
constexpr Shape kShapeLight{128, 1, true, true};
constexpr Shape kShapeTwoIn{128, 1, true, true};
constexpr Shape kShapeTwoIn1{128, 2, true, true};
constexpr Shape kShapeHalfSingle{128, 2, true, true, 1, true};
constexpr Shape kShapeHalfMulti{256, 2, false, true};
constexpr Shape kShapeHalf{256, 1, true, true};
// The copy comparators (the HBM ceiling a kernel is compared with): one
// wave per workgroup, the fastest plain copy of 1 -> 3 and 2 -> 2 FP32
// arrays measured on MI355X (about 2 % above 256 threads).
constexpr Shape kShapeCopy{64, 1, false, true};

template <class Op, class = void>
struct is_copy : std::false_type {};
template <class Op>
struct is_copy<Op, std::void_t<decltype(Op::kIsCopy)>> : std::true_type {};

template <class Op, class = void>
struct wide_single : std::false_type {};
template <class Op>
struct wide_single<Op, std::void_t<decltype(Op::kWideSingle)>>
    : std::integral_constant<bool, Op::kWideSingle> {};

template <class ST, class Op>
constexpr Shape shape_for() {
  if (sizeof(typename ST::raw) >= 4 && is_copy<Op>::value)
    return kShapeCopy;
  if (sizeof(typename ST::raw) == 2) {
    if (Op::NIN == 1)
      return Op::NOUT == 1 ? kShapeHalfSingle : kShapeHalfMulti;
    return kShapeHalf;
  }
  if (Op::NIN >= 2)
    return Op::NOUT == 1 ? kShapeTwoIn1 : kShapeTwoIn;
  // the method's sin, cos and tan of FP32 storage with the FP64 forms (not
  // the carried FP32 evaluation, whose grouped form measured no faster,
  // 6.16 against 6.15 TB/s over eight placements, nor the paper-literal
  // arithmetic)
  if (Op::NOUT == 3 && sizeof(typename ST::raw) == 4 &&
      std::is_same<typename Op::Table, TablesFwd>::value)
    return kShapeMulti3;
  if (Op::NOUT >= 2)
    return sizeof(typename ST::raw) == 8 ? kShapeMulti64
                                         : kShapeMulti;
  // the functors that evaluate the method use the LDS table
  if (!Op::Table::kUsed) return kShapeLight;
  // FP64 storage, and in FP32 the tan guard and the paper-literal FP64
  // arithmetic, need more than 64 VGPRs: no occupancy bound
  if (sizeof(typename ST::raw) == 8 || wide_single<Op>::value ||
      std::is_same<typename Op::Table, PaperTables>::value)
    return kShapeSingleWide;
  return kShapeSingle;
}

template <bool NT, class V = u32x4>
__device__ inline V vload(const char *base, int64_t v) {
  const V *p = reinterpret_cast<const V *>(base) + v;
  if constexpr (NT) return __builtin_nontemporal_load(p);
  return *p;
}
template <bool NT, class V>
__device__ inline void vstore(char *base, int64_t v, V x) {
  V *p = reinterpret_cast<V *>(base) + v;
  if constexpr (NT) {
    __builtin_nontemporal_store(x, p);
  } else {
    *p = x;
  }
}

// The vector bodies' stores: nontemporal at device scope (sc1 nt).  Source
// code reaches that cache policy only through the raw buffer store (a global
// store takes nt alone; an inline-asm store would hide the store from the
// compiler's hazard handling).  Each resource covers one workgroup's span of
// one output stream (base = the span's first byte, num_records = its length),
// so offsets stay 32-bit for any array size and the hardware's range check
// bounds every store to the span.  Word 3 is the raw (untyped) buffer format
// of gfx9.  Same-run on MI355X with identical outputs, against nt global
// stores: fused FP32 sin+cos+tan 6205 -> 6277 GB/s, BF16 fused +1.7 %,
// FP32 forward+backward +2.2 %, FP64 fused +1.2 %, single-output kernels
// equal; plain stores were 2-10 % slower than either.
constexpr int kBufferWord3 = 0x00020000;
constexpr int kStoreNtDevice = 2 | 16;  // nt, sc1
struct SpanStore {
  __amdgpu_buffer_rsrc_t r;
  __device__ SpanStore(char *span, int bytes)
      : r(__builtin_amdgcn_make_buffer_rsrc(span, 0, bytes, kBufferWord3)) {}
  __device__ void put(uint32_t byte_off, u32x4 x) const {
    __builtin_amdgcn_raw_buffer_store_b128(x, r, byte_off, 0, kStoreNtDevice);
  }
  __device__ void put(uint32_t byte_off, u32x2 x) const {
    __builtin_amdgcn_raw_buffer_store_b64(x, r, byte_off, 0, kStoreNtDevice);
  }
};

template <class ST, class Op>
__device__ inline void scalar_element(const IoPtrs &io, int64_t i,
                                      const typename Op::Table &tb) {
  using raw = typename ST::raw;
  typename ST::val in[Op::NIN], out[Op::NOUT];
#pragma unroll
  for (int k = 0; k < Op::NIN; ++k)
    in[k] = ST::load(reinterpret_cast<const raw *>(io.in[k])[i]);
  Op::apply(in, out, tb, io.flags);
#pragma unroll
  for (int k = 0; k < Op::NOUT; ++k)
    reinterpret_cast<raw *>(io.out[k])[i] = ST::store(out[k]);
}

// Vector body: elements [head, head + nvec*VEC) in 16-byte accesses, UNROLL
// accesses per stream per thread, all loads issued before any compute (LF:
// also before the table fill and its barrier); NTS: the stores go through
// SpanStore; GROUP: every output is computed before any store, then each
// output array's UNROLL stores are issued together.  The workgroup with
// blockIdx 0 also does the scalar head [0, head) and tail
// [head + nvec*VEC, n).
template <class ST, class Op, int BLOCK, int UNROLL, bool NTL, bool NTS,
          int MINB, bool LF, bool GROUP>
__global__ __launch_bounds__(BLOCK, MINB) void map_vec_kernel(IoPtrs io, int64_t head,
                                                        int64_t nvec, int64_t n) {
  using raw = typename ST::raw;
  constexpr int VEC = ST::kVec;
  __shared__ typename Op::Table tb;
  if constexpr (Op::Table::kUsed && !LF) {
    Op::Table::init(tb);
    __syncthreads();
  }
  const int64_t v0 = int64_t(blockIdx.x) * (UNROLL * BLOCK) + threadIdx.x;
  const char *in_base[Op::NIN];
  char *out_base[Op::NOUT];
#pragma unroll
  for (int k = 0; k < Op::NIN; ++k)
    in_base[k] = io.in[k] + head * int64_t(sizeof(raw));
#pragma unroll
  for (int k = 0; k < Op::NOUT; ++k)
    out_base[k] = io.out[k] + head * int64_t(sizeof(raw));
  typename ST::vec in_raw[UNROLL][Op::NIN];
#pragma unroll
  for (int u = 0; u < UNROLL; ++u) {
    const int64_t v = v0 + int64_t(u) * BLOCK;
    if (v < nvec) {
#pragma unroll
      for (int k = 0; k < Op::NIN; ++k) in_raw[u][k] = vload<NTL, typename ST::vec>(in_base[k], v);
    } else if constexpr (GROUP) {
#pragma unroll
      for (int k = 0; k < Op::NIN; ++k) in_raw[u][k] = typename ST::vec{};
    }
  }
  if constexpr (Op::Table::kUsed && LF) {
    Op::Table::init(tb);
    __syncthreads();
  }
  using vec = typename ST::vec;
  constexpr int kVB = int(sizeof(vec));
  constexpr int kSpan = UNROLL * BLOCK * kVB;
  const int64_t span0 = int64_t(blockIdx.x) * (UNROLL * BLOCK);
  static_assert(!GROUP || NTS, "grouped stores go through SpanStore");
  vec out_raw[GROUP ? UNROLL : 1][Op::NOUT];
#pragma unroll
  for (int u = 0; u < UNROLL; ++u) {
    const int64_t v = v0 + int64_t(u) * BLOCK;
    // GROUP: every vector is computed, past the end on zeros, so that the
    // UNROLL evaluations are straight-line code the compiler interleaves
    // (under one branch each they ran one after another: 5.82 against
    // 6.46 TB/s)
    if (GROUP || v < nvec) {
      using val = typename ST::val;
      val arg[Op::NIN][VEC], res[Op::NOUT][VEC];
#pragma unroll
      for (int k = 0; k < Op::NIN; ++k) ST::unpack(in_raw[u][k], arg[k]);
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        val in[Op::NIN], out[Op::NOUT];
#pragma unroll
        for (int k = 0; k < Op::NIN; ++k) in[k] = arg[k][e];
        Op::apply(in, out, tb, io.flags);
#pragma unroll
        for (int k = 0; k < Op::NOUT; ++k) res[k][e] = out[k];
      }
#pragma unroll
      for (int k = 0; k < Op::NOUT; ++k) {
        if constexpr (GROUP) {
          out_raw[u][k] = ST::pack(res[k]);
        } else if constexpr (NTS) {
          const SpanStore ss(out_base[k] + span0 * kVB, kSpan);
          ss.put(uint32_t(v - span0) * uint32_t(kVB), ST::pack(res[k]));
        } else {
          vstore<false>(out_base[k], v, ST::pack(res[k]));
        }
      }
    }
  }
  if constexpr (GROUP) {
#pragma unroll
    for (int k = 0; k < Op::NOUT; ++k) {
      const SpanStore ss(out_base[k] + span0 * kVB, kSpan);
#pragma unroll
      for (int u = 0; u < UNROLL; ++u) {
        const int64_t v = v0 + int64_t(u) * BLOCK;
        if (v < nvec) ss.put(uint32_t(v - span0) * uint32_t(kVB), out_raw[u][k]);
      }
    }
  }
  if (blockIdx.x == 0) {
    const int64_t tail0 = head + nvec * VEC;
    const int64_t extra = head + (n - tail0);
    for (int64_t e = threadIdx.x; e < extra; e += BLOCK)
      scalar_element<ST, Op>(io, e < head ? e : tail0 + (e - head), tb);
  }
}

// Launches `kernel` and returns the status of this launch itself (not a
// sticky error left by earlier, unrelated calls).  The arguments are
// converted to the kernel's own parameter types (non-deduced context), so
// each slot of argv has exactly the size the kernel reads.
template <typename T>
struct Same {
  using type = T;
};
template <typename... KArgs>
hipError_t launch(void (*kernel)(KArgs...), int64_t blocks, int threads,
                  hipStream_t stream, typename Same<KArgs>::type... args) {
  void *argv[] = {static_cast<void *>(&args)...};
  return hipLaunchKernel(reinterpret_cast<const void *>(kernel),
                         dim3(unsigned(blocks)), dim3(unsigned(threads)), argv,
                         0, stream);
}

// Multi-frequency encoding: plane 2j holds sin_a(2^j x), plane 2j+1
// cos_a(2^j x), j < nfreq, each plane n elements long.  One read of x, 2 nfreq
// writes; 2^j x is exact (it overflows to +-Inf, hence NaN, only for
// |x| >= 2^(128-j) in FP32, 2^(1024-j) in FP64).  VEC_PATH: 16-byte accesses
// (every plane then starts 16-byte aligned at element `head`), U of them per
// thread, block-strided, so that per frequency a workgroup writes U * 2 KiB
// contiguous to each plane and issues the U stores of one plane together;
// otherwise one element per lane.  Nontemporal device-scope stores.  At 2^26
// FP32 inputs and 8 frequencies, U = 4 moves 6.47 TB/s against 6.02 for
// U = 1 (0.94 of the same-run write-only fill); launch bounds asking for two
// or four waves per SIMD made the compiler spill and fall to ~0.95 TB/s.
// FP32 runs one-wave groups (ahead of 128 threads on 12 of 12 array
// placements in two processes, mean +0.9 %; issuing the loads before the
// table fill added nothing), BF16 and FP64 128-thread groups.
template <class ST>
constexpr int encode_unroll() {
  return sizeof(typename ST::raw) == 4 ? 4 : 1;
}
template <class ST>
constexpr int encode_block() {
  return sizeof(typename ST::raw) == 4 ? 64 : 128;
}
__device__ inline float pow2(int j, float) {
  return __uint_as_float(uint32_t(127 + j) << 23);
}
__device__ inline double pow2(int j, double) {
  return __longlong_as_double(int64_t(1023 + j) << 52);
}
template <class ST, bool VEC_PATH, int UNROLL, int BLOCK>
__global__ __launch_bounds__(BLOCK) void encode_kernel(
    const char *x, char *y, int64_t n, int nfreq, int64_t head, int64_t nvec) {
  using raw = typename ST::raw;
  using val = typename ST::val;
  using Core = FwdOp<kSin | kCos, false, sizeof(raw) == 2>;
  constexpr int VEC = VEC_PATH ? ST::kVec : 1;
  constexpr int U = VEC_PATH ? UNROLL : 1;
  __shared__ typename Core::Table tb;
  Core::Table::init(tb);
  __syncthreads();
  const int64_t plane = n * int64_t(sizeof(raw));
  const int64_t v0 = int64_t(blockIdx.x) * (U * BLOCK) + threadIdx.x;
  const char *xb = x + head * int64_t(sizeof(raw));
  val xf[U][VEC];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int64_t v = v0 + int64_t(u) * BLOCK;
#pragma unroll
    for (int e = 0; e < VEC; ++e) xf[u][e] = val(0);
    if (v < nvec) {
      if constexpr (VEC_PATH) {
        ST::unpack(vload<false, typename ST::vec>(xb, v), xf[u]);
      } else {
        xf[u][0] = ST::load(reinterpret_cast<const raw *>(x)[v]);
      }
    }
  }
  if (v0 < nvec) {
    for (int j = 0; j < nfreq; ++j) {
      val sv[U][VEC], cv[U][VEC];
#pragma unroll
      for (int u = 0; u < U; ++u) {
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          const val in[1] = {xf[u][e] * pow2(j, val())};
          val out[2];
          Core::apply(in, out, tb, 0u);
          sv[u][e] = out[0];
          cv[u][e] = out[1];
        }
      }
      char *ps = y + (2 * j) * plane + head * int64_t(sizeof(raw));
      char *pc = ps + plane;
      if constexpr (VEC_PATH) {
        // this group's span of each plane, one SpanStore each
        constexpr int kVB = int(sizeof(typename ST::vec));
        const int64_t span0 = int64_t(blockIdx.x) * (U * BLOCK);
        const SpanStore ss(ps + span0 * kVB, U * BLOCK * kVB);
        const SpanStore sc(pc + span0 * kVB, U * BLOCK * kVB);
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int64_t v = v0 + int64_t(u) * BLOCK;
          if (v < nvec) ss.put(uint32_t(v - span0) * kVB, ST::pack(sv[u]));
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int64_t v = v0 + int64_t(u) * BLOCK;
          if (v < nvec) sc.put(uint32_t(v - span0) * kVB, ST::pack(cv[u]));
        }
      } else {
        if (v0 < nvec) {
          reinterpret_cast<raw *>(ps)[v0] = ST::store(sv[0][0]);
          reinterpret_cast<raw *>(pc)[v0] = ST::store(cv[0][0]);
        }
      }
    }
  }
  if (VEC_PATH && blockIdx.x == 0) {  // scalar head and tail
    const int64_t tail0 = head + nvec * VEC;
    const int64_t extra = head + (n - tail0);
    for (int64_t e = threadIdx.x; e < extra; e += BLOCK) {
      const int64_t i = e < head ? e : tail0 + (e - head);
      const val xi = ST::load(reinterpret_cast<const raw *>(x)[i]);
      for (int j = 0; j < nfreq; ++j) {
        const val in[1] = {xi * pow2(j, val())};
        val out[2];
        Core::apply(in, out, tb, 0u);
        reinterpret_cast<raw *>(y + (2 * j) * plane)[i] = ST::store(out[0]);
        reinterpret_cast<raw *>(y + (2 * j + 1) * plane)[i] = ST::store(out[1]);
      }
    }
  }
}

template <class ST>
hipError_t launch_encode(const void *x, void *y, int64_t n, int nfreq,
                         hipStream_t stream) {
  using raw = typename ST::raw;
  constexpr int VEC = ST::kVec;
  const uintptr_t mis = uintptr_t(x) & 15u;
  const bool vec_ok = (uintptr_t(y) & 15u) == mis && mis % sizeof(raw) == 0 &&
                      (n * int64_t(sizeof(raw))) % 16 == 0;
  const char *xc = static_cast<const char *>(x);
  char *yc = static_cast<char *>(y);
  if (vec_ok) {
    int64_t head = mis ? int64_t((16u - mis) / sizeof(raw)) : 0;
    if (head > n) head = n;
    const int64_t nvec = (n - head) / VEC;
    constexpr int kBlock = encode_block<ST>();
    const int64_t per = int64_t(encode_unroll<ST>()) * kBlock;
    int64_t blocks = (nvec + per - 1) / per;
    if (blocks < 1) blocks = 1;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    return launch(encode_kernel<ST, true, encode_unroll<ST>(), kBlock>,
                  blocks, kBlock, stream, xc, yc, n, nfreq, head, nvec);
  } else {
    constexpr int kBlock = 128;
    const int64_t blocks = (n + kBlock - 1) / kBlock;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    return launch(encode_kernel<ST, false, 1, kBlock>, blocks, kBlock, stream,
                  xc, yc, n, nfreq, int64_t(0), n);
  }
}

// ---------------------------------------------------------------------------
// Bandwidth probes (measurement comparators, not the method): plain 16-byte
// streams with one access per stream per thread, the kernels' pattern, to
// measure what HBM delivers for a byte mix.  The read probe folds each
// vector to one word and stores it only when it equals `key` (a value the
// caller picks; the store target is a 1024-word sink), so that the loads
// stay live while the probe writes next to nothing.
// ---------------------------------------------------------------------------
template <int BLOCK, bool NTL>
__global__ __launch_bounds__(BLOCK) void probe_read_kernel(const char *x,
                                                           int64_t nvec,
                                                           uint32_t key,
                                                           uint32_t *sink) {
  const int64_t v = int64_t(blockIdx.x) * BLOCK + threadIdx.x;
  if (v < nvec) {
    const u32x4 w = vload<NTL>(x, v);
    const uint32_t acc = w[0] ^ w[1] ^ w[2] ^ w[3];
    if (acc == key) sink[blockIdx.x & 1023u] = acc;
  }
}
// Writes (NIN = 0) or copies (NIN = 1) into NOUT arrays.  STORE: 0 plain,
// 1 nontemporal, 2 nontemporal at device scope (the kernels' SpanStore).
template <int BLOCK, int NIN, int NOUT, bool NTL, int STORE>
__global__ __launch_bounds__(BLOCK) void probe_stream_kernel(IoPtrs io,
                                                             int64_t nvec) {
  const int64_t v = int64_t(blockIdx.x) * BLOCK + threadIdx.x;
  if (v < nvec) {
    u32x4 w = {uint32_t(v), 0u, 0u, 0u};
    if constexpr (NIN == 1) w = vload<NTL>(io.in[0], v);
#pragma unroll
    for (int k = 0; k < NOUT; ++k) {
      if constexpr (STORE == 2) {
        const int64_t span0 = int64_t(blockIdx.x) * BLOCK;
        const SpanStore ss(io.out[k] + span0 * 16, BLOCK * 16);
        ss.put(uint32_t(v - span0) * 16u, w);
      } else {
        vstore<STORE == 1>(io.out[k], v, w);
      }
    }
  }
}

template <int BLOCK, bool NTL, int STORE>
hipError_t launch_probe(int kind, const void *x, void *const *out, int n_out,
                        int64_t nvec, hipStream_t s) {
  const int64_t blocks = (nvec + BLOCK - 1) / BLOCK;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  if (kind == 0)
    return launch(probe_read_kernel<BLOCK, NTL>, blocks, BLOCK, s,
                  static_cast<const char *>(x), nvec, 0x9e3779b9u,
                  static_cast<uint32_t *>(out[0]));
  IoPtrs io{};
  io.in[0] = static_cast<const char *>(x);
  for (int k = 0; k < n_out; ++k) io.out[k] = static_cast<char *>(out[k]);
  switch ((kind == 2 ? 4 : 0) + n_out) {
    case 1: return launch(probe_stream_kernel<BLOCK, 0, 1, NTL, STORE>, blocks, BLOCK, s, io, nvec);
    case 2: return launch(probe_stream_kernel<BLOCK, 0, 2, NTL, STORE>, blocks, BLOCK, s, io, nvec);
    case 3: return launch(probe_stream_kernel<BLOCK, 0, 3, NTL, STORE>, blocks, BLOCK, s, io, nvec);
    case 5: return launch(probe_stream_kernel<BLOCK, 1, 1, NTL, STORE>, blocks, BLOCK, s, io, nvec);
    case 6: return launch(probe_stream_kernel<BLOCK, 1, 2, NTL, STORE>, blocks, BLOCK, s, io, nvec);
    default: return launch(probe_stream_kernel<BLOCK, 1, 3, NTL, STORE>, blocks, BLOCK, s, io, nvec);
  }
}
template <int BLOCK>
hipError_t launch_probe_flags(int kind, const void *x, void *const *out,
                              int n_out, int64_t nvec, uint32_t flags,
                              hipStream_t s) {
  const bool ntl = flags & TA_PROBE_NT_LOAD;
  const int store = (flags & TA_PROBE_NT_STORE)
                        ? ((flags & TA_PROBE_DEVICE_SCOPE) ? 2 : 1) : 0;
  switch ((ntl ? 3 : 0) + store) {
    case 0: return launch_probe<BLOCK, false, 0>(kind, x, out, n_out, nvec, s);
    case 1: return launch_probe<BLOCK, false, 1>(kind, x, out, n_out, nvec, s);
    case 2: return launch_probe<BLOCK, false, 2>(kind, x, out, n_out, nvec, s);
    case 3: return launch_probe<BLOCK, true, 0>(kind, x, out, n_out, nvec, s);
    case 4: return launch_probe<BLOCK, true, 1>(kind, x, out, n_out, nvec, s);
    default: return launch_probe<BLOCK, true, 2>(kind, x, out, n_out, nvec, s);
  }
}

// Fallback when the buffers disagree on their address modulo 16.
constexpr int kScalarBlock = 256;
template <class ST, class Op>
__global__ __launch_bounds__(kScalarBlock) void map_scalar_kernel(IoPtrs io,
                                                                  int64_t n) {
  __shared__ typename Op::Table tb;
  if constexpr (Op::Table::kUsed) {
    Op::Table::init(tb);
    __syncthreads();
  }
  const int64_t stride = int64_t(gridDim.x) * kScalarBlock;
  for (int64_t i = int64_t(blockIdx.x) * kScalarBlock + threadIdx.x; i < n;
       i += stride)
    scalar_element<ST, Op>(io, i, tb);
}

// Inputs of at most 256 MiB in all (the Infinity Cache's size) are read with
// plain loads whatever the shape says: a launch after the one that wrote or
// read the arrays then hits in the cache, which nontemporal loads would pass
// by.  On MI355X, arrays re-read launch after launch: single-output kernels
// +7-34 % with plain loads up to 256 MiB of input (FP32 sin at 2^23: 773
// against 651 Gelem/s; FP64 sin at 2^22: 400 against 297), nontemporal loads
// +2-4 % from 512 MiB; the two- and three-input backward kernels the same
// (sin backward +5-25 % up to 256 MiB read, -5 % from 512 MiB; the sincos
// backward +18 % at 192 MiB, -3.5 % at 384 MiB); below 32 MiB in and out
// either is the same.
constexpr int64_t kCacheResidentBytes = int64_t(256) << 20;

// The vector body in shape SH over [head, head + nvec*VEC) (plus the scalar
// head and tail), with the load policy by size above.
template <class ST, class Op, const Shape &SH>
hipError_t launch_vec(const IoPtrs &io, int64_t head, int64_t nvec, int64_t n,
                      hipStream_t stream) {
  using raw = typename ST::raw;
  const int64_t per_block = int64_t(SH.unroll) * SH.block;
  int64_t blocks = (nvec + per_block - 1) / per_block;
  if (blocks < 1) blocks = 1;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  if constexpr (SH.nt_load) {
    if (n <= kCacheResidentBytes / int64_t(Op::NIN * sizeof(raw)))
      return launch(
          map_vec_kernel<ST, Op, SH.block, SH.unroll, false, SH.nt_store,
                         SH.min_waves, SH.loads_first, SH.grouped>,
          blocks, SH.block, stream, io, head, nvec, n);
  }
  return launch(
      map_vec_kernel<ST, Op, SH.block, SH.unroll, SH.nt_load, SH.nt_store,
                     SH.min_waves, SH.loads_first, SH.grouped>,
      blocks, SH.block, stream, io, head, nvec, n);
}

template <class ST, class Op>
hipError_t launch_map(const void *const *in, void *const *out, int64_t n,
                      hipStream_t stream, uint32_t flags) {
  using raw = typename ST::raw;
  constexpr int VEC = ST::kVec;
  IoPtrs io{};
  io.flags = flags;
  const uintptr_t mis = uintptr_t(in[0]) & 15u;
  bool same = (mis % sizeof(raw)) == 0;
  for (int k = 0; k < Op::NIN; ++k) {
    io.in[k] = static_cast<const char *>(in[k]);
    same = same && ((uintptr_t(in[k]) & 15u) == mis);
  }
  for (int k = 0; k < Op::NOUT; ++k) {
    io.out[k] = static_cast<char *>(out[k]);
    same = same && ((uintptr_t(out[k]) & 15u) == mis);
  }
  if (same) {
    int64_t head = mis ? int64_t((16u - mis) / sizeof(raw)) : 0;
    if (head > n) head = n;
    const int64_t nvec = (n - head) / VEC;
    static constexpr Shape sh = shape_for<ST, Op>();
    // the grouped shape is for streams from HBM; inputs that fit the
    // Infinity Cache take the one-access shape (sin+cos+tan at 2^22-2^26
    // FP32: 0.2-11 % faster that way, 1-1.5 % slower from 2^27)
    if constexpr (sh.grouped) {
      if (n <= kCacheResidentBytes / int64_t(Op::NIN * sizeof(raw)))
        return launch_vec<ST, Op, kShapeMulti>(io, head, nvec, n, stream);
    }
    return launch_vec<ST, Op, sh>(io, head, nvec, n, stream);
  }
  int64_t blocks = (n + kScalarBlock - 1) / kScalarBlock;
  if (blocks > 65536) blocks = 65536;
  return launch(map_scalar_kernel<ST, Op>, blocks, kScalarBlock, stream, io,
                n);
}

// 16-bit storage takes 8-byte accesses (F16x4/BF16x4) for one input and
// several outputs, and for two inputs and two outputs (the fused forward and
// backward) on inputs above 256 MiB; 16-byte ones otherwise.  (The fused
// forward and backward over [64, 4096, 256] BF16, 256 MiB of input, ran at
// 772 Gelem/s with 8-byte accesses against 833 with 16-byte ones in the
// benchmark's sequence of launches.)
template <class Op>
bool eight_byte_16bit(int64_t n) {
  if constexpr (Op::NIN == 1 && Op::NOUT >= 2) return true;
  if constexpr (Op::NIN == 2 && Op::NOUT == 2)
    return n > kCacheResidentBytes / int64_t(2 * sizeof(uint16_t));
  return false;
}

template <class Op>
hipError_t launch_dtype(ta_dtype dt, const void *const *in, void *const *out,
                        int64_t n, hipStream_t s, uint32_t flags) {
  switch (dt) {
    case TA_F32: return launch_map<F32, Op>(in, out, n, s, flags);
    case TA_F16:
      if (eight_byte_16bit<typename Op::LowH>(n))
        return launch_map<F16x4, typename Op::LowH>(in, out, n, s, flags);
      return launch_map<F16, typename Op::LowH>(in, out, n, s, flags);
    case TA_BF16:
      if (eight_byte_16bit<typename Op::Low>(n))
        return launch_map<BF16x4, typename Op::Low>(in, out, n, s, flags);
      return launch_map<BF16, typename Op::Low>(in, out, n, s, flags);
    case TA_F64: return launch_map<F64, Op>(in, out, n, s, flags);
    default: break;
  }
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Host-side validation (before any HIP call)
// ---------------------------------------------------------------------------
thread_local int g_last_hip_error = 0;

inline size_t dtype_size(ta_dtype dt) {
  return dt == TA_F64 ? 8 : (dt == TA_F32 ? 4 : 2);
}
inline bool dtype_ok(int dt) {
  return dt == TA_F32 || dt == TA_F16 || dt == TA_BF16 || dt == TA_F64;
}

// Outputs may alias an input exactly; any other overlap is an error.
inline bool overlap_ok(const void *const *in, int nin, void *const *out,
                       int nout, int64_t n, size_t es) {
  const uintptr_t bytes = uintptr_t(n) * es;
  auto inter = [&](uintptr_t a, uintptr_t b) { return a < b + bytes && b < a + bytes; };
  for (int j = 0; j < nout; ++j) {
    const uintptr_t o = uintptr_t(out[j]);
    for (int i = 0; i < nin; ++i) {
      const uintptr_t p = uintptr_t(in[i]);
      if (o != p && inter(o, p)) return false;
    }
    for (int k = 0; k < j; ++k)
      if (inter(o, uintptr_t(out[k]))) return false;
  }
  return true;
}

inline ta_status check_common(const void *const *in, int nin, void *const *out,
                              int nout, int64_t n, int dt) {
  if (!dtype_ok(dt)) return TA_EDTYPE;
  if (n < 0) return TA_EINVAL;
  if (n == 0) return TA_OK;
  for (int i = 0; i < nin; ++i)
    if (!in[i]) return TA_EINVAL;
  for (int j = 0; j < nout; ++j)
    if (!out[j]) return TA_EINVAL;
  if (!overlap_ok(in, nin, out, nout, n, dtype_size(ta_dtype(dt))))
    return TA_EOVERLAP;
  return TA_OK;
}

inline ta_status finish(hipError_t e) {
  if (e != hipSuccess) {
    g_last_hip_error = int(e);
    return TA_EHIP;
  }
  return TA_OK;
}

template <class Op>
ta_status run(const void *const *in, void *const *out, int64_t n, ta_dtype dt,
              hipStream_t s, uint32_t flags = 0u) {
  const ta_status st = check_common(in, Op::NIN, out, Op::NOUT, n, dt);
  if (st != TA_OK || n == 0) return st;
  return finish(launch_dtype<Op>(dt, in, out, n, s, flags));
}

template <int MASK>
ta_status paper(const void *x, void *const *outs, int64_t n, ta_dtype dt,
                uint32_t flags, hipStream_t s) {
  const void *in[1] = {x};
  return run<PaperOp<MASK>>(in, outs, n, dt, s, flags);
}

template <int MASK, bool GUARD>
ta_status fwd(const void *x, void *const *outs, int64_t n, ta_dtype dt,
              hipStream_t s) {
  const void *in[1] = {x};
  return run<FwdOp<MASK, GUARD>>(in, outs, n, dt, s);
}

// Flags of the *_ex forward calls.  TA_FLAG_FORCE_FP32_REDUCTION selects the
// FP32 evaluation for FP32 storage (16-bit storage always uses it); it is
// not valid for FP64 storage or together with TA_FLAG_FORCE_FP64_REDUCTION.
inline ta_status check_fwd_flags(uint32_t flags, ta_dtype dt) {
  if (!dtype_ok(dt)) return TA_EDTYPE;
  const uint32_t known = TA_FLAG_TAN_GUARD | TA_FLAG_FORCE_FP64_REDUCTION |
                         TA_FLAG_FORCE_FP32_REDUCTION;
  if (flags & ~known) return TA_EINVAL;
  if ((flags & TA_FLAG_FORCE_FP32_REDUCTION) &&
      ((flags & TA_FLAG_FORCE_FP64_REDUCTION) || dt == TA_F64))
    return TA_EINVAL;
  return TA_OK;
}

template <int MASK, bool GUARD>
ta_status fwd_ex(const void *x, void *const *outs, int64_t n, ta_dtype dt,
                 uint32_t flags, hipStream_t s) {
  const ta_status st = check_fwd_flags(flags, dt);
  if (st != TA_OK) return st;
  if ((flags & TA_FLAG_FORCE_FP32_REDUCTION) && dt == TA_F32) {
    using Op = FwdOp<MASK, GUARD, false, true>;
    const void *in[1] = {x};
    const ta_status c = check_common(in, Op::NIN, outs, Op::NOUT, n, dt);
    if (c != TA_OK || n == 0) return c;
    return finish(launch_map<F32, Op>(in, outs, n, s, 0u));
  }
  return fwd<MASK, GUARD>(x, outs, n, dt, s);
}

template <int MASK>
ta_status taylor(const void *x, void *y, int64_t n, int terms, ta_dtype dt,
                 hipStream_t s) {
  if (!dtype_ok(dt)) return TA_EDTYPE;
  const void *in[1] = {x};
  void *out[1] = {y};
  switch (terms) {
    case 5: return run<TaylorOp<MASK, 5>>(in, out, n, dt, s);
    case 7: return run<TaylorOp<MASK, 7>>(in, out, n, dt, s);
    case 9: return run<TaylorOp<MASK, 9>>(in, out, n, dt, s);
  }
  return TA_EINVAL;
}

template <int WHICH, bool WITH_Y>
ta_status bwd(const void *x, const void *gy, void *y, void *gx, int64_t n,
              ta_dtype dt, hipStream_t s) {
  const void *in[2] = {x, gy};
  if constexpr (WITH_Y) {
    void *out[2] = {y, gx};
    return run<BwdOp<WHICH, true>>(in, out, n, dt, s);
  } else {
    void *out[1] = {gx};
    return run<BwdOp<WHICH, false>>(in, out, n, dt, s);
  }
}

}  // namespace ta

using namespace ta;

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

ta_status ta_sin_ex(const void *x, void *y, int64_t n, ta_dtype dt,
                    hipStream_t s, uint32_t flags) {
  void *o[1] = {y};
  return fwd_ex<kSin, false>(x, o, n, dt, flags, s);
}

ta_status ta_sin(const void *x, void *y, int64_t n, ta_dtype dt, hipStream_t s) {
  return ta_sin_ex(x, y, n, dt, s, 0u);
}

ta_status ta_cos_ex(const void *x, void *y, int64_t n, ta_dtype dt,
                    hipStream_t s, uint32_t flags) {
  void *o[1] = {y};
  return fwd_ex<kCos, false>(x, o, n, dt, flags, s);
}

ta_status ta_cos(const void *x, void *y, int64_t n, ta_dtype dt, hipStream_t s) {
  return ta_cos_ex(x, y, n, dt, s, 0u);
}

ta_status ta_tan_ex(const void *x, void *y, int64_t n, ta_dtype dt,
                    hipStream_t s, uint32_t flags) {
  void *o[1] = {y};
  if (flags & TA_FLAG_TAN_GUARD) return fwd_ex<kTan, true>(x, o, n, dt, flags, s);
  return fwd_ex<kTan, false>(x, o, n, dt, flags, s);
}

ta_status ta_tan(const void *x, void *y, int64_t n, ta_dtype dt, hipStream_t s) {
  return ta_tan_ex(x, y, n, dt, s, 0u);
}

ta_status ta_sincos_ex(const void *x, void *ys, void *yc, void *yt, int64_t n,
                       ta_dtype dt, hipStream_t s, uint32_t flags) {
  if (yt) {
    void *o[3] = {ys, yc, yt};
    if (flags & TA_FLAG_TAN_GUARD)
      return fwd_ex<kSin | kCos | kTan, true>(x, o, n, dt, flags, s);
    return fwd_ex<kSin | kCos | kTan, false>(x, o, n, dt, flags, s);
  }
  void *o[2] = {ys, yc};
  return fwd_ex<kSin | kCos, false>(x, o, n, dt, flags, s);
}

ta_status ta_sincos(const void *x, void *ys, void *yc, void *yt, int64_t n,
                    ta_dtype dt, hipStream_t s) {
  return ta_sincos_ex(x, ys, yc, yt, n, dt, s, 0u);
}

ta_status ta_taylor_sin(const void *x, void *y, int64_t n, int terms,
                        ta_dtype dt, hipStream_t s) {
  return taylor<kSin>(x, y, n, terms, dt, s);
}
ta_status ta_taylor_cos(const void *x, void *y, int64_t n, int terms,
                        ta_dtype dt, hipStream_t s) {
  return taylor<kCos>(x, y, n, terms, dt, s);
}
ta_status ta_taylor_tan(const void *x, void *y, int64_t n, int terms,
                        ta_dtype dt, hipStream_t s) {
  return taylor<kTan>(x, y, n, terms, dt, s);
}

ta_status ta_sin_bwd(const void *x, const void *gy, void *gx, int64_t n,
                     ta_dtype dt, hipStream_t s) {
  return bwd<kSin, false>(x, gy, nullptr, gx, n, dt, s);
}
ta_status ta_cos_bwd(const void *x, const void *gy, void *gx, int64_t n,
                     ta_dtype dt, hipStream_t s) {
  return bwd<kCos, false>(x, gy, nullptr, gx, n, dt, s);
}
ta_status ta_tan_bwd(const void *x, const void *gy, void *gx, int64_t n,
                     ta_dtype dt, hipStream_t s) {
  return bwd<kTan, false>(x, gy, nullptr, gx, n, dt, s);
}

ta_status ta_sincos_bwd(const void *x, const void *gs, const void *gc,
                        void *gx, int64_t n, ta_dtype dt, hipStream_t s) {
  if (!dtype_ok(dt)) return TA_EDTYPE;
  void *out[1] = {gx};
  if (gs && gc) {
    const void *in[3] = {x, gs, gc};
    return run<SinCosBwdOp<true, true>>(in, out, n, dt, s);
  }
  if (gs) {
    const void *in[2] = {x, gs};
    return run<SinCosBwdOp<true, false>>(in, out, n, dt, s);
  }
  if (gc) {
    const void *in[2] = {x, gc};
    return run<SinCosBwdOp<false, true>>(in, out, n, dt, s);
  }
  return n < 0 || n > 0 ? TA_EINVAL : TA_OK;
}

ta_status ta_sin_fwdbwd(const void *x, const void *gy, void *y, void *gx,
                        int64_t n, ta_dtype dt, hipStream_t s) {
  return bwd<kSin, true>(x, gy, y, gx, n, dt, s);
}
ta_status ta_cos_fwdbwd(const void *x, const void *gy, void *y, void *gx,
                        int64_t n, ta_dtype dt, hipStream_t s) {
  return bwd<kCos, true>(x, gy, y, gx, n, dt, s);
}
ta_status ta_tan_fwdbwd(const void *x, const void *gy, void *y, void *gx,
                        int64_t n, ta_dtype dt, hipStream_t s) {
  return bwd<kTan, true>(x, gy, y, gx, n, dt, s);
}

ta_status ta_builtin_sincos(const void *x, void *ys, void *yc, void *yt,
                            int64_t n, int kind, ta_dtype dt, hipStream_t s) {
  if (!dtype_ok(dt)) return TA_EDTYPE;
  if (kind < 0 || kind > 2) return TA_EINVAL;
  if (dt == TA_F64 && kind == 1) return TA_EDTYPE;
  if (!ys || (yt && !yc)) return n == 0 ? TA_OK : TA_EINVAL;
  const void *in[1] = {x};
  void *o[3] = {ys, yc, yt};
  const int no = yt ? 3 : (yc ? 2 : 1);
  switch (kind * 4 + no) {
    case 0 * 4 + 1: return run<BuiltinOp<0, 1>>(in, o, n, dt, s);
    case 0 * 4 + 2: return run<BuiltinOp<0, 2>>(in, o, n, dt, s);
    case 0 * 4 + 3: return run<BuiltinOp<0, 3>>(in, o, n, dt, s);
    case 1 * 4 + 1: return run<BuiltinOp<1, 1>>(in, o, n, dt, s);
    case 1 * 4 + 2: return run<BuiltinOp<1, 2>>(in, o, n, dt, s);
    case 1 * 4 + 3: return run<BuiltinOp<1, 3>>(in, o, n, dt, s);
    case 2 * 4 + 1: return run<BuiltinOp<2, 1>>(in, o, n, dt, s);
    case 2 * 4 + 2: return run<BuiltinOp<2, 2>>(in, o, n, dt, s);
    default: return run<BuiltinOp<2, 3>>(in, o, n, dt, s);
  }
}

ta_status ta_builtin_sin_fwdbwd(const void *x, const void *gy, void *y,
                                void *gx, int64_t n, int kind, ta_dtype dt,
                                hipStream_t s) {
  if (!dtype_ok(dt)) return TA_EDTYPE;
  if (kind < 0 || kind > 1) return TA_EINVAL;
  if (dt == TA_F64 && kind == 1) return TA_EDTYPE;
  const void *in[2] = {x, gy};
  void *o[2] = {y, gx};
  if (kind == 0) return run<BuiltinFwdBwdOp<0>>(in, o, n, dt, s);
  return run<BuiltinFwdBwdOp<1>>(in, o, n, dt, s);
}

ta_status ta_copy(const void *const *in, int n_in, void *const *out, int n_out,
                  int64_t n, ta_dtype dt, hipStream_t s) {
  if (!dtype_ok(dt)) return TA_EDTYPE;
  if (!in || !out || n_in < 1 || n_in > 3 || n_out < 1 || n_out > 3)
    return TA_EINVAL;
  switch (n_in * 4 + n_out) {
    case 1 * 4 + 1: return run<CopyOp<1, 1>>(in, out, n, dt, s);
    case 1 * 4 + 2: return run<CopyOp<1, 2>>(in, out, n, dt, s);
    case 1 * 4 + 3: return run<CopyOp<1, 3>>(in, out, n, dt, s);
    case 2 * 4 + 1: return run<CopyOp<2, 1>>(in, out, n, dt, s);
    case 2 * 4 + 2: return run<CopyOp<2, 2>>(in, out, n, dt, s);
    case 2 * 4 + 3: return run<CopyOp<2, 3>>(in, out, n, dt, s);
    case 3 * 4 + 1: return run<CopyOp<3, 1>>(in, out, n, dt, s);
    case 3 * 4 + 2: return run<CopyOp<3, 2>>(in, out, n, dt, s);
    default: return run<CopyOp<3, 3>>(in, out, n, dt, s);
  }
}

ta_status ta_stream_probe(int kind, const void *x, void *const *out,
                          int n_out, int64_t n, uint32_t flags,
                          hipStream_t s) {
  if (kind < 0 || kind > 2 || n < 0) return TA_EINVAL;
  if (flags & ~uint32_t(TA_PROBE_NT_LOAD | TA_PROBE_NT_STORE |
                       TA_PROBE_BLOCK256 | TA_PROBE_DEVICE_SCOPE))
    return TA_EINVAL;
  if ((flags & TA_PROBE_DEVICE_SCOPE) && !(flags & TA_PROBE_NT_STORE))
    return TA_EINVAL;
  if (kind == 0 ? n_out != 1 : (n_out < 1 || n_out > 3)) return TA_EINVAL;
  if (n == 0) return TA_OK;
  if (!out) return TA_EINVAL;
  if (n % 4 != 0 || (kind != 1 && (!x || (uintptr_t(x) & 15u))))
    return TA_EINVAL;
  for (int k = 0; k < n_out; ++k)
    if (!out[k] || (uintptr_t(out[k]) & 15u)) return TA_EINVAL;
  // the read probe's sink is 1024 words; the other outputs are n floats
  const uintptr_t obytes = kind == 0 ? 4096u : uintptr_t(n) * 4u;
  const uintptr_t ib = uintptr_t(x), ibytes = uintptr_t(n) * 4u;
  for (int j = 0; j < n_out; ++j) {
    const uintptr_t o = uintptr_t(out[j]);
    if (kind != 1 && o < ib + ibytes && ib < o + obytes) return TA_EOVERLAP;
    for (int k = 0; k < j; ++k) {
      const uintptr_t p = uintptr_t(out[k]);
      if (o < p + obytes && p < o + obytes) return TA_EOVERLAP;
    }
  }
  const int64_t nvec = n / 4;
  const hipError_t e =
      (flags & TA_PROBE_BLOCK256)
          ? launch_probe_flags<256>(kind, x, out, n_out, nvec, flags, s)
          : launch_probe_flags<64>(kind, x, out, n_out, nvec, flags, s);
  return finish(e);
}

ta_status ta_paper_sincos(const void *x, void *ys, void *yc, void *yt,
                          int64_t n, ta_dtype dt, hipStream_t s,
                          uint32_t flags) {
  if (!dtype_ok(dt)) return TA_EDTYPE;
  if (flags & ~uint32_t(TA_FLAG_TAN_GUARD | TA_FLAG_LITERAL_DIVISOR |
                       TA_FLAG_FORCE_FP64_REDUCTION))
    return TA_EINVAL;
  void *o[3];
  int m = 0, k = 0;
  if (ys) { o[k++] = ys; m |= kSin; }
  if (yc) { o[k++] = yc; m |= kCos; }
  if (yt) { o[k++] = yt; m |= kTan; }
  switch (m) {
    case kSin: return paper<kSin>(x, o, n, dt, flags, s);
    case kCos: return paper<kCos>(x, o, n, dt, flags, s);
    case kTan: return paper<kTan>(x, o, n, dt, flags, s);
    case kSin | kCos: return paper<kSin | kCos>(x, o, n, dt, flags, s);
    case kSin | kTan: return paper<kSin | kTan>(x, o, n, dt, flags, s);
    case kCos | kTan: return paper<kCos | kTan>(x, o, n, dt, flags, s);
    case kSin | kCos | kTan:
      return paper<kSin | kCos | kTan>(x, o, n, dt, flags, s);
  }
  return n < 0 || n > 0 ? TA_EINVAL : TA_OK;  // no output requested
}

ta_status ta_sincos_encode(const void *x, void *y, int64_t n, int nfreq,
                           ta_dtype dt, hipStream_t s) {
  if (!dtype_ok(dt)) return TA_EDTYPE;
  if (n < 0 || nfreq < 1 || nfreq > 16) return TA_EINVAL;
  if (n == 0) return TA_OK;
  if (!x || !y) return TA_EINVAL;
  const uintptr_t es = dtype_size(dt);
  const uintptr_t xb = uintptr_t(x), yb = uintptr_t(y);
  const uintptr_t xe = xb + uintptr_t(n) * es;
  const uintptr_t ye = yb + uintptr_t(n) * es * uintptr_t(2 * nfreq);
  if (xb < ye && yb < xe) return TA_EOVERLAP;
  hipError_t e = hipErrorInvalidValue;
  switch (dt) {
    case TA_F32: e = launch_encode<F32>(x, y, n, nfreq, s); break;
    case TA_F16: e = launch_encode<F16>(x, y, n, nfreq, s); break;
    case TA_BF16: e = launch_encode<BF16>(x, y, n, nfreq, s); break;
    case TA_F64: e = launch_encode<F64>(x, y, n, nfreq, s); break;
    default: break;
  }
  return finish(e);
}

const char *ta_status_str(ta_status st) {
  switch (st) {
    case TA_OK: return "TA_OK";
    case TA_EINVAL: return "TA_EINVAL: invalid argument";
    case TA_EDTYPE: return "TA_EDTYPE: unsupported dtype";
    case TA_EOVERLAP: return "TA_EOVERLAP: output partially overlaps another buffer";
    case TA_EHIP: return "TA_EHIP: HIP launch failed";
    default: break;
  }
  return "unknown ta_status";
}

int ta_last_hip_error(void) { return g_last_hip_error; }

const char *ta_version(void) { return "ta 0.1.0 (gfx950)"; }

}  // extern "C"
