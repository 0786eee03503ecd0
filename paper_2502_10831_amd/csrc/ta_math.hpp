// ta_math.hpp -- per-element device arithmetic of the piecewise trigonometric
// approximations (Goyal & Arora, arXiv 2502.10831) for gfx950.
//
// Split of the work (one element):
//   1. Argument reduction, FP64.  x = q*(pi/2) + r, |r| <= pi/4 up to the
//      rounding of 2/pi in q (FP64 Cody-Waite with a two-word pi/2 below
//      2^29; a 2/pi bit-table reduction above).  a = |r| in degrees gives the
//      piece inside [0, 45] (slot 3 of the table takes the excess); the parity
//      of q says whether the fold angle is rho = a (q even) or its complement
//      (q odd, rho = 90 - a degrees).  This is the Section 3 fold
//      rho = arcsin|sin x|, with the sign of each output from (q mod 4, sign r).
//   2. The piece's two linear forms N, D (Appendix A integer coefficients),
//      FP64, each rounded once to FP32.  Pieces above 45 degrees are written
//      in the complement variable, so D of the last piece is 11 * (90 - t)
//      with no cancellation at the pole.  FP64 FMA issues at the same rate as
//      unpacked FP32 FMA on gfx950, so this costs no more than an FP32
//      reduction with a carried residual and rounds N and D only once.
//   3. Everything after is FP32 (16-bit storage runs steps 1 and 2 in FP32
//      as well; FP64 storage runs every step in FP64, further below):
//      Q = N^2 + D^2 (Appendix A.4), an inverse
//      square root (v_rsq_f32 plus one Newton step whose residual is computed
//      exactly with FMAs), sin = N*y, cos = D*y, and tan = N/D as a reciprocal
//      plus one exact-residual correction.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ta {

// ---------------------------------------------------------------------------
// Constants.  Derived from pi with 400-bit mpmath arithmetic; a CPU test
// re-derives each of them from this file's text.
// ---------------------------------------------------------------------------
constexpr double kTwoOverPi = 0x1.45f306dc9c883p-1;   // RN(2/pi)
constexpr double kPio2Hi = 0x1.921fb54442d18p+0;      // RN(pi/2)
constexpr double kPio2Lo = 0x1.1a62633145c07p-54;     // RN(pi/2 - kPio2Hi)
constexpr double kDegPerRad = 0x1.ca5dc1a63c1f8p+5;   // RN(180/pi)
constexpr double kRoundMagic = 0x1.8p52;              // 1.5 * 2^52
constexpr float kLargeArg = 0x1p29f;  // |x| at and above: bit-table reduction
constexpr float kRoundMagicF = 0x1.8p23f;  // 1.5 * 2^23 (FP32 rounding)

// Bits 1..256 of the binary expansion of 2/pi, most significant first.
__constant__ uint32_t kTwoOverPiBits[8] = {
    0xA2F9836Eu, 0x4E441529u, 0xFC2757D1u, 0xF534DDC0u,
    0xDB629599u, 0x3C439041u, 0xFE5163ABu, 0xDEBBC561u};

// Appendix A integer forms, degrees: tan t ~ (a t + b) / (c t + d).
// Piece 0: eq. (9); 1: eq. (5); 2: eq. (6); 3: eq. (7); 4: eq. (8);
// 5: eq. (10).
constexpr int kA[6] = {11, 10, 6, 10, 4, 1};
constexpr int kB[6] = {0, 10, 46, 217, 297, 542};
constexpr int kC[6] = {-1, -4, -5, -13, -10, -11};
constexpr int kD[6] = {632, 657, 541, 1252, 910, 990};

// Row r = j + 4*(q & 1) of the per-element coefficient table, where j is
// the 15-degree slot of a = |r| in degrees (0-2 on [0, 45]; 3 just above
// 45, reached when q is the neighbour of the nearest quadrant).  q even:
// rho = a, piece k = j, N = b + a_k t, D = d + c_k t with t = a.  q odd:
// rho = 90 - a, piece k = 5 - j, and with t = a (the complement)
// N = (90 a_k + b_k) - a_k t and D = (90 c_k + d_k) - c_k t.  The fold, the
// signs and these forms hold for any |r| < pi/2, so slot 3 (piece 3, or
// piece 2 about 90 degrees) continues both families exactly.
struct PieceRow {
  double iN, sN, iD, sD;  // N = iN + sN t, D = iD + sD t (t in degrees)
};

__host__ __device__ constexpr int piece_of_row(int idx) {
  return idx < 4 ? idx : 5 - (idx - 4);
}

__host__ __device__ constexpr PieceRow piece_row(int idx) {
  const int k = piece_of_row(idx);
  return idx < 4 ? PieceRow{double(kB[k]), double(kA[k]), double(kD[k]),
                            double(kC[k])}
                 : PieceRow{double(90 * kA[k] + kB[k]), double(-kA[k]),
                            double(90 * kC[k] + kD[k]), double(-kC[k])};
}

// (180/pi) * (a_k d_k - b_k c_k): d(tan piece)/d rho = this / D^2, and the
// factor omega of d sin/d rho = omega cos is this / (N^2 + D^2).
__host__ __device__ constexpr double kdet_of_row(int idx) {
  const int k = piece_of_row(idx);
  return kDegPerRad * double(kA[k] * kD[k] - kB[k] * kC[k]);
}

// Per-workgroup copy of the table in LDS (no table in HBM), rows indexed
// j + 4*(q & 1).  Stored as two arrays of 16-byte (intercept, slope) pairs,
// for N and for D: the eight rows of one array then fill 32 distinct LDS
// banks, so a wave reading rows of both quadrant families has no bank
// conflict (rows of 32 bytes put rows j and j + 4 on the same banks).
// One lane writes it with immediates; the caller synchronises.
struct Lin {
  double i, s;  // value = i + s t
};

// Each kernel family writes only the arrays it reads: the forward (FP32 and
// FP64 storage) the N and D pairs, the backward also the derivative factors,
// the 16-bit kernels the FP32 rows and the FP32 factors.
struct TablesFwd {
  Lin n[8], d[8];
  double magic;  // 1.5 2^52, the rounding constant of the reduction
  static constexpr bool kUsed = true;
  __device__ static void fill(TablesFwd &tb) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const PieceRow r = piece_row(i);
      tb.n[i] = Lin{r.iN, r.sN};
      tb.d[i] = Lin{r.iD, r.sD};
    }
    tb.magic = kRoundMagic;
  }
  __device__ static void init(TablesFwd &tb) {
    if (threadIdx.x == 0) fill(tb);
  }
};
struct TablesBwd : TablesFwd {
  double kdet64[8];  // FP64 storage
  float kdet[8];
  __device__ static void init(TablesBwd &tb) {
    if (threadIdx.x == 0) {
      fill(tb);
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        tb.kdet64[i] = kdet_of_row(i);
        tb.kdet[i] = float(kdet_of_row(i));
      }
    }
  }
};
// The table of the FP32 evaluation (16-bit storage, and FP32 storage under
// the FP32-reduction flag) carries the output signs: 32 rows, row =
// j | sr << 2 | q0 << 3 | q1 << 4 (j the 15-degree slot, q0 and q1 the low
// bits of q, sr the sign of r), each holding base row b = j + 4 q0 with N
// negated where sin x is negative, q1 ^ (sr & ~q0), and D negated where
// cos x is negative, q1 ^ (q0 & ~sr).  sin = N y, cos = D y and tan = N / D
// then come out signed (N = iN + sN t with both negated is exactly -N; Q is
// unchanged) and these kernels apply no sign step.  The coefficients are
// integers below 2048, exact in FP16: a row is four FP16 values, 8 bytes, so
// the 32 rows span 256 bytes, one pass over the 64 LDS banks (no two rows
// share a bank), and the FMA reads them as FP16 operands directly
// (v_fma_mix_f32).  The byte offset of a row, 8 row, is one funnel shift
// and one and-or: bits 5-7 of ((q : hr) >> 26) are sr, q0, q1.
constexpr int kRows16 = 32;
__host__ __device__ constexpr int row16_base(int row) {
  return (row & 3) | ((row >> 1) & 4);
}
__host__ __device__ constexpr bool row_sin_neg(int row) {
  return (((row >> 4) & 1) ^ (((row >> 2) & 1) & (((row >> 3) & 1) ^ 1))) != 0;
}
__host__ __device__ constexpr bool row_cos_neg(int row) {
  return (((row >> 4) & 1) ^ (((row >> 3) & 1) & (((row >> 2) & 1) ^ 1))) != 0;
}
// 8 * row for slot j, quadrant bits q and the word whose bit 31 is the
// sign of r.
__device__ inline uint32_t row16_offset(uint32_t j, uint32_t q, uint32_t hr) {
  return (__builtin_amdgcn_alignbit(q, hr, 26) & 0xe0u) | (j << 3);
}
struct alignas(8) CoefH {
  _Float16 iN, sN, iD, sD;
};
// FP16 bit pattern of an integer |v| < 2048 (exact in FP16).
__host__ __device__ constexpr uint32_t half_bits(int v) {
  if (v == 0) return 0u;
  const uint32_t sign = v < 0 ? 0x8000u : 0u;
  const int a = v < 0 ? -v : v;
  int e = 0;
  while ((a >> (e + 1)) != 0) ++e;  // floor(log2 a), at most 10
  return sign | (uint32_t(e + 15) << 10) | (uint32_t(a << (10 - e)) & 0x3ffu);
}
// Base row b as two words of FP16 pairs: (iN, sN) and (iD, sD), low half
// first (the CoefH layout).
__host__ __device__ constexpr uint32_t row_word(int b, int w) {
  return w == 0 ? half_bits(int(piece_row(b).iN)) |
                      (half_bits(int(piece_row(b).sN)) << 16)
                : half_bits(int(piece_row(b).iD)) |
                      (half_bits(int(piece_row(b).sD)) << 16);
}
// The forward table: lanes 0-31 write one row each, the base row's two words
// picked among immediates by selects, the signs by flipping the FP16 sign
// bits of both halves; the caller synchronises.
struct Tables16 {
  CoefH h[kRows16];
  // 1.5 2^23 for the rounding of x 2/pi, read once into a register: an FMA
  // with a register addend and a scalar factor is one instruction, where two
  // immediate operands cost a copy per element.
  float magic;
  static constexpr bool kUsed = true;
  __device__ static void fill_row(Tables16 &tb, int i) {
    const int b = row16_base(i);
    uint32_t w0 = row_word(0, 0), w1 = row_word(0, 1);
#pragma unroll
    for (int k = 1; k < 8; ++k)
      if (b == k) {
        w0 = row_word(k, 0);
        w1 = row_word(k, 1);
      }
    if (row_sin_neg(i)) w0 ^= 0x80008000u;
    if (row_cos_neg(i)) w1 ^= 0x80008000u;
    uint32_t *dst = reinterpret_cast<uint32_t *>(&tb.h[i]);
    dst[0] = w0;
    dst[1] = w1;
    if (i == 0) tb.magic = kRoundMagicF;
  }
  __device__ static void init(Tables16 &tb) {
    if (threadIdx.x < kRows16) fill_row(tb, int(threadIdx.x));
  }
};
// The 16-bit backward adds (180/pi) det of each row's piece.
struct Tables16Bwd : Tables16 {
  float kdet[kRows16];
  __device__ static void fill_row(Tables16Bwd &tb, int i) {
    Tables16::fill_row(tb, i);
    const int b = row16_base(i);
    float kd = float(kdet_of_row(0));
#pragma unroll
    for (int k = 1; k < 8; ++k)
      if (b == k) kd = float(kdet_of_row(k));
    tb.kdet[i] = kd;
  }
  __device__ static void init(Tables16Bwd &tb) {
    if (threadIdx.x < kRows16) fill_row(tb, int(threadIdx.x));
  }
};

// For element functors that need no table.
struct NoTable {
  static constexpr bool kUsed = false;
  __device__ static void init(NoTable &) {}
};

// ---------------------------------------------------------------------------
// 1. Argument reduction
// ---------------------------------------------------------------------------

// |x| >= 2^29 (and +-Inf): x = m * 2^e exactly (m < 2^24, e in [6, 104]).
// x*(2/pi) mod 4 needs only the 2/pi bits from 2^-(e-1) down; a 128-bit
// window of them times m gives q mod 4 and the fraction to ~2^-96.
__device__ inline void reduce_large(float x, double &r, uint32_t &q) {
  const uint32_t ux = __float_as_uint(x);
  const uint32_t ex = (ux >> 23) & 0xffu;
  if (ex == 0xffu) {  // +-Inf (NaN never reaches here)
    r = __builtin_nan("");
    q = 0;
    return;
  }
  const int e = int(ex) - 150;
  const uint32_t m = (ux & 0x7fffffu) | 0x800000u;
  const int i0 = e - 1;  // 1-based index of the first 2/pi bit needed
  const int w0 = (i0 - 1) >> 5;
  const int sh = (i0 - 1) & 31;
  uint32_t w[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const uint64_t pair = (uint64_t(kTwoOverPiBits[w0 + k]) << 32) |
                          kTwoOverPiBits[w0 + k + 1];
    w[k] = uint32_t(pair >> (32 - sh));
  }
  // P = m * window mod 2^128, as four 32-bit words (p3 most significant).
  const uint64_t a3 = uint64_t(m) * w[3], a2 = uint64_t(m) * w[2];
  const uint64_t a1 = uint64_t(m) * w[1], a0 = uint64_t(m) * w[0];
  uint64_t acc = (a3 >> 32) + (a2 & 0xffffffffu);
  const uint32_t p1 = uint32_t(acc);
  acc = (acc >> 32) + (a2 >> 32) + (a1 & 0xffffffffu);
  const uint32_t p2 = uint32_t(acc);
  acc = (acc >> 32) + (a1 >> 32) + (a0 & 0xffffffffu);
  const uint32_t p3 = uint32_t(acc);
  const uint32_t p0 = uint32_t(a3);
  // x*(2/pi) mod 4 = P / 2^126: quadrant = top two bits, fraction below,
  // rounded to nearest by reading the fraction as a signed 126-bit number.
  const uint64_t top = (uint64_t(p3) << 34) | (uint64_t(p2) << 2) | (p1 >> 30);
  const uint32_t nxt = (p1 << 2) | (p0 >> 30);
  const int64_t stop = int64_t(top);
  const double frac = double(stop) * 0x1p-64 + double(nxt) * 0x1p-96;
  uint32_t qq = (p3 >> 30) + uint32_t(stop < 0 ? 1 : 0);
  double rr = __builtin_fma(frac, kPio2Hi, frac * kPio2Lo);
  if (ux >> 31) {
    rr = -rr;
    qq = 0u - qq;
  }
  r = rr;
  q = qq;
}

// r and the low bits of q (two's complement) for any float x, given
// qb = x RN(2/pi) + 1.5 2^52 rounded (q = the integer in the low mantissa
// bits; the rounding of 2/pi can give the neighbour of the nearest quadrant
// for an x next to an odd multiple of pi/4, and |r| then exceeds pi/4 by at
// most |x| 2^-54 pi/2: pieces 2 and 3 meet continuously there and slot 3
// of the table continues both quadrant families).
__device__ inline void reduce_from(float x, double qb, double &r, uint32_t &q) {
  const double xd = double(x);
  const double qd = qb - kRoundMagic;  // +0 when q = 0, so r keeps x's zero
  q = uint32_t(__double2loint(qb));    // low word of the mantissa = q
  double rr = __builtin_fma(-qd, kPio2Hi, xd);  // exact
  r = __builtin_fma(-qd, kPio2Lo, rr);
  if (__builtin_expect(__builtin_fabsf(x) >= kLargeArg, 0)) reduce_large(x, r, q);
}
// Kernels with an LDS table pass 1.5 2^52 from it: held in a register, the
// rounding is one FMA.
__device__ inline void reduce(float x, double &r, uint32_t &q, double magic) {
  reduce_from(x, __builtin_fma(double(x), kTwoOverPi, magic), r, q);
}
// Table-less kernels: a product and an add, both constants from scalar
// registers (one FMA would take a per-element copy of the 64-bit addend).
__device__ inline void reduce(float x, double &r, uint32_t &q) {
  reduce_from(x, double(x) * kTwoOverPi + kRoundMagic, r, q);
}

// Folded element: everything the later stages need.
constexpr double kPi12 = 0x1.0c152382d7366p-2;  // RN(pi/12)

// 15-degree slot of t in [0, 60) degrees: floor(t/15) by a truncating
// conversion (t at or just above 45 gives slot 3, the continuation of both
// families).  Within an ulp of 15 or 30 the product may round across the
// node (the pieces' jump: either side is accepted there).  NaN converts to
// 0.
__device__ inline uint32_t slot_of(double t) {
  return uint32_t(t * (1.0 / 15.0));
}

struct Folded {
  double r;       // reduced argument, |r| <= pi/4 (+ q's rounding; abs_r())
  double t;       // |r| in degrees, [0, 45] (+ the same excess, slot 3)
  uint32_t q;     // quadrant, low bits
  uint32_t hr;    // high word of r: bit 31 = sign of r
  uint32_t row;   // LDS table slot j + 4*(q & 1)
  __device__ double abs_r() const { return __builtin_fabs(r); }
};

__device__ inline Folded fold_finish(Folded f) {
  f.hr = uint32_t(__double2hiint(f.r));
  f.t = f.abs_r() * kDegPerRad;  // the abs folds into the multiply
  // j = 15-degree slot of |r|; the family (q & 1) selects slots 4..6
  const uint32_t j = slot_of(f.t);
  f.row = ((f.q << 2) & 4u) | j;
  return f;
}
__device__ inline Folded fold(float x, double magic) {
  Folded f;
  reduce(x, f.r, f.q, magic);
  return fold_finish(f);
}
__device__ inline Folded fold(float x) {
  Folded f;
  reduce(x, f.r, f.q);
  return fold_finish(f);
}

// Output signs as bit 31 of a word (other bits are don't-care).  With
// a = sign of r, b = q0, c = q1 (all at bit 31), each is one 3-input
// boolean function (one v_bitop3_b32):
//   sin: c ^ (a & ~b)   (q1 ^ sr for even q, q1 for odd q)
//   cos: c ^ (b & ~a)   (q1 for even q, q1 ^ 1 ^ sr for odd q)
//   tan: a ^ b
// Written as the v_bitop3_b32 truth tables (bit i of the table is the
// result for the input bits a b c = i, a most significant), so that the
// negated operand costs no separate v_not: the compiler otherwise shifts a
// negated q, and only bit 31 of any of these words is used.
//   sin: b ^ (a & ~c) = 0x9c,  cos: b ^ (c & ~a) = 0xc6
// with a = hr, b = q << 30, c = q << 31.
template <class F>
__device__ inline uint32_t sin_mask(const F &f) {
  return __builtin_amdgcn_bitop3_b32(f.hr, f.q << 30, f.q << 31, 0x9c);
}
template <class F>
__device__ inline uint32_t cos_mask(const F &f) {
  return __builtin_amdgcn_bitop3_b32(f.hr, f.q << 30, f.q << 31, 0xc6);
}
template <class F>
__device__ inline uint32_t tan_mask(const F &f) { return f.hr ^ (f.q << 31); }

// Applies the sign in bit 31 of m to v: v ^ (m & 0x80000000).  The unsigned
// values of the method (N y, D y, N/D with N, D >= 0) and of the Taylor
// series on [0, pi/2] are non-negative, so this sets the sign.
__device__ inline float flip_sign(float v, uint32_t m) {
  return __uint_as_float(__float_as_uint(v) ^ (m & 0x80000000u));
}
__device__ inline double flip_sign(double v, uint32_t m) {
  return __longlong_as_double(__double_as_longlong(v) ^
                              (int64_t(m & 0x80000000u) << 32));
}

// ---------------------------------------------------------------------------
// 2. Linear forms (FP64, rounded once)
// ---------------------------------------------------------------------------
struct Forms {
  float n, d, q;  // N, D and Q = N^2 + D^2, each rounded once from FP64
};

__device__ inline Forms forms(const Folded &f, const TablesFwd &tb) {
  const Lin a = tb.n[f.row], b = tb.d[f.row];
  const double nd = __builtin_fma(a.s, f.t, a.i);
  const double dd = __builtin_fma(b.s, f.t, b.i);
  const double qd = __builtin_fma(nd, nd, dd * dd);
  return Forms{float(nd), float(dd), float(qd)};
}

// ---------------------------------------------------------------------------
// The evaluation in FP32: always for 16-bit storage (outputs keep 8 or 11
// bits), and, with the reduction residual carried (CARRY, below), for FP32
// storage with TA_FLAG_FORCE_FP32_REDUCTION.
// For |x| < 2^16 (every FP16 value, BF16 below 65536): q = the integer
// nearest x RN(2/pi), by one FMA adding 1.5 2^23 (q is then the low bits of
// that sum, and the sum less 1.5 2^23 is +0 when q = 0), and a three-word
// Cody-Waite r = x - q pi/2 (the first step exact: x and q C1 are multiples
// of 2^-23 there and |r| < 1), relative error ~2^-23.  The three words are
// rounded down, so all are positive and each -q Ci is -0 when q = 0: r then
// keeps the sign of a zero x.  The rounding of 2/pi can put q on the neighbour
// of the nearest quadrant near odd multiples of pi/4, leaving |r| a little
// above pi/4: slot 3 of the table continues both families, so that costs
// nothing.  Larger BF16 values take the FP64 fold.  Then t = |r| 180/pi,
// and N, D (signed) and Q by FP32 FMAs from the signed FP16 row of
// Tables16.  Relative errors (u = 2^-24): r 2u, t 4u, N and D 5u.
// ---------------------------------------------------------------------------
constexpr float kTwoOverPiF = 0x1.45f306p-1f;  // RN24(2/pi)
constexpr float kPio2F1 = 0x1.921fb4p+0f;      // RD24(pi/2)
constexpr float kPio2F2 = 0x1.4442d0p-24f;     // RD24(pi/2 - F1)
constexpr float kPio2F3 = 0x1.84698ap-48f;     // RN24(pi/2 - F1 - F2)
constexpr float kDegPerRadF = 0x1.ca5dc2p+5f;  // RN24(180/pi)
constexpr float kDegPerRadLoF = -0x1.670f82p-21f;  // RN24(180/pi - kDegPerRadF)
constexpr float kSmall16 = 0x1p16f;
// The carried FP32 evaluation (FP32 storage) holds below 2^20: q < 2^20
// keeps x 2/pi + 1.5 2^23 an exact integer rounding, and q times the
// truncation of the three-word pi/2 (below 2^-72) stays under 2^-52, against
// |r| >= 4.19e-9 for every FP32 below 2^20 (x = 252.898209 comes closest).
constexpr float kSmall32 = 0x1p20f;
// 1.5 2^11: (t + kGridT) - kGridT rounds t in [0, 64) degrees to a multiple
// of 2^-12, so that s t + i is exact in FP32 for the table's integers.
constexpr float kGridT = 0x1.8p11f;

struct FoldedL {
  uint32_t q;    // quadrant, low bits
  uint32_t hr;   // bit 31 = sign of r
  uint32_t off;  // byte offset of the Tables16 row (8 row)
  uint32_t row;  // the row, j | sr << 2 | q0 << 3 | q1 << 4
  float ar;      // |r|
  __device__ float abs_r() const { return ar; }
};

// CARRY (FP32 storage, outputs of 24 bits): the reduction keeps its
// rounding error, r = rh + rl, and the degrees t = |r| 180/pi are carried
// as t + tl with t on a 2^-12 grid, so that each linear form is one exact
// FMA (s t + i: a multiple of 2^-12 below 2^12) and one rounding FMA that
// adds s tl.  Steps, for |x| < 2^20:
//   r1 = x - q C1 exactly (x and q C1 are multiples of 2^-22 for |x| >= 2,
//   of 2^-24 for q = +-1 below that, and |r1| < 1); q C2 = ph + pl exactly
//   (one product, one FMA); rh = r1 - ph with its error e by the three-op
//   sum (exact: r1 is a multiple of 2^-22 >= ulp(ph)); rl = e - pl - q C3.
//   t = |rh| 180/pi to 24 bits, then to the grid; tl = the exact remainder
//   of |rh| K_hi, plus |rh| K_lo + |rl| K_hi (K_hi + K_lo = 180/pi).
// Relative errors: r and t below 2^-40, N and D one rounding each (0.5u),
// Q 1u; the outputs stay within about 3.1 ulp of the formula (against
// 2.5 for FP64 forms rounded once).  Lanes with |x| >= 2^20, +-Inf or NaN
// take the FP64 fold (t + tl from the FP64 degrees).
// MAY_BE_LARGE false: the caller's inputs are below 2^16 or not finite (FP16
// storage); +-Inf and NaN then give NaN r, t and forms, and the row (the
// conversion of NaN is 0, the family bit is one bit) stays in the table.
template <bool MAY_BE_LARGE = true, bool CARRY = false>
__device__ inline Forms fold_forms_f32(float x, const Tables16 &tb, FoldedL &f) {
  // The FP32 fold on every lane; lanes at or above the threshold, +-Inf or
  // NaN then overwrite it with the FP64 fold (a rare branch with no else
  // side, so a wave without such lanes only tests and skips it).
  const float qb = __builtin_fmaf(x, kTwoOverPiF, tb.magic);
  const float qf = qb - kRoundMagicF;
  f.q = __float_as_uint(qb);  // 2^22 + q in the mantissa: low bits of q
  float t, tl = 0.0f;
  if constexpr (CARRY) {
    const float r1 = __builtin_fmaf(-qf, kPio2F1, x);
    const float ph = qf * kPio2F2;
    const float pl = __builtin_fmaf(qf, kPio2F2, -ph);
    const float rh = r1 - ph;
    const float rl = __builtin_fmaf(-qf, kPio2F3, ((r1 - rh) - ph) - pl);
    f.hr = __float_as_uint(rh);
    f.ar = __builtin_fabsf(rh);
    // rl with the sign that makes |r| = f.ar + arl
    const float arl = __uint_as_float(__float_as_uint(rl) ^ (f.hr & 0x80000000u));
    const float th = f.ar * kDegPerRadF;
    f.off = row16_offset(uint32_t(th * (1.0f / 15.0f)), f.q, f.hr);
    t = (th + kGridT) - kGridT;
    tl = __builtin_fmaf(f.ar, kDegPerRadF, -t) +
         __builtin_fmaf(f.ar, kDegPerRadLoF, arl * kDegPerRadF);
  } else {
    float r = __builtin_fmaf(-qf, kPio2F1, x);
    r = __builtin_fmaf(-qf, kPio2F2, r);
    r = __builtin_fmaf(-qf, kPio2F3, r);
    f.hr = __float_as_uint(r);
    f.ar = __builtin_fabsf(r);
    t = f.ar * kDegPerRadF;
    f.off = row16_offset(uint32_t(t * (1.0f / 15.0f)), f.q, f.hr);
  }
  constexpr float kSmall = CARRY ? kSmall32 : kSmall16;
  if (MAY_BE_LARGE && __builtin_expect(!(__builtin_fabsf(x) < kSmall), 0)) {
    const Folded g = fold(x);
    f.q = g.q;
    f.hr = g.hr;
    f.off = row16_offset(g.row & 3u, g.q, g.hr);  // slot j: low two bits
    f.ar = float(g.abs_r());
    if constexpr (CARRY) {
      t = (float(g.t) + kGridT) - kGridT;
      tl = float(g.t - double(t));
    } else {
      t = float(g.t);
    }
  }
  f.row = f.off >> 3;
  const CoefH c = *reinterpret_cast<const CoefH *>(
      reinterpret_cast<const char *>(tb.h) + f.off);
  float n, d;  // signed N and D
  if constexpr (CARRY) {
    n = __builtin_fmaf(float(c.sN), tl, __builtin_fmaf(float(c.sN), t, float(c.iN)));
    d = __builtin_fmaf(float(c.sD), tl, __builtin_fmaf(float(c.sD), t, float(c.iD)));
  } else {
    n = __builtin_fmaf(float(c.sN), t, float(c.iN));
    d = __builtin_fmaf(float(c.sD), t, float(c.iD));
  }
  return Forms{n, d, __builtin_fmaf(n, n, d * d)};
}

// ---------------------------------------------------------------------------
// 3. FP32 normalisation
// ---------------------------------------------------------------------------

// 1/sqrt(q): hardware estimate, then one Newton step y + (y/2)(1 - q y^2)
// with 1 - q y^2 formed from the exact square y^2 = p + pe.
__device__ inline float rsqrt_refined(float q) {
  const float y = __builtin_amdgcn_rsqf(q);
  const float p = y * y;
  const float pe = __builtin_fmaf(y, y, -p);
  float e = __builtin_fmaf(-q, p, 1.0f);
  e = __builtin_fmaf(-q, pe, e);
  return __builtin_fmaf(0.5f * y, e, y);
}

// n/d: reciprocal estimate, quotient, exact residual n - d*t0, correction.
// The residual is formed as d t0 - n and subtracted (the same value as
// adding n - d t0), so that n = -0 (a signed table row) gives -0: +0 + -0
// would round to +0.
__device__ inline float div_refined(float n, float d) {
  const float r = __builtin_amdgcn_rcpf(d);
  const float t0 = n * r;
  const float res = __builtin_fmaf(d, t0, -n);
  return __builtin_fmaf(-res, r, t0);
}

// 1/d refined by one Newton step.
__device__ inline float rcp_refined(float d) {
  const float r = __builtin_amdgcn_rcpf(d);
  return __builtin_fmaf(__builtin_fmaf(-d, r, 1.0f), r, r);
}

// Unrefined hardware estimates, for outputs rounded to 16 bits.
__device__ inline float rsqrt_est(float q) { return __builtin_amdgcn_rsqf(q); }
__device__ inline float rcp_est(float d) { return __builtin_amdgcn_rcpf(d); }
__device__ inline float div_est(float n, float d) { return n * rcp_est(d); }

// ---------------------------------------------------------------------------
// Taylor baseline: first `TERMS` Maclaurin terms on the folded angle rho.
// ---------------------------------------------------------------------------
__host__ __device__ constexpr double factorial(int m) {
  double f = 1.0;
  for (int i = 2; i <= m; ++i) f *= double(i);
  return f;
}
// tan^{(2j+1)}(0)/(2j+1)!: 1, 1/3, 2/15, 17/315, 62/2835, 1382/155925,
// 21844/6081075, 929569/638512875, 6404582/10854718875.
__host__ __device__ constexpr double tan_coef(int j) {
  constexpr double num[9] = {1.0, 1.0, 2.0, 17.0, 62.0, 1382.0, 21844.0,
                             929569.0, 6404582.0};
  constexpr double den[9] = {1.0, 3.0, 15.0, 315.0, 2835.0, 155925.0,
                             6081075.0, 638512875.0, 10854718875.0};
  return num[j] / den[j];
}
__host__ __device__ constexpr float sin_coef(int j) {
  return float(((j & 1) ? -1.0 : 1.0) / factorial(2 * j + 1));
}
__host__ __device__ constexpr float cos_coef(int j) {
  return float(((j & 1) ? -1.0 : 1.0) / factorial(2 * j));
}

// rho in FP32 from the fold: a for even q, pi/2 - a for odd q.
__device__ inline float fold_rho(const Folded &f) {
  const double rho = (f.q & 1u) ? (kPio2Hi - f.abs_r()) + kPio2Lo : f.abs_r();
  return float(rho);
}

template <int TERMS>
__device__ inline float taylor_sin_unsigned(float rho) {
  const float z = rho * rho;
  float s = sin_coef(TERMS - 1);
#pragma unroll
  for (int j = TERMS - 2; j >= 0; --j) s = __builtin_fmaf(s, z, sin_coef(j));
  return s * rho;
}
template <int TERMS>
__device__ inline float taylor_cos_unsigned(float rho) {
  const float z = rho * rho;
  float s = cos_coef(TERMS - 1);
#pragma unroll
  for (int j = TERMS - 2; j >= 0; --j) s = __builtin_fmaf(s, z, cos_coef(j));
  return s;
}
template <int TERMS>
__device__ inline float taylor_tan_unsigned(float rho) {
  const float z = rho * rho;
  float s = float(tan_coef(TERMS - 1));
#pragma unroll
  for (int j = TERMS - 2; j >= 0; --j)
    s = __builtin_fmaf(s, z, float(tan_coef(j)));
  return s * rho;
}

// ---------------------------------------------------------------------------
// FP64 storage: the same method with every stage in FP64.
//   Reduction to a double-double r = rh + rl (|r| <= pi/4, relative error
//   below 2^-69 for every finite double): Cody-Waite with a three-word pi/2
//   below 2^29, a 2/pi bit-table reduction above.  t = |r| 180/pi with a
//   two-word constant, N and D by one FMA each, Q = N^2 + D^2, an inverse
//   square root and a reciprocal refined to full FP64 precision.
// ---------------------------------------------------------------------------
constexpr double kPio2Lo2 = -0x1.f1976b7ed8fbcp-110;   // RN(pi/2 - Hi - Lo)
constexpr double kDegPerRadLo = -0x1.1e7ab456405f9p-49;  // RN(180/pi - kDegPerRad)
constexpr double kLargeArg64 = 0x1p29;

// Bits of 2/pi for the FP64 bit-table reduction: word 0 is zero (bits -31
// to 0 of the expansion), word w holds bits 32(w-1)+1 .. 32w.
__constant__ uint32_t kTwoOverPiBits64[40] = {
    0x00000000u, 0xA2F9836Eu, 0x4E441529u, 0xFC2757D1u, 0xF534DDC0u,
    0xDB629599u, 0x3C439041u, 0xFE5163ABu, 0xDEBBC561u, 0xB7246E3Au,
    0x424DD2E0u, 0x06492EEAu, 0x09D1921Cu, 0xFE1DEB1Cu, 0xB129A73Eu,
    0xE88235F5u, 0x2EBB4484u, 0xE99C7026u, 0xB45F7E41u, 0x3991D639u,
    0x835339F4u, 0x9C845F8Bu, 0xBDF9283Bu, 0x1FF897FFu, 0xDE05980Fu,
    0xEF2F118Bu, 0x5A0A6D1Fu, 0x6D367ECFu, 0x27CB09B7u, 0x4F463F66u,
    0x9E5FEA2Du, 0x7527BAC7u, 0xEBE5F17Bu, 0x3D0739F7u, 0x8A5292EAu,
    0x6BFB5FB1u, 0x1F8D5D08u, 0x56033046u, 0xFC7B6BABu, 0xF0CFBC20u};

// Error-free transforms: a + b = s + e exactly (Knuth), and the same for
// |a| >= |b| with three operations (Dekker).
__device__ inline void two_sum(double a, double b, double &s, double &e) {
  s = a + b;
  const double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}
__device__ inline void fast_two_sum(double a, double b, double &s, double &e) {
  s = a + b;
  e = b - (s - a);
}

// |x| >= 2^29 (and +-Inf).  x = m 2^e (m < 2^53, e in [-23, 971]); the 2/pi
// bits from 2^-(e-1) down, a 192-bit window, times m give x 2/pi mod 4: the
// quadrant in the top two bits and a 190-bit fraction, which is rounded to
// nearest (read as a signed number), summed exactly into a double-double
// and multiplied by pi/2.  The window's truncation is below 2^-137 in the
// fraction, far under the smallest |r| of any double (~2^-61).
__device__ inline void reduce_large64(double x, double &rh, double &rl,
                                      uint32_t &q) {
  const uint64_t ux = uint64_t(__double_as_longlong(x));
  const uint32_t ex = uint32_t(ux >> 52) & 0x7ffu;
  if (ex == 0x7ffu) {  // +-Inf (NaN never reaches here)
    rh = rl = __builtin_nan("");
    q = 0;
    return;
  }
  const int e = int(ex) - 1075;
  const uint64_t m = (ux & 0xfffffffffffffull) | (1ull << 52);
  const uint32_t ml = uint32_t(m), mh = uint32_t(m >> 32);
  const int b0 = e + 30;  // (first needed bit, 1-based) + 31 >= 7
  const int w0 = b0 >> 5, sh = b0 & 31;
  uint32_t w[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const uint64_t pair = (uint64_t(kTwoOverPiBits64[w0 + k]) << 32) |
                          kTwoOverPiBits64[w0 + k + 1];
    w[k] = uint32_t(pair >> (32 - sh));
  }
  // P = m * W mod 2^192 (W = w[0] 2^160 + ... + w[5]) as 32-bit limbs p[L]
  // of weight 2^(32 L): limb L gathers lo(ml w[5-L]), hi(ml w[6-L]),
  // lo(mh w[6-L]) and hi(mh w[7-L]).
  uint64_t a[6], b[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    a[k] = uint64_t(ml) * w[k];
    b[k] = uint64_t(mh) * w[k];
  }
  uint32_t p[6];
  uint64_t acc = a[5] & 0xffffffffu;
  p[0] = uint32_t(acc);
#pragma unroll
  for (int L = 1; L < 6; ++L) {
    acc = (acc >> 32) + (a[6 - L] >> 32) + (a[5 - L] & 0xffffffffu) +
          (b[6 - L] & 0xffffffffu);
    if (L >= 2) acc += b[7 - L] >> 32;
    p[L] = uint32_t(acc);
  }
  // quadrant = bits 191..190; fraction = bits 189..0, rounded to nearest:
  // a fraction >= 1/2 becomes (fraction - 1) with the next quadrant.
  const uint32_t neg = (p[5] >> 29) & 1u;
  uint32_t qq = (p[5] >> 30) + neg;
  p[5] &= 0x3fffffffu;
  // |fraction|: two's complement of the 190 bits when negative
  const uint32_t flip = 0u - neg;
  uint64_t carry = neg;
#pragma unroll
  for (int L = 0; L < 6; ++L) {
    const uint64_t v = uint64_t(p[L] ^ flip) + carry;
    p[L] = uint32_t(v);
    carry = v >> 32;
  }
  p[5] &= 0x3fffffffu;
  // |fraction| = sum p[L] 2^(32 L - 190), all terms >= 0: exact two-sums
  double hi = double(p[5]) * 0x1p-30, lo = 0.0;
#pragma unroll
  for (int L = 4; L >= 0; --L) {
    double e2;
    two_sum(hi, double(p[L]) * __builtin_ldexp(1.0, 32 * L - 190), hi, e2);
    lo += e2;
  }
  fast_two_sum(hi, lo, hi, lo);
  // r = fraction * pi/2
  double h = hi * kPio2Hi;
  double l = __builtin_fma(hi, kPio2Hi, -h) + (hi * kPio2Lo + lo * kPio2Hi);
  fast_two_sum(h, l, h, l);
  if (neg) {
    h = -h;
    l = -l;
  }
  if (ux >> 63) {
    h = -h;
    l = -l;
    qq = 0u - qq;
  }
  rh = h;
  rl = l;
  q = qq;
}

// x = q pi/2 + rh + rl for any double x.
// qb = x RN(2/pi) + 1.5 2^52 rounded, q in its low mantissa bits (one FMA
// with the constant from a kernel's LDS table, else a product and an add, as
// for FP32 inputs).  The rounding of 2/pi can make q the neighbour of the
// nearest quadrant next to an odd multiple of pi/4; |r| then exceeds pi/4 by
// at most |x| 2^-54 pi/2 (2^-24 below 2^29), and slot 3 of the table
// continues both quadrant families there, so r needs no correction.
__device__ inline void reduce64_from(double x, double qb, double &rh, double &rl,
                                     uint32_t &q) {
  const double qd = qb - kRoundMagic;
  q = uint32_t(__double2loint(qb));
  const double r1 = __builtin_fma(-qd, kPio2Hi, x);  // exact
  const double p = qd * kPio2Lo;
  const double pe = __builtin_fma(qd, kPio2Lo, -p);  // qd Lo = p + pe
  double s, se;
  two_sum(r1, -p, s, se);
  const double tail = __builtin_fma(-qd, kPio2Lo2, se - pe);
  fast_two_sum(s, tail, rh, rl);
  rh = __builtin_copysign(rh, s);  // keeps the sign of a zero x
  if (__builtin_expect(__builtin_fabs(x) >= kLargeArg64, 0))
    reduce_large64(x, rh, rl, q);
}
__device__ inline void reduce64(double x, double &rh, double &rl, uint32_t &q,
                                double magic) {
  reduce64_from(x, __builtin_fma(x, kTwoOverPi, magic), rh, rl, q);
}
__device__ inline void reduce64(double x, double &rh, double &rl, uint32_t &q) {
  reduce64_from(x, x * kTwoOverPi + kRoundMagic, rh, rl, q);
}

struct Folded64 {
  double rh, rl;  // reduced argument, |rh + rl| <= pi/4
  double t;       // |r| in degrees, [0, 45]
  uint32_t q;     // quadrant, low bits
  uint32_t hr;    // high word of rh: bit 31 = sign of r
  uint32_t row;   // LDS table slot j + 4*(q & 1)
  __device__ double abs_r() const { return __builtin_fabs(rh); }
  // rl with the sign of |r| (rh + rl = sign(rh) (|rh| + abs_rl()))
  __device__ double abs_rl() const { return flip_sign(rl, hr); }
};

__device__ inline Folded64 fold64_finish(Folded64 f) {
  f.hr = uint32_t(__double2hiint(f.rh));
  const double ra = f.abs_r();
  f.t = __builtin_fma(ra, kDegPerRad,
                      __builtin_fma(ra, kDegPerRadLo, f.abs_rl() * kDegPerRad));
  f.row = ((f.q << 2) & 4u) | slot_of(f.t);
  return f;
}
__device__ inline Folded64 fold64(double x, double magic) {
  Folded64 f;
  reduce64(x, f.rh, f.rl, f.q, magic);
  return fold64_finish(f);
}
__device__ inline Folded64 fold64(double x) {
  Folded64 f;
  reduce64(x, f.rh, f.rl, f.q);
  return fold64_finish(f);
}

struct Forms64 {
  double n, d, q;
};
__device__ inline Forms64 forms64(const Folded64 &f, const TablesFwd &tb) {
  const Lin a = tb.n[f.row], b = tb.d[f.row];
  const double nd = __builtin_fma(a.s, f.t, a.i);
  const double dd = __builtin_fma(b.s, f.t, b.i);
  return Forms64{nd, dd, __builtin_fma(nd, nd, dd * dd)};
}

// 1/sqrt(q), q in [10^5, 10^7]: hardware estimate, one Newton step, then a
// second whose residual 1 - q y^2 is formed exactly from y^2 = p + pe.
__device__ inline double rsqrt64_refined(double q) {
  double y = __builtin_amdgcn_rsq(q);
  y = __builtin_fma(0.5 * y, __builtin_fma(-(q * y), y, 1.0), y);
  const double p = y * y;
  const double pe = __builtin_fma(y, y, -p);
  double e = __builtin_fma(-q, p, 1.0);
  e = __builtin_fma(-q, pe, e);
  return __builtin_fma(0.5 * y, e, y);
}
// 1/d: hardware estimate and two Newton steps.
__device__ inline double rcp64_refined(double d) {
  double r = __builtin_amdgcn_rcp(d);
  r = __builtin_fma(__builtin_fma(-d, r, 1.0), r, r);
  return __builtin_fma(__builtin_fma(-d, r, 1.0), r, r);
}
// n/d: quotient from the refined reciprocal, exact residual, correction.
__device__ inline double div64_refined(double n, double d) {
  const double r = rcp64_refined(d);
  const double t0 = n * r;
  return __builtin_fma(__builtin_fma(-d, t0, n), r, t0);
}

// rho in FP64 (a for even q, pi/2 - a for odd q).
__device__ inline double fold_rho64(const Folded64 &f) {
  return (f.q & 1u) ? (kPio2Hi - f.abs_r()) + (kPio2Lo - f.abs_rl())
                    : f.abs_r();
}

// FP64 Taylor baseline: the same terms with FP64 coefficients and Horner.
__host__ __device__ constexpr double sin_coef64(int j) {
  return ((j & 1) ? -1.0 : 1.0) / factorial(2 * j + 1);
}
__host__ __device__ constexpr double cos_coef64(int j) {
  return ((j & 1) ? -1.0 : 1.0) / factorial(2 * j);
}
template <int TERMS>
__device__ inline double taylor_sin_unsigned(double rho) {
  const double z = rho * rho;
  double s = sin_coef64(TERMS - 1);
#pragma unroll
  for (int j = TERMS - 2; j >= 0; --j) s = __builtin_fma(s, z, sin_coef64(j));
  return s * rho;
}
template <int TERMS>
__device__ inline double taylor_cos_unsigned(double rho) {
  const double z = rho * rho;
  double s = cos_coef64(TERMS - 1);
#pragma unroll
  for (int j = TERMS - 2; j >= 0; --j) s = __builtin_fma(s, z, cos_coef64(j));
  return s;
}
template <int TERMS>
__device__ inline double taylor_tan_unsigned(double rho) {
  const double z = rho * rho;
  double s = tan_coef(TERMS - 1);
#pragma unroll
  for (int j = TERMS - 2; j >= 0; --j) s = __builtin_fma(s, z, tan_coef(j));
  return s * rho;
}

// ---------------------------------------------------------------------------
// The paper's literal arithmetic (Section 3, Algorithms 1-4), FP64: radian
// coefficients, piece index floor(rho/divisor), the fast inverse square root
// in place of 1/sqrt and of the division.  Reproduces the error columns of
// Tables 1-3; not the default path.
// ---------------------------------------------------------------------------
constexpr uint64_t kFisrMagic = 0x5fe6eb50c7b537a9ull;  // Algorithm 1
constexpr double kLiteralDivisor = 0.261;  // pseudocode of proposed_sin/tan

// Algorithm 1: magic-constant initial guess, one Newton-Raphson step.
__device__ inline double fisr(double number) {
  const double x2 = number * 0.5;
  const int64_t i = int64_t(kFisrMagic) - (__double_as_longlong(number) >> 1);
  const double y = __longlong_as_double(i);
  return y * (1.5 - ((x2 * y) * y));
}

// Radian coefficients of piece k: a = a_k K, b, c = c_k K, d and the
// quadratic x a^2 + ..: qx = a^2 + c^2, qy = 2(ab + cd), qz = b^2 + d^2
// (Appendix A.4), evaluated in that order.
struct PaperRow {
  double a, b, c, d, qx, qy, qz;
};

// In LDS as four arrays of 16-byte pairs, (a, b), (c, d), (qx, qy),
// (qz, 0), eight rows each: a wave reading different pieces hits distinct
// banks (rows of 64 bytes would put pieces k and k + 2 on the same banks).
struct PaperTables {
  Lin ab[8], cd[8], qxy[8], qz0[8];
  static constexpr bool kUsed = true;
  __device__ static void init(PaperTables &tb) {
    if (threadIdx.x == 0) {
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        PaperRow r;
        r.a = double(kA[k]) * kDegPerRad;
        r.b = double(kB[k]);
        r.c = double(kC[k]) * kDegPerRad;
        r.d = double(kD[k]);
        r.qx = r.a * r.a + r.c * r.c;
        r.qy = 2.0 * (r.a * r.b + r.c * r.d);
        r.qz = r.b * r.b + r.d * r.d;
        tb.ab[k] = Lin{r.a, r.b};
        tb.cd[k] = Lin{r.c, r.d};
        tb.qxy[k] = Lin{r.qx, r.qy};
        tb.qz0[k] = Lin{r.qz, 0.0};
      }
    }
  }
  __device__ PaperRow row(int k) const {
    return PaperRow{ab[k].i, ab[k].s, cd[k].i, cd[k].s, qxy[k].i, qxy[k].s,
                    qz0[k].i};
  }
};

// Algorithms 2-4 at the folded angle `ang` (radians, [0, pi/2]); unsigned.
__device__ inline void paper_eval(double ang, double divisor,
                                  const PaperTables &tb, double &s, double &c,
                                  double &t) {
  int k = int(ang / divisor);
  k = k > 5 ? 5 : k;
  const PaperRow r = tb.row(k);
  const double poly_s = r.a * ang + r.b;             // Algorithm 2: poly
  const double ang2 = ang * ang;                     // Algorithm 2: ang2
  const double inner = r.qx * ang2 + r.qy * ang + r.qz;
  const double inv = fisr(inner);
  s = poly_s * inv;
  const double poly_c = r.c * ang + r.d;             // Algorithm 3
  c = poly_c * inv;
  const double tmp = fisr(poly_c);                   // Algorithm 4
  t = poly_s * (tmp * tmp);
}

}  // namespace ta
