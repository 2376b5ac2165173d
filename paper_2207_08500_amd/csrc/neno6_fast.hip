// Reduced-precision NENO6 path for gfx950: FP32 state and reconstruction,
// classifier layers on MFMA in BF16 or FP16 with FP32 accumulation.
//
// Classifier mapping (weight-stationary, activations never leave the lanes):
// every layer is computed transposed, Y^T[out][evals] = W[out][in] X^T[in][evals],
// with the weights as the MFMA A operand (loaded once per wave into registers
// in a lane order prepared by k_prepare) and 32 evaluations as the B operand
// columns.  The 32x32 accumulator layout leaves lane (j, h) = (l % 32, l / 32)
// holding rows {8b + 4h + r : b, r = 0..3} of column j; the next layer reads
// its K slots from exactly those registers, so the K order of each weight
// matrix is permuted at preparation time instead of moving activations.
//   L1 6(+1 bias slot) -> 64 : 2 x v_mfma_f32_32x32x16 (K = 16: each feature
//                              as its 16-bit value and the rounding remainder)
//   L2 64 -> 32               : 4 x v_mfma_f32_32x32x16  (bias in the C input)
//   L3 32 -> 16               : 2 x v_mfma_f32_16x16x32 (the tile's columns in
//                              two blocks of 16, bias in the C input)
//   L4 16 -> 8, both blocks   : 1 x v_mfma_f32_16x16x32 (block-diagonal)
//   L5 8 -> 4, both tiles     : 1 x v_mfma_f32_16x16x32 (four diagonal blocks),
//                              bias added in FP32
// The inference tables hold the network with every hidden neuron scaled by an
// a-priori bound of its pre-activation, so the clamp of the packed conversion
// to [0, 1] is the ReLU (the training forward uses plain weights, K = 8 in
// L1, L3..L5 on v_mfma_f32_32x32x*, and a packed integer max as the ReLU).
//
// One lane computes one face (projection, split, features, combine).  The
// L1 inputs of the two 32-column tiles of a wave are exchanged between lane
// halves with v_permlane32_swap, the L2 outputs between lane groups with
// v_permlane16_swap.  The last product takes the L4 outputs of both tiles at
// once, and each lane group ends with the logits of the 16 columns its own
// stencils are in: every lane then holds its own stencil's four logits in
// registers 0..3.  Evaluations whose smallest |logit| is below
// the re-check margin are evaluated again inside the same kernel, before the
// combine: in FP32 (mlp_f32_16 on MFMA, or the vector units in the scalar
// kernels), or, as an option for FP16 operands (SPLIT), in two-part FP16
// passes (mlp_split32).
#include <algorithm>

#include "neno6_device.h"
#include "neno6_fast.h"

namespace n6 {

namespace {

typedef uint32_t u32;
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef short s16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
typedef u32 u32x2 __attribute__((ext_vector_type(2)));
typedef u32 u32x4 __attribute__((ext_vector_type(4)));

constexpr int TPB = 256;
constexpr int WPB = TPB / 64;
constexpr int TAB_REGS = 112;
// registers of the inference L3..L5 on v_mfma_f32_16x16x32 (the rows before
// them: L1 / L2 and the training layout of L3..L5 and its biases)
constexpr int R_T3 = 92, R_T4 = 96, R_T5 = 100, R_C3 = 104, R_C4 = 108;
constexpr int TAB_BYTES = TAB_REGS * 64 * 4;
constexpr int PREP_BF16_OFF = 16384;
constexpr int PREP_F16_OFF = PREP_BF16_OFF + TAB_BYTES;
constexpr int PREP_B5_OFF = PREP_F16_OFF + TAB_BYTES;
constexpr int PREP_SCALE_OFF = 81920;  // per-neuron activation scales (FP64)
constexpr int PREP_F4_OFF = 98304;     // FP32 16x16x4 operand table of the re-check (F4_REGS)
constexpr int PREP_LO_OFF = 118784;    // FP16 remainder table of the two-part re-check (LO_REGS)
constexpr size_t PREP_BYTES = 131072;
static_assert(PREP_B5_OFF + 16 <= (int)PREP_BYTES, "prepared block layout");

// ---- packing -----------------------------------------------------------------
template <int PREC> N6_DEV u32 pack2(float a, float b);
template <> N6_DEV u32 pack2<2>(float a, float b) {
  const f32x2 v = {a, b};
  return __builtin_bit_cast(u32, __builtin_convertvector(v, bf16x2));
}
template <> N6_DEV u32 pack2<3>(float a, float b) {
  const f32x2 v = {a, b};
  return __builtin_bit_cast(u32, __builtin_convertvector(v, f16x2));
}
template <int PREC> N6_DEV f32x2 unpack2(u32 v);
template <> N6_DEV f32x2 unpack2<2>(u32 v) {
  return __builtin_convertvector(__builtin_bit_cast(bf16x2, v), f32x2);
}
template <> N6_DEV f32x2 unpack2<3>(u32 v) {
  return __builtin_convertvector(__builtin_bit_cast(f16x2, v), f32x2);
}
N6_DEV u32 relu2(u32 x) {
  const s16x2 z = {0, 0};
  return __builtin_bit_cast(u32, __builtin_elementwise_max(__builtin_bit_cast(s16x2, x), z));
}
template <int PREC> N6_DEV u32 relu_pack(float a, float b) { return relu2(pack2<PREC>(a, b)); }
// Hidden activations of the inference tables: the conversion's clamp to
// [0, 1] is the ReLU, because k_prepare scales every hidden neuron by an
// a-priori bound on its pre-activation (ReLU(s z) = s ReLU(z) for s > 0, and
// the scaled pre-activation never exceeds 1).  One instruction per pair of
// activations instead of a conversion and a packed max.
//   act_block<PREC, NPAIR>(c, first, o): o[p] = pack(c[first + 2p],
//   c[first + 2p + 1]), activations applied.
// FP16: plain code (a conversion followed by a clamp of the packed halves to
// [0, 1], which the compiler folds into the conversion's clamp); the compiler
// then places the MFMA -> VALU hazard waits itself and fills them with
// independent work.  BF16: the compiler does not fold the clamp there, so the
// block is inline asm with the hazard waits as part of it: before the first
// conversion the 8-pass v_mfma_f32_32x32x16 that produced the tile must have
// written it back (NumPasses + 4 = 12 wait states on gfx950), and after the
// last one an MFMA may read the results only two wait states later.  Outputs
// are early-clobber: the block reads its inputs after it has written some
// outputs.
template <int PREC, int NPAIR> struct ActBlock;
template <> struct ActBlock<2, 8> {
  static N6_DEV void run(const f32x16 &c, int first, u32 *o) {
    asm volatile("s_nop 11\n\tv_cvt_pk_bf16_f32 %0, %8, %9 clamp\n\tv_cvt_pk_bf16_f32 %1, %10, %11 clamp\n\tv_cvt_pk_bf16_f32 %2, %12, %13 clamp\n\tv_cvt_pk_bf16_f32 %3, %14, %15 clamp\n\tv_cvt_pk_bf16_f32 %4, %16, %17 clamp\n\tv_cvt_pk_bf16_f32 %5, %18, %19 clamp\n\tv_cvt_pk_bf16_f32 %6, %20, %21 clamp\n\tv_cvt_pk_bf16_f32 %7, %22, %23 clamp\n\ts_nop 1"
                 : "=&v"(o[0]), "=&v"(o[1]), "=&v"(o[2]), "=&v"(o[3]), "=&v"(o[4]), "=&v"(o[5]), "=&v"(o[6]), "=&v"(o[7])
                 : "v"(c[first + 0]), "v"(c[first + 1]), "v"(c[first + 2]), "v"(c[first + 3]), "v"(c[first + 4]), "v"(c[first + 5]), "v"(c[first + 6]), "v"(c[first + 7]), "v"(c[first + 8]), "v"(c[first + 9]), "v"(c[first + 10]), "v"(c[first + 11]), "v"(c[first + 12]), "v"(c[first + 13]), "v"(c[first + 14]), "v"(c[first + 15]));
  }
};
template <int NPAIR> struct ActBlock<3, NPAIR> {
  static N6_DEV void run(const f32x16 &c, int first, u32 *o) {
    const f16x2 z = {0, 0}, one = {1, 1};
#pragma unroll
    for (int p = 0; p < NPAIR; ++p) {
      const f32x2 v = {c[first + 2 * p], c[first + 2 * p + 1]};
      const f16x2 h = __builtin_convertvector(v, f16x2);
      o[p] = __builtin_bit_cast(u32, __builtin_elementwise_min(__builtin_elementwise_max(h, z), one));
    }
  }
};
template <int PREC, int NPAIR>
N6_DEV void act_block(const f32x16 &c, int first, u32 *o) {
  ActBlock<PREC, NPAIR>::run(c, first, o);
}

template <int PREC> N6_DEV f32x16 mma8(u32x2 a, u32x2 b, f32x16 c);
template <> N6_DEV f32x16 mma8<2>(u32x2 a, u32x2 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(__builtin_bit_cast(s16x4, a),
                                                  __builtin_bit_cast(s16x4, b), c, 0, 0, 0);
}
template <> N6_DEV f32x16 mma8<3>(u32x2 a, u32x2 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x8f16(__builtin_bit_cast(f16x4, a),
                                              __builtin_bit_cast(f16x4, b), c, 0, 0, 0);
}
template <int PREC> N6_DEV f32x16 mma16(u32x4 a, u32x4 b, f32x16 c);
template <> N6_DEV f32x16 mma16<2>(u32x4 a, u32x4 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                 __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}
template <> N6_DEV f32x16 mma16<3>(u32x4 a, u32x4 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a),
                                                __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
}

typedef float f32x4 __attribute__((ext_vector_type(4)));
template <int PREC> N6_DEV f32x4 mma4x(u32x4 a, u32x4 b, f32x4 c);
template <> N6_DEV f32x4 mma4x<2>(u32x4 a, u32x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                 __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}
template <> N6_DEV f32x4 mma4x<3>(u32x4 a, u32x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a),
                                                __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
}

// Activations of a 16x16 accumulator tile (four values a lane, two pairs),
// as act_block: FP16 in plain code, BF16 as inline asm with the hazard waits
// (a v_mfma_f32_16x16x32 needs fewer than the 12 wait states waited here).
template <int PREC> N6_DEV void act4(const f32x4 &c, u32 *o);
template <> N6_DEV void act4<3>(const f32x4 &c, u32 *o) {
  const f16x2 z = {0, 0}, one = {1, 1};
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    const f32x2 v = {c[2 * p], c[2 * p + 1]};
    o[p] = __builtin_bit_cast(u32, __builtin_elementwise_min(
                                       __builtin_elementwise_max(__builtin_convertvector(v, f16x2), z), one));
  }
}
template <> N6_DEV void act4<2>(const f32x4 &c, u32 *o) {
  asm volatile("s_nop 11\n\tv_cvt_pk_bf16_f32 %0, %2, %3 clamp\n\tv_cvt_pk_bf16_f32 %1, %4, %5 clamp\n\ts_nop 1"
               : "=&v"(o[0]), "=&v"(o[1])
               : "v"(c[0]), "v"(c[1]), "v"(c[2]), "v"(c[3]));
}

// Swap lanes 16..31 of x with lanes 0..15 of y, and lanes 48..63 of x with
// lanes 32..47 of y.
N6_DEV void swap16(u32 &x, u32 &y) {
  const auto r = __builtin_amdgcn_permlane16_swap(x, y, false, false);
  x = r[0];
  y = r[1];
}

// Swap lanes 32..63 of x with lanes 0..31 of y.
N6_DEV void swap32(u32 &x, u32 &y) {
  const auto r = __builtin_amdgcn_permlane32_swap(x, y, false, false);
  x = r[0];
  y = r[1];
}

// ---- classifier registers ------------------------------------------------------
// Inference: L1 (K = 16, the features in two parts) and L2 on
// v_mfma_f32_32x32x16, L3..L5 on v_mfma_f32_16x16x32 (operands t3, t4, t5,
// biases c3, c4 in the 16x16 accumulator layout).
struct Wts {
  u32x4 a1x[2];  // L1, K = 16: the features' leading and trailing parts
  u32x4 a2[4];
  f32x16 b2;
  u32x4 t3, t4, t5;
  f32x4 c3, c4;
  float b5[4];
};

// Training (BF16): L1 with K = 8 and L2..L5 on v_mfma_f32_32x32x*, the
// layout its backward tables are permuted for.
struct WtsT {
  u32x2 a1[2];
  u32x4 a2[4], a3[2], a4, a5;
  f32x16 b2, b3, b4;
  float b5[4];
};

template <int PREC>
N6_DEV void load_wts(const void *prepared, int lane, Wts &w) {
  const u32 *t = (const u32 *)((const char *)prepared + (PREC == 2 ? PREP_BF16_OFF : PREP_F16_OFF));
#define N6R(r) t[(r)*64 + lane]
#define N6R4(r) u32x4{N6R(r), N6R((r) + 1), N6R((r) + 2), N6R((r) + 3)}
  w.a1x[0] = N6R4(84);
  w.a1x[1] = N6R4(88);
#pragma unroll
  for (int s = 0; s < 4; ++s) w.a2[s] = N6R4(4 + 4 * s);
#pragma unroll
  for (int r = 0; r < 16; ++r) w.b2[r] = __builtin_bit_cast(float, N6R(36 + r));
  w.t3 = N6R4(R_T3);
  w.t4 = N6R4(R_T4);
  w.t5 = N6R4(R_T5);
  w.c3 = __builtin_bit_cast(f32x4, N6R4(R_C3));
  w.c4 = __builtin_bit_cast(f32x4, N6R4(R_C4));
#undef N6R4
#undef N6R
  const float *b5 = (const float *)((const char *)prepared + PREP_B5_OFF);
#pragma unroll
  for (int k = 0; k < 4; ++k) w.b5[k] = b5[k];
}

N6_DEV void load_wts_train(const void *prepared, int lane, WtsT &w) {
  const u32 *t = (const u32 *)((const char *)prepared + PREP_BF16_OFF);
#define N6R(r) t[(r)*64 + lane]
  w.a1[0] = u32x2{N6R(0), N6R(1)};
  w.a1[1] = u32x2{N6R(2), N6R(3)};
#pragma unroll
  for (int s = 0; s < 4; ++s) w.a2[s] = u32x4{N6R(4 + 4 * s), N6R(5 + 4 * s), N6R(6 + 4 * s), N6R(7 + 4 * s)};
#pragma unroll
  for (int s = 0; s < 2; ++s) w.a3[s] = u32x4{N6R(20 + 4 * s), N6R(21 + 4 * s), N6R(22 + 4 * s), N6R(23 + 4 * s)};
  w.a4 = u32x4{N6R(28), N6R(29), N6R(30), N6R(31)};
  w.a5 = u32x4{N6R(32), N6R(33), N6R(34), N6R(35)};
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    w.b2[r] = __builtin_bit_cast(float, N6R(36 + r));
    w.b3[r] = __builtin_bit_cast(float, N6R(52 + r));
    w.b4[r] = __builtin_bit_cast(float, N6R(68 + r));
  }
#undef N6R
  const float *b5 = (const float *)((const char *)prepared + PREP_B5_OFF);
#pragma unroll
  for (int k = 0; k < 4; ++k) w.b5[k] = b5[k];
}

// L1..L4 of one 32-evaluation tile; `bin` is the L1 B operand of lane (j, h)
// (K slots 8h..8h+7 of column j: h = 0 the leading parts of the features and
// the constant 1 of the folded L1 bias, h = 1 their trailing parts).
//
// L3..L4 run on v_mfma_f32_16x16x32 with the tile's columns in two blocks of
// 16 (block A: columns 0..15, block B: 16..31).  Lane group G = l / 16 of a
// 16x16x32 product supplies K slots 8G..8G+7 of column l % 16, and its
// result holds rows 4G..4G+3 of that column.  After L2, lane (j, h) holds the
// packed activations of L2 rows {8b + 4h + r} of column j in h2[0..7]
// (X = h2[0..3]: b = 0, 1; Y = h2[4..7]: b = 2, 3); swapping X of groups 1, 3
// with Y of groups 0, 2 gives every group block A's data in X and block B's
// in Y, in the same K order for both blocks (group G: X or Y of h = G / 2),
// which the L3 operand table follows.  L3 leaves neurons 4G..4G+3 of each
// block in group G; L4 takes both blocks in one product, K slots 8G..8G+3
// from block A and 8G+4..8G+7 from block B, with block A's eight neurons as
// rows 0..7 and block B's as rows 8..15 (block-diagonal weights).  Returns
// the packed L4 activations of group G: rows 4G..4G+3 (G = 0, 1: block A,
// neurons 4G..4G+3; G = 2, 3: block B, neurons 4G-8..4G-5).
template <int PREC>
N6_DEV u32x2 mlp_front(const Wts &w, u32x4 bin) {
  const f32x16 zero = {};
  const f32x16 c1a = mma16<PREC>(w.a1x[0], bin, zero);
  const f32x16 c1b = mma16<PREC>(w.a1x[1], bin, zero);
  u32 h1a[8], h1b[8];
  act_block<PREC, 8>(c1a, 0, h1a);
  act_block<PREC, 8>(c1b, 0, h1b);
  f32x16 c2 = mma16<PREC>(w.a2[0], u32x4{h1a[0], h1a[1], h1a[2], h1a[3]}, w.b2);
  c2 = mma16<PREC>(w.a2[1], u32x4{h1a[4], h1a[5], h1a[6], h1a[7]}, c2);
  c2 = mma16<PREC>(w.a2[2], u32x4{h1b[0], h1b[1], h1b[2], h1b[3]}, c2);
  c2 = mma16<PREC>(w.a2[3], u32x4{h1b[4], h1b[5], h1b[6], h1b[7]}, c2);
  u32 h2[8];
  act_block<PREC, 8>(c2, 0, h2);
#pragma unroll
  for (int q = 0; q < 4; ++q) swap16(h2[q], h2[4 + q]);
  const f32x4 c3a = mma4x<PREC>(w.t3, u32x4{h2[0], h2[1], h2[2], h2[3]}, w.c3);
  const f32x4 c3b = mma4x<PREC>(w.t3, u32x4{h2[4], h2[5], h2[6], h2[7]}, w.c3);
  u32 h3[4];
  act4<PREC>(c3a, h3);
  act4<PREC>(c3b, h3 + 2);
  const f32x4 c4 = mma4x<PREC>(w.t4, u32x4{h3[0], h3[1], h3[2], h3[3]}, w.c4);
  u32 h4[2];
  act4<PREC>(c4, h4);
  return u32x2{h4[0], h4[1]};
}

// mlp_front for both 32-evaluation tiles of a wave, their chains
// interleaved: each phase issues one tile's MFMAs while the other tile's
// conversions of the previous layer run, so a wave has MFMA work queued
// while it waits for results (the scheduling barriers keep the phase order;
// tile 1's L1 products are issued between tile 0's L1 conversions, which
// keeps the live accumulators to three 32x32 tiles).  Used by the 1D pass
// with FP16 operands (3.5 % shorter steps there); with BF16 operands, whose
// conversion blocks carry fixed waits, and in the 2D sweep kernel (two
// waves per SIMD) it measured 1.7 % and 2.8 % slower than two mlp_front
// calls.
template <int PREC>
N6_DEV void mlp_front2(const Wts &w, u32x4 bin0, u32x4 bin1, u32x2 &o0, u32x2 &o1) {
  const f32x16 zero = {};
  const f32x16 a0 = mma16<PREC>(w.a1x[0], bin0, zero);
  const f32x16 b0 = mma16<PREC>(w.a1x[1], bin0, zero);
  __builtin_amdgcn_sched_barrier(0);
  u32 p0[8], q0[8];
  act_block<PREC, 8>(a0, 0, p0);
  const f32x16 a1 = mma16<PREC>(w.a1x[0], bin1, zero);
  act_block<PREC, 8>(b0, 0, q0);
  const f32x16 b1 = mma16<PREC>(w.a1x[1], bin1, zero);
  __builtin_amdgcn_sched_barrier(0);
  f32x16 c20 = mma16<PREC>(w.a2[0], u32x4{p0[0], p0[1], p0[2], p0[3]}, w.b2);
  c20 = mma16<PREC>(w.a2[1], u32x4{p0[4], p0[5], p0[6], p0[7]}, c20);
  c20 = mma16<PREC>(w.a2[2], u32x4{q0[0], q0[1], q0[2], q0[3]}, c20);
  c20 = mma16<PREC>(w.a2[3], u32x4{q0[4], q0[5], q0[6], q0[7]}, c20);
  __builtin_amdgcn_sched_barrier(0);
  u32 p1[8], q1[8];
  act_block<PREC, 8>(a1, 0, p1);
  act_block<PREC, 8>(b1, 0, q1);
  f32x16 c21 = mma16<PREC>(w.a2[0], u32x4{p1[0], p1[1], p1[2], p1[3]}, w.b2);
  c21 = mma16<PREC>(w.a2[1], u32x4{p1[4], p1[5], p1[6], p1[7]}, c21);
  c21 = mma16<PREC>(w.a2[2], u32x4{q1[0], q1[1], q1[2], q1[3]}, c21);
  c21 = mma16<PREC>(w.a2[3], u32x4{q1[4], q1[5], q1[6], q1[7]}, c21);
  __builtin_amdgcn_sched_barrier(0);
  u32 h20[8];
  act_block<PREC, 8>(c20, 0, h20);
#pragma unroll
  for (int q = 0; q < 4; ++q) swap16(h20[q], h20[4 + q]);
  const f32x4 c3a0 = mma4x<PREC>(w.t3, u32x4{h20[0], h20[1], h20[2], h20[3]}, w.c3);
  const f32x4 c3b0 = mma4x<PREC>(w.t3, u32x4{h20[4], h20[5], h20[6], h20[7]}, w.c3);
  __builtin_amdgcn_sched_barrier(0);
  u32 h21[8];
  act_block<PREC, 8>(c21, 0, h21);
#pragma unroll
  for (int q = 0; q < 4; ++q) swap16(h21[q], h21[4 + q]);
  const f32x4 c3a1 = mma4x<PREC>(w.t3, u32x4{h21[0], h21[1], h21[2], h21[3]}, w.c3);
  const f32x4 c3b1 = mma4x<PREC>(w.t3, u32x4{h21[4], h21[5], h21[6], h21[7]}, w.c3);
  __builtin_amdgcn_sched_barrier(0);
  u32 h30[4];
  act4<PREC>(c3a0, h30);
  act4<PREC>(c3b0, h30 + 2);
  const f32x4 c40 = mma4x<PREC>(w.t4, u32x4{h30[0], h30[1], h30[2], h30[3]}, w.c4);
  __builtin_amdgcn_sched_barrier(0);
  u32 h31[4];
  act4<PREC>(c3a1, h31);
  act4<PREC>(c3b1, h31 + 2);
  const f32x4 c41 = mma4x<PREC>(w.t4, u32x4{h31[0], h31[1], h31[2], h31[3]}, w.c4);
  __builtin_amdgcn_sched_barrier(0);
  u32 h40[2], h41[2];
  act4<PREC>(c40, h40);
  act4<PREC>(c41, h41);
  o0 = u32x2{h40[0], h40[1]};
  o1 = u32x2{h41[0], h41[1]};
}

// The six features of one stencil as packed pairs: x[0..2] their values
// rounded to the table precision, x[3..5] what that rounding left (so the
// first layer sees each feature to about twice the precision's bits).
// With `scale` (a power of two) the features times scale.
template <int PREC>
N6_DEV void feature_pack(const float s[6], u32 x[6], float scale = 1.f) {
  float M = 1.f;
#pragma unroll
  for (int j = 0; j < 6; ++j) M = fmaxf(M, fabsf(s[j]));
  const float r = __builtin_amdgcn_rcpf(M) * scale;
#pragma unroll
  for (int p = 0; p < 3; ++p) {
    const float a = s[2 * p] * r, b = s[2 * p + 1] * r;
    x[p] = pack2<PREC>(a, b);
    const f32x2 hi = unpack2<PREC>(x[p]);
    x[3 + p] = pack2<PREC>(a - hi[0], b - hi[1]);
  }
}
template <int PREC> N6_DEV u32 one_zero() { return pack2<PREC>(1.f, 0.f); }

// Kept mask (bits 0..3) and near-cutoff flag (bit 4) from four logits.
N6_DEV u32 mask_near(const float z[4], float margin) {
  u32 m = 0;
  float amin = fabsf(z[0]);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    m |= z[k] > 0.f ? 0u : (1u << k);
    amin = fminf(amin, fabsf(z[k]));
  }
  return m | (amin < margin ? 16u : 0u);
}

// Classifies the stencil held by every lane of the wave (all 64 lanes must
// call it together): tile 0 = the stencils of lanes 0..31, tile 1 = lanes
// 32..63.  Returns the lane's mask | near-flag << 4; with z != 0 also returns
// the lane's four logits.  PAIR: the two tiles' chains interleaved
// (mlp_front2); same results.
template <int PREC, bool PAIR = false>
N6_DEV u32 classify_packed(const Wts &w, const u32 xin[6], float margin, float *z_out) {
  // K slots of the first layer: lanes 0..31 carry the leading parts (slots
  // 0..5) and the bias input 1 (slot 6), lanes 32..63 the trailing parts
  // (slots 8..13).  Tile 0 (faces of lanes 0..31) keeps the leading parts
  // of lanes 0..31 and gets the trailing parts of the same faces from lanes
  // 0..31 moved up; tile 1 the other way round.
  u32 a[3], b[3];
#pragma unroll
  for (int p = 0; p < 3; ++p) {
    a[p] = xin[p];
    b[p] = xin[3 + p];
    swap32(a[p], b[p]);
  }
  const u32 cin = (threadIdx.x & 32) ? 0u : one_zero<PREC>();
  u32x2 h0, h1;
  if constexpr (PAIR) {
    mlp_front2<PREC>(w, u32x4{a[0], a[1], a[2], cin}, u32x4{b[0], b[1], b[2], cin}, h0, h1);
  } else {
    h0 = mlp_front<PREC>(w, u32x4{a[0], a[1], a[2], cin});
    h1 = mlp_front<PREC>(w, u32x4{b[0], b[1], b[2], cin});
  }
  // L5 for the four 16-column blocks at once: K slots 8G..8G+3 from tile 0,
  // 8G+4..8G+7 from tile 1 (each group's L4 rows), output rows 4B..4B+3 the
  // logits of block B = (tile 0 A, tile 0 B, tile 1 A, tile 1 B): lane group G
  // ends with the logits of the block its own stencil is in
  const f32x4 zero = {};
  const f32x4 c = mma4x<PREC>(w.t5, u32x4{h0[0], h0[1], h1[0], h1[1]}, zero);
  float z[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) z[k] = c[k] + w.b5[k];
  if (z_out) {
#pragma unroll
    for (int k = 0; k < 4; ++k) z_out[k] = z[k];
  }
  return mask_near(z, margin);
}

template <int PREC>
N6_DEV u32 classify_wave(const Wts &w, const float s[6], float margin, float *z_out) {
  u32 x[6];
  feature_pack<PREC>(s, x);
  return classify_packed<PREC>(w, x, margin, z_out);
}

N6_DEV const float *uniform_f32(const void *prepared) {
  const uint64_t v = (uint64_t)prepared;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return (const float *)(((uint64_t)hi << 32) | lo);
}

// ---- per-face setup, FP32 -----------------------------------------------------
// Face k of line p of a 1D batch: the line's first cell o and length n.
struct Face1 {
  int p, n, k;
  uint32_t o;
};

N6_DEV Face1 face1(const Line1D &ln, int64_t g) {
  Face1 f;
  f.p = line_of_face(ln, g);
  const int64_t o = ln.offsets[f.p];
  f.o = (uint32_t)o;
  f.n = (int)(ln.offsets[f.p + 1] - o);
  f.k = (int)(g - o - f.p);
  return f;
}

// Roe average of a 1D face; the right eigenvectors R follow from it.
struct Roe1 {
  float ut, ct, Ht, q2;
};

N6_DEV void roe_R1(const Roe1 &w, float R[3][3]) {
#pragma clang fp contract(off)
  R[0][0] = 1.f;             R[0][1] = 1.f;  R[0][2] = 1.f;
  R[1][0] = w.ut - w.ct;     R[1][1] = w.ut; R[1][2] = w.ut + w.ct;
  R[2][0] = __builtin_fmaf(-w.ut, w.ct, w.Ht); R[2][1] = w.q2; R[2][2] = __builtin_fmaf(w.ut, w.ct, w.Ht);
}

// 1D Euler face: split stencils s[2m + sign][6] ('-' mirrored), the face's
// Roe average, and the state qc and pressure pc of the cell to the right of
// the face (cell k of the line; a ghost for the line's last face).
N6_DEV void setup1d(const Line1D &ln, const float *__restrict__ q, const Face1 &fa, float s[6][6],
                    Roe1 &rw, float qc[3], float &pc, bool *flat = nullptr) {
  // No implicit contraction: every fused multiply-add is written out, so the
  // six cells of a stencil go through the same operations (equal cells give
  // bitwise equal stencil values) and a face computed twice gives the same bits.
#pragma clang fp contract(off)
  const int n = fa.n, k = fa.k;
  const float gm = (float)ln.gamma, g1 = gm - 1.f;
  // uniform per-variable bases and 32-bit per-lane offsets (total < 2^29)
  const float *qv0 = q, *qv1 = q + ln.total, *qv2 = q + 2 * ln.total;
  float qs[6][3], lam[6][3], F[6][3];
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    const uint32_t ci = fa.o + (uint32_t)ghost32(k - 3 + j, n, ln.bc);
    qs[j][0] = qv0[ci];
    qs[j][1] = qv1[ci];
    qs[j][2] = qv2[ci];
  }
  float uu[6], pp[6], ir[6];
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    ir[j] = __builtin_amdgcn_rcpf(qs[j][0]);
    uu[j] = qs[j][1] * ir[j];
    pp[j] = g1 * __builtin_fmaf(-0.5f * qs[j][1], uu[j], qs[j][2]);
    const float c = __builtin_amdgcn_sqrtf((gm * pp[j]) * ir[j]);
    lam[j][0] = uu[j] - c;
    lam[j][1] = uu[j];
    lam[j][2] = uu[j] + c;
    F[j][0] = qs[j][1];
    F[j][1] = __builtin_fmaf(qs[j][1], uu[j], pp[j]);
    F[j][2] = (qs[j][2] + pp[j]) * uu[j];
  }
#pragma unroll
  for (int v = 0; v < 3; ++v) qc[v] = qs[3][v];
  pc = pp[3];
  if (flat) {  // six equal cells: every split stencil is constant
    bool f = true;
#pragma unroll
    for (int j = 1; j < 6; ++j) f = f && qs[j][0] == qs[0][0] && qs[j][1] == qs[0][1] && qs[j][2] == qs[0][2];
    *flat = f;
  }
  // Roe average of cells i (j = 2) and i+1 (j = 3)
  const float sL = __builtin_amdgcn_sqrtf(qs[2][0]), sR = __builtin_amdgcn_sqrtf(qs[3][0]);
  const float id = __builtin_amdgcn_rcpf(sL + sR);
  const float ut = __builtin_fmaf(sL, uu[2], sR * uu[3]) * id;
  const float HL = (qs[2][2] + pp[2]) * ir[2], HR = (qs[3][2] + pp[3]) * ir[3];
  const float Ht = __builtin_fmaf(sL, HL, sR * HR) * id;
  const float q2 = (0.5f * ut) * ut;
  const float c2 = g1 * (Ht - q2);
  const float ct = __builtin_amdgcn_sqrtf(c2);
  const float ic = __builtin_amdgcn_rcpf(ct);
  const float b1 = (g1 * ic) * ic;
  const float b2 = b1 * q2;
  const float uc = ut * ic;
  rw = Roe1{ut, ct, Ht, q2};
  // H = L / 2: the split (g +- alpha v) / 2 then needs no final halving
  // (scaling by a power of two is exact, so the values are those of L)
  const float H[3][3] = {{0.25f * (b2 + uc), -0.25f * __builtin_fmaf(b1, ut, ic), 0.25f * b1},
                         {0.5f * (1.f - b2), 0.5f * (b1 * ut), -0.5f * b1},
                         {0.25f * (b2 - uc), -0.25f * __builtin_fmaf(b1, ut, -ic), 0.25f * b1}};
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    float alpha = 0.f;
#pragma unroll
    for (int j = 0; j < 6; ++j) alpha = fmaxf(alpha, fabsf(lam[j][m]));
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      const float v = __builtin_fmaf(H[m][2], qs[j][2], __builtin_fmaf(H[m][1], qs[j][1], H[m][0] * qs[j][0]));
      const float gg = __builtin_fmaf(H[m][2], F[j][2], __builtin_fmaf(H[m][1], F[j][1], H[m][0] * F[j][0]));
      s[2 * m][j] = __builtin_fmaf(alpha, v, gg);
      s[2 * m + 1][5 - j] = __builtin_fmaf(-alpha, v, gg);
    }
  }
}

// Roe state of a 2D face: normal and transverse velocity, sound speed,
// enthalpy and kinetic energy; R follows from it and the sweep direction.
struct Roe2 {
  float nt, st, ct, Ht, q2;
};

// Right eigenvectors of the face in the (rho, rho u, rho v, E) ordering.
N6_DEV void roe_R2(int dir, const Roe2 &w, float R[4][4]) {
  // (rho, rho u_n, rho u_s, E) ordering, permuted into (rho, rho u, rho v, E)
  const float Rn[4][4] = {{1.f, 1.f, 0.f, 1.f},
                          {w.nt - w.ct, w.nt, 0.f, w.nt + w.ct},
                          {w.st, w.st, 1.f, w.st},
                          {__builtin_fmaf(-w.nt, w.ct, w.Ht), w.q2, w.st, __builtin_fmaf(w.nt, w.ct, w.Ht)}};
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    R[0][m] = Rn[0][m];
    R[1][m] = dir == 0 ? Rn[1][m] : Rn[2][m];
    R[2][m] = dir == 0 ? Rn[2][m] : Rn[1][m];
    R[3][m] = Rn[3][m];
  }
}

// 2D Euler face f of sweep dir: s[2m + sign][6] and the face's Roe state.
N6_DEV void setup2d(const Grid2D &gd, int dir, const float *__restrict__ q, int64_t f,
                    float s[8][6], Roe2 &rw) {
#pragma clang fp contract(off)
  const int64_t cells = gd.nx * gd.ny;
  const float gm = (float)gd.gamma, g1 = gm - 1.f;
  // the six cells in the face's own ordering (rho, rho u_n, rho u_s, E): the
  // momentum planes are picked by address, so no register array is indexed
  // by the sweep direction
  float qs[6][4];
  // 32-bit in-grid indices (the C ABI limits a grid to 2^28 cells)
  const int nx = (int)gd.nx, ny = (int)gd.ny, ff = (int)f, c32 = (int)cells;
  const int pl[4] = {0, (dir == 0 ? 1 : 2) * c32, (dir == 0 ? 2 : 1) * c32, 3 * c32};
  if (dir == 0) {
    const int y = ff / (nx + 1), k = ff - y * (nx + 1);
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      const int ci = y * nx + ghost32(k - 3 + j, nx, gd.bc);
#pragma unroll
      for (int r = 0; r < 4; ++r) qs[j][r] = q[pl[r] + ci];
    }
  } else {
    const int k = ff / nx, x = ff - k * nx;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      const int ci = ghost32(k - 3 + j, ny, gd.bc) * nx + x;
#pragma unroll
      for (int r = 0; r < 4; ++r) qs[j][r] = q[pl[r] + ci];
    }
  }
  float un[6], us[6], pp[6], ir[6], lamc[6];
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    ir[j] = __builtin_amdgcn_rcpf(qs[j][0]);
    un[j] = qs[j][1] * ir[j];
    us[j] = qs[j][2] * ir[j];
    pp[j] = g1 * (qs[j][3] - 0.5f * __builtin_fmaf(qs[j][1], un[j], qs[j][2] * us[j]));
    lamc[j] = __builtin_amdgcn_sqrtf((gm * pp[j]) * ir[j]);
  }
  const float sL = __builtin_amdgcn_sqrtf(qs[2][0]), sR = __builtin_amdgcn_sqrtf(qs[3][0]);
  const float id = __builtin_amdgcn_rcpf(sL + sR);
  const float nt = __builtin_fmaf(sL, un[2], sR * un[3]) * id;
  const float st = __builtin_fmaf(sL, us[2], sR * us[3]) * id;
  const float HL = (qs[2][3] + pp[2]) * ir[2], HR = (qs[3][3] + pp[3]) * ir[3];
  const float Ht = __builtin_fmaf(sL, HL, sR * HR) * id;
  const float q2 = 0.5f * __builtin_fmaf(nt, nt, st * st);
  const float c2 = g1 * (Ht - q2);
  const float ct = __builtin_amdgcn_sqrtf(c2);
  const float ic = __builtin_amdgcn_rcpf(ct);
  const float b1 = (g1 * ic) * ic;
  const float b2 = b1 * q2;
  const float nc = nt * ic;
  rw = Roe2{nt, st, ct, Ht, q2};
  const float Ln[4][4] = {{0.5f * (b2 + nc), -0.5f * __builtin_fmaf(b1, nt, ic), (-0.5f * b1) * st, 0.5f * b1},
                          {1.f - b2, b1 * nt, b1 * st, -b1},
                          {-st, 0.f, 1.f, 0.f},
                          {0.5f * (b2 - nc), -0.5f * __builtin_fmaf(b1, nt, -ic), (-0.5f * b1) * st, 0.5f * b1}};
  // normal-direction fluxes of the six cells in the (rho, n, s, E) ordering
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    float alpha = 0.f;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      const float lm = m == 0 ? un[j] - lamc[j] : (m == 3 ? un[j] + lamc[j] : un[j]);
      alpha = fmaxf(alpha, fabsf(lm));
    }
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      const float Fn0 = qs[j][1];
      const float Fn1 = __builtin_fmaf(qs[j][1], un[j], pp[j]);
      const float Fn2 = qs[j][2] * un[j];
      const float Fn3 = (qs[j][3] + pp[j]) * un[j];
      const float v = __builtin_fmaf(Ln[m][3], qs[j][3], __builtin_fmaf(Ln[m][2], qs[j][2],
                      __builtin_fmaf(Ln[m][1], qs[j][1], Ln[m][0] * qs[j][0])));
      const float gg = __builtin_fmaf(Ln[m][3], Fn3, __builtin_fmaf(Ln[m][2], Fn2,
                       __builtin_fmaf(Ln[m][1], Fn1, Ln[m][0] * Fn0)));
      s[2 * m][j] = 0.5f * __builtin_fmaf(alpha, v, gg);
      s[2 * m + 1][5 - j] = 0.5f * __builtin_fmaf(-alpha, v, gg);
    }
  }
}

N6_DEV void setup2d(const Grid2D &gd, int dir, const float *__restrict__ q, int64_t f,
                    float s[8][6], float R[4][4]) {
  Roe2 rw;
  setup2d(gd, dir, q, f, s, rw);
  roe_R2(dir, rw, R);
}

template <int NV>
N6_DEV void back_project(const float R[NV][NV], const float hs[NV], float Fo[NV]) {
#pragma clang fp contract(off)
#pragma unroll
  for (int r = 0; r < NV; ++r) {
    float acc = 0.f;
#pragma unroll
    for (int m = 0; m < NV; ++m) acc = fmaf(R[r][m], hs[m], acc);
    Fo[r] = acc;
  }
}

constexpr int F4_A1 = 0, F4_A2 = 8, F4_A3 = 40, F4_A4 = 48, F4_A5 = 52, F4_B2 = 56, F4_B3 = 64,
              F4_B4 = 68, F4_REGS = 72;
N6_DEV void mlp_f32_16(const float *tab, const float *b5, int lane, const float x[6], float z[4]);
// Remainder table of the two-part FP16 re-check (registers of u32 pairs,
// stored as [register / 4][lane][register % 4]).
constexpr int LO_A1X = 0, LO_A2 = 8, LO_T3 = 24, LO_T4 = 28, LO_S5A = 32, LO_S5B = 36, LO_REGS = 40;
constexpr float SPLIT_SCALE = 256.f;
N6_DEV void mlp_split32(const Wts &w, const u32 *lotab, int lane, u32x4 bin, float z[4]);
// First-layer input of a two-part pass for lane (j, h) from the stencil of
// evaluation j: h = 0 the leading parts and the bias input, h = 1 the
// trailing parts (features and bias input times SPLIT_SCALE).
N6_DEV u32x4 split_input(const float s[6], int lane) {
  u32 xe[6];
  feature_pack<3>(s, xe, SPLIT_SCALE);
  return (lane & 32) ? u32x4{xe[3], xe[4], xe[5], 0u}
                     : u32x4{xe[0], xe[1], xe[2], pack2<3>(SPLIT_SCALE, 0.f)};
}

// ---- fused face kernel, 2D sweeps --------------------------------------------------
// Faces of one 2D sweep.  One lane per face, 64 consecutive faces per wave
// and iteration.  The split stencils and the face's five Roe values wait in
// LDS (a lane-private slot, no barrier) while the classifier runs, so that
// the live registers during the MFMA phase are the weights, the packed
// features and one pair of tiles; R is rebuilt for the back-projection.
// W waves per workgroup; the workgroups loop over the tiles (grid-stride).
// With xcd != 0 the workgroup numbering is permuted so that the workgroups
// the hardware places on one XCD (every 8th) take a contiguous run of tiles
// (the host only sets it when gridDim.x is a multiple of 8).  Two waves per
// SIMD: the kernel holds 212 registers and a four-wave workgroup 78.8 KB of
// LDS (a build trimmed to three waves spilled 47 registers and was 30 %
// slower).  Near-cutoff
// evaluations (a few percent in 2D) are listed per tile in LDS and evaluated
// again before the combine: in FP32 passes of 16 (mlp_f32_16, its table in
// LDS) or, with SPLIT (FP16 operands), in two-part FP16 passes of 32
// (mlp_split32, remainder table in LDS).
template <int PREC, int W, bool MLP, bool SPLIT>
__global__ void __launch_bounds__(W * 64) __attribute__((amdgpu_waves_per_eu(2)))
k_fast_faces(Grid2D gd, int dir, int selector, const void *__restrict__ prepared, float margin,
             const float *__restrict__ q, const uint8_t *__restrict__ min, float *__restrict__ Fh,
             uint8_t *__restrict__ masks, u32 *__restrict__ nrecheck, int xcd) {
  constexpr int NV = 4, NE = 8, NR = 5;
  constexpr int NS = NE * 6 + NR;
  __shared__ float stash[W][NS][64];
  // re-check list (lane << 3 | kind) and the re-checked labels (kind, lane)
  __shared__ uint16_t relist[W][MLP ? NE * 64 : 1];
  __shared__ uint8_t relab[W][MLP ? NE : 1][64];
  // the re-check's operand table (FP32 table, or with SPLIT the remainder
  // table), staged once per workgroup
  static_assert(!SPLIT || PREC == 3, "two-part re-check with FP16 operands only");
  constexpr int TREGS = SPLIT ? LO_REGS : F4_REGS;
  __shared__ u32 tlds[MLP ? TREGS * 64 : 1];
  __shared__ CombTab ctab;
  comb_fill(ctab);
  const float *b5 = (const float *)((const char *)prepared + PREP_B5_OFF);
  if constexpr (MLP) {
    const u32 *g = (const u32 *)((const char *)prepared + (SPLIT ? PREP_LO_OFF : PREP_F4_OFF));
    for (int i = threadIdx.x; i < TREGS * 64; i += W * 64) tlds[i] = g[i];
    __syncthreads();
  }
  const float *f4tab = (const float *)tlds;
  u32 nre = 0u;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t nf = dir == 0 ? (gd.nx + 1) * gd.ny : gd.nx * (gd.ny + 1);
  const int64_t nchunk = (nf + 63) / 64;
  const int64_t nb = gridDim.x;
  const int64_t lb = xcd ? (int64_t)(blockIdx.x % 8) * (nb / 8) + blockIdx.x / 8 : blockIdx.x;
  Wts w;
  if constexpr (MLP) load_wts<PREC>(prepared, lane, w);
  for (int64_t ch = lb * W + wv; ch < nchunk; ch += nb * W) {
    const int64_t f = ch * 64 + lane;
    const bool valid = f < nf;
    const int64_t fc = valid ? f : nf - 1;
    {
      float s[NE][6];
      Roe2 rw;
      setup2d(gd, dir, q, fc, s, rw);
      const float R[NR] = {rw.nt, rw.st, rw.ct, rw.Ht, rw.q2};
#pragma unroll
      for (int e = 0; e < NE; ++e)
#pragma unroll
        for (int j = 0; j < 6; ++j) stash[wv][e * 6 + j][lane] = s[e][j];
#pragma unroll
      for (int a = 0; a < NR; ++a) stash[wv][NE * 6 + a][lane] = R[a];
    }
    u32 sel[NE], near = 0u;
    // the classifier phase at raised wave priority: its MFMA -> convert
    // chains are issued as soon as they are ready, and the other waves'
    // set-up and combine work fills the gaps
    if constexpr (MLP) __builtin_amdgcn_s_setprio(1);
    // each evaluation's features are formed from its stashed stencil right
    // before it is classified; the next stencil is read meanwhile
    float sn[6];
    if constexpr (MLP) {
#pragma unroll
      for (int j = 0; j < 6; ++j) sn[j] = stash[wv][j][lane];
    }
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      if constexpr (MLP) {
        u32 xe[6];
        feature_pack<PREC>(sn, xe);
        if (e + 1 < NE) {
#pragma unroll
          for (int j = 0; j < 6; ++j) sn[j] = stash[wv][(e + 1) * 6 + j][lane];
        }
        const u32 mk = classify_packed<PREC>(w, xe, margin, nullptr);
        sel[e] = mk & 15u;
        near |= (mk >> 4) << e;
      } else if (selector == 1) {
        sel[e] = 15u;
      } else if (selector == 2) {
        sel[e] = 0u;
      } else if (selector == 4) {  // TENO6-opt, decided in FP64
        float se[6];
#pragma unroll
        for (int j = 0; j < 6; ++j) se[j] = stash[wv][e * 6 + j][lane];
        sel[e] = teno_mask_of<float>(se);
      } else {
        sel[e] = (min[(e >> 1) * nf + fc] >> ((e & 1) * 4)) & 15u;
      }
    }
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (MLP) {
      __builtin_amdgcn_s_setprio(0);
      // near-cutoff evaluations of the tile, evaluated again (FP32 in passes
      // of 16, or two-part FP16 in passes of 32); their labels replace the
      // reduced-precision ones
      const u32 want = valid ? near : 0u;
      if (__ballot(want != 0u) != 0ull) {  // wave-uniform
        const u32 c = (u32)__popc(want);
        u32 inc = c;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
          const u32 tt = __shfl_up(inc, o);
          inc += lane >= o ? tt : 0u;
        }
        const int nnear = (int)__shfl(inc, 63);
        u32 pos = inc - c, m = want;
        while (m) {
          relist[wv][pos++] = (uint16_t)(((u32)lane << 3) | (u32)(__ffs(m) - 1));
          m &= m - 1u;
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        if constexpr (SPLIT) {
          const int jcol = lane & 31;
          for (int b0 = 0; b0 < nnear; b0 += 32) {
            const int i = b0 + jcol;
            const bool ok = i < nnear;
            const u32 ent = relist[wv][ok ? i : b0];
            const int src = (int)(ent >> 3), e = (int)(ent & 7u);
            float se[6], z[4];
#pragma unroll
            for (int j = 0; j < 6; ++j) se[j] = stash[wv][e * 6 + j][src];
            mlp_split32(w, tlds, lane, split_input(se, lane), z);
            if (lane < 32 && ok) relab[wv][e][src] = (uint8_t)mask_from_logits<float>(z);
          }
        } else {
          const int jcol = lane & 15;
          for (int b0 = 0; b0 < nnear; b0 += 16) {
            const int i = b0 + jcol;
            const bool ok = i < nnear;
            const u32 ent = relist[wv][ok ? i : b0];
            const int src = (int)(ent >> 3), e = (int)(ent & 7u);
            float se[6], x[6], z[4];
#pragma unroll
            for (int j = 0; j < 6; ++j) se[j] = stash[wv][e * 6 + j][src];
            features<float>(se, x);
            mlp_f32_16(f4tab, b5, lane, x, z);
            if (lane < 16 && ok) relab[wv][e][src] = (uint8_t)mask_from_logits<float>(z);
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll
        for (int e = 0; e < NE; ++e)
          if ((want >> e) & 1u) sel[e] = relab[wv][e][lane];
        nre += (u32)nnear;
      }
    }
    float hs[NV], Fo[NV], R[NV][NV];
#pragma unroll
    for (int m = 0; m < NV; ++m) {
      float sp[6], sm[6];
#pragma unroll
      for (int j = 0; j < 6; ++j) {
        sp[j] = stash[wv][(2 * m) * 6 + j][lane];
        sm[j] = stash[wv][(2 * m + 1) * 6 + j][lane];
      }
      hs[m] = comb_pair_tab(ctab, sp, sel[2 * m], sm, sel[2 * m + 1]);
    }
    const Roe2 rw{stash[wv][NE * 6][lane], stash[wv][NE * 6 + 1][lane], stash[wv][NE * 6 + 2][lane],
                  stash[wv][NE * 6 + 3][lane], stash[wv][NE * 6 + 4][lane]};
    roe_R2(dir, rw, R);
    back_project<NV>(R, hs, Fo);
    if (valid) {
#pragma unroll
      for (int r = 0; r < NV; ++r) Fh[r * nf + f] = Fo[r];
#pragma unroll
      for (int m = 0; m < NV; ++m) masks[m * nf + f] = (uint8_t)(sel[2 * m] | (sel[2 * m + 1] << 4));
    }
  }
  // diagnostic count of re-checked evaluations, spread over eight counters
  if (MLP && nrecheck && lane == 0 && nre) atomicAdd(nrecheck + ((blockIdx.x * W + wv) & 7), nre);
}

// ---- FP32 re-check in 16-evaluation passes ------------------------------------------
// The classifier in FP32 on v_mfma_f32_16x16x4_f32 for up to 16 evaluations,
// in the same transposed, weight-stationary tiling: lane l = (j, k) with
// j = l % 16 (evaluation) and k = l / 16 provides K slot k of each step, and
// the 16x16 accumulator leaves rows 4k + r (r = 0..3) of column j in lane
// l's register r, which is exactly K slot k of step r of the next layer, so
// the activations stay in the lanes.  Operand table (k_prepare,
// register-major, one FP32 value per lane and register):
//   A1 [8]   L1: output tile T (rows 16T..16T+15) x step s: slot 4s + k
//            (slots 0..5 features, 6 the folded bias, 7 zero)
//   A2 [32]  L2: output tile T2 x input tile T1 x register r
//   A3 [8]   L3: input tile T2 x register r;  A4 [4], A5 [4]: register r
//            (L4 outputs padded to 16 rows, L5 to 16 rows and 16 inputs)
//   B2 [8], B3 [4], B4 [4]: biases of L2..L4 in the accumulator layout
// b5 is added to the logits (rows 0..3: registers 0..3 of lanes 0..15).
static_assert(PREP_F4_OFF + F4_REGS * 64 * 4 <= PREP_LO_OFF &&
                  PREP_LO_OFF + LO_REGS * 64 * 4 <= (int)PREP_BYTES,
              "prepared block layout");

N6_DEV float f4_table_value(const double *__restrict__ P, int reg, int lane) {
  const int i = lane % 16, k = lane / 16;
  double x = 0.0;
  if (reg < F4_A2) {
    const int T = reg / 2, slot = 4 * (reg % 2) + k, o = 16 * T + i;
    x = slot < 6 ? P[OW1 + o * 6 + slot] : (slot == 6 ? P[OB1 + o] : 0.0);
  } else if (reg < F4_A3) {
    const int u = reg - F4_A2, T2 = u / 16, T1 = (u % 16) / 4, r = u % 4;
    x = P[OW2 + (16 * T2 + i) * 64 + 16 * T1 + 4 * k + r];
  } else if (reg < F4_A4) {
    const int u = reg - F4_A3, T2 = u / 4, r = u % 4;
    x = P[OW3 + i * 32 + 16 * T2 + 4 * k + r];
  } else if (reg < F4_A5) {
    const int in = 4 * k + (reg - F4_A4);
    x = i < 8 ? P[OW4 + i * 16 + in] : 0.0;
  } else if (reg < F4_B2) {
    const int in = 4 * k + (reg - F4_A5);
    x = (i < 4 && in < 8) ? P[OW5 + i * 8 + in] : 0.0;
  } else if (reg < F4_B3) {
    const int u = reg - F4_B2;
    x = P[OB2 + 16 * (u / 4) + 4 * k + u % 4];
  } else if (reg < F4_B4) {
    x = P[OB3 + 4 * k + (reg - F4_B3)];
  } else {
    const int row = 4 * k + (reg - F4_B4);
    x = row < 8 ? P[OB4 + row] : 0.0;
  }
  return (float)x;
}

N6_DEV f32x4 mma4(float a, float b, f32x4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
N6_DEV f32x4 relu4(f32x4 c) {
#pragma unroll
  for (int r = 0; r < 4; ++r) c[r] = fmaxf(c[r], 0.f);
  return c;
}

// Zero, hidden from the optimiser: loads at an address offset by it are
// neither hoisted out of a loop nor merged with earlier loads of the same
// address.
N6_DEV int opaque_zero() {
  int z = 0;
  asm volatile("" : "+s"(z));
  return z;
}

// FP32 logits of the 16 evaluations of a pass: lane (j, k) holds the features
// x of evaluation j; lanes 0..15 return its four logits.  tab: the operand
// table; b5: the output biases.
N6_DEV void mlp_f32_16(const float *tab, const float *b5, int lane, const float x[6], float z[4]) {
  // Each block of operands (L1; each half of L2; L3; L4 with L5) is read
  // through a freshly hidden offset, all its loads issued before its first
  // MFMA (the barrier keeps them together): one memory round trip per block,
  // and the loads are neither hoisted out of the tile loop (72 registers)
  // nor issued all at the start of the pass.
  const int k = lane >> 4;
  const f32x4 zero = {};
  const float *t = tab + opaque_zero() + lane;
  float a1[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) a1[i] = t[(F4_A1 + i) * 64];
  __builtin_amdgcn_sched_barrier(0);
  f32x4 c1[4] = {zero, zero, zero, zero};
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int slot = 4 * s + k;
    float b = 0.f;
#pragma unroll
    for (int q = 0; q < 6; ++q) b = slot == q ? x[q] : b;
    b = slot == 6 ? 1.f : b;
#pragma unroll
    for (int T = 0; T < 4; ++T) c1[T] = mma4(a1[2 * T + s], b, c1[T]);
  }
#pragma unroll
  for (int T = 0; T < 4; ++T) c1[T] = relu4(c1[T]);
  f32x4 c2[2];
#pragma unroll
  for (int T2 = 0; T2 < 2; ++T2) {
    t = tab + opaque_zero() + lane;
    float a2[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) a2[i] = t[(F4_A2 + 16 * T2 + i) * 64];
#pragma unroll
    for (int r = 0; r < 4; ++r) c2[T2][r] = t[(F4_B2 + 4 * T2 + r) * 64];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int T1 = 0; T1 < 4; ++T1)
#pragma unroll
      for (int r = 0; r < 4; ++r) c2[T2] = mma4(a2[4 * T1 + r], c1[T1][r], c2[T2]);
    c2[T2] = relu4(c2[T2]);
  }
  t = tab + opaque_zero() + lane;
  float a3[8];
  f32x4 c3;
#pragma unroll
  for (int i = 0; i < 8; ++i) a3[i] = t[(F4_A3 + i) * 64];
#pragma unroll
  for (int r = 0; r < 4; ++r) c3[r] = t[(F4_B3 + r) * 64];
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int T2 = 0; T2 < 2; ++T2)
#pragma unroll
    for (int r = 0; r < 4; ++r) c3 = mma4(a3[4 * T2 + r], c2[T2][r], c3);
  c3 = relu4(c3);
  t = tab + opaque_zero() + lane;
  float a4[4], a5[4];
  f32x4 c4;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    a4[r] = t[(F4_A4 + r) * 64];
    a5[r] = t[(F4_A5 + r) * 64];
    c4[r] = t[(F4_B4 + r) * 64];
  }
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int r = 0; r < 4; ++r) c4 = mma4(a4[r], c3[r], c4);
  c4 = relu4(c4);
  f32x4 c5 = zero;
#pragma unroll
  for (int r = 0; r < 4; ++r) c5 = mma4(a5[r], c4[r], c5);
#pragma unroll
  for (int r = 0; r < 4; ++r) z[r] = c5[r] + b5[r];
}

// ---- two-part FP16 re-check in 32-evaluation passes (option, FP16 operands) ----------
// Every operand in two FP16 parts, FP32 accumulation: weights as their FP16
// value (the registers of the FP16 classifier) plus the FP16 rounding of what
// that leaves (the remainder table), activations likewise, carried times
// SPLIT_SCALE = 2^8 (features, the bias input and the biases of L2..L4 too;
// the logits are scaled back): most scaled hidden activations are below 2^-3,
// whose FP16 remainders would otherwise fall among the subnormals and lose
// bits (the logit error is then about three times larger).  Each product
// W a = W_hi a_hi + W_hi a_lo + W_lo a_hi drops only W_lo a_lo, so an operand
// carries about 21 significant bits (FP32: 24) and the three terms are three
// K steps of the FP16 MFMA on one accumulator: 27 instructions of
// v_mfma_f32_32x32x16_f16 (32 cycles each) per 32 evaluations, against 56 of
// v_mfma_f32_16x16x4_f32 (32 cycles each) per 16 in FP32.
//
// Split of an accumulator tile into packed leading and trailing parts:
// ReLU, the FP16 rounding of the activation and the FP16 rounding of what is
// left (hi[p], lo[p] from elements f + 2p, f + 2p + 1).
template <int NPAIR>
N6_DEV void split_tile(const f32x16 &c, int f, u32 *hi, u32 *lo) {
#pragma unroll
  for (int p = 0; p < NPAIR; ++p) {
    const float a = fmaxf(c[f + 2 * p], 0.f), b = fmaxf(c[f + 2 * p + 1], 0.f);
    hi[p] = pack2<3>(a, b);
    const f32x2 h = unpack2<3>(hi[p]);
    lo[p] = pack2<3>(a - h[0], b - h[1]);
  }
}
N6_DEV void split_quad(const f32x4 &c, u32 *hi, u32 *lo) {
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    const float a = fmaxf(c[2 * p], 0.f), b = fmaxf(c[2 * p + 1], 0.f);
    hi[p] = pack2<3>(a, b);
    const f32x2 h = unpack2<3>(hi[p]);
    lo[p] = pack2<3>(a - h[0], b - h[1]);
  }
}

// Logits of the 32 evaluations of a pass: lane (j, h) holds K slots 8h..8h+7
// of evaluation j's first-layer input (h = 0: leading parts of the features
// and the bias input 1; h = 1: their trailing parts), as in the FP16
// classifier; every lane returns the four logits of evaluation j.  lotab: the
// remainder table (in LDS or through the caches).
N6_DEV void mlp_split32(const Wts &w, const u32 *lotab, int lane, u32x4 bin, float z[4]) {
  // the scale hidden from the optimiser: the scaled biases are formed in the
  // pass, not hoisted out of the caller's tile loop (28 registers)
  float S = SPLIT_SCALE;
  asm volatile("" : "+v"(S));
  // table loads through a hidden offset: issued in the pass, not hoisted
  const u32x4 *lt = (const u32x4 *)lotab + (lane + opaque_zero());
  const f32x16 zero = {};
  f32x16 c1a = mma16<3>(w.a1x[0], bin, zero);
  f32x16 c1b = mma16<3>(w.a1x[1], bin, zero);
  c1a = mma16<3>(lt[(LO_A1X / 4) * 64], bin, c1a);
  c1b = mma16<3>(lt[(LO_A1X / 4 + 1) * 64], bin, c1b);
  u32 h1[16], l1[16];
  split_tile<8>(c1a, 0, h1, l1);
  split_tile<8>(c1b, 0, h1 + 8, l1 + 8);
  f32x16 c2 = w.b2 * S;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const u32x4 H = {h1[4 * s], h1[4 * s + 1], h1[4 * s + 2], h1[4 * s + 3]};
    const u32x4 L = {l1[4 * s], l1[4 * s + 1], l1[4 * s + 2], l1[4 * s + 3]};
    c2 = mma16<3>(w.a2[s], H, c2);
    c2 = mma16<3>(w.a2[s], L, c2);
    c2 = mma16<3>(lt[(LO_A2 / 4 + s) * 64], H, c2);
  }
  u32 h2[8], l2[8];
  split_tile<8>(c2, 0, h2, l2);
  // L3..L5 on 16x16x32 as in mlp_front, each product in three parts
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    swap16(h2[q], h2[4 + q]);
    swap16(l2[q], l2[4 + q]);
  }
  const u32x4 t3lo = lt[(LO_T3 / 4) * 64], t4lo = lt[(LO_T4 / 4) * 64];
  f32x4 c3[2];
  u32 h3[4], l3[4];
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    const u32x4 H = {h2[4 * b], h2[4 * b + 1], h2[4 * b + 2], h2[4 * b + 3]};
    const u32x4 L = {l2[4 * b], l2[4 * b + 1], l2[4 * b + 2], l2[4 * b + 3]};
    c3[b] = w.c3 * S;
    c3[b] = mma4x<3>(w.t3, H, c3[b]);
    c3[b] = mma4x<3>(w.t3, L, c3[b]);
    c3[b] = mma4x<3>(t3lo, H, c3[b]);
    split_quad(c3[b], h3 + 2 * b, l3 + 2 * b);
  }
  f32x4 c4 = w.c4 * S;
  {
    const u32x4 H = {h3[0], h3[1], h3[2], h3[3]}, L = {l3[0], l3[1], l3[2], l3[3]};
    c4 = mma4x<3>(w.t4, H, c4);
    c4 = mma4x<3>(w.t4, L, c4);
    c4 = mma4x<3>(t4lo, H, c4);
  }
  u32 h4[2], l4[2];
  split_quad(c4, h4, l4);
  const u32x4 B5 = {h4[0], h4[1], l4[0], l4[1]};
  const f32x4 zero4 = {};
  f32x4 c5 = mma4x<3>(lt[(LO_S5A / 4) * 64], B5, zero4);
  c5 = mma4x<3>(lt[(LO_S5B / 4) * 64], B5, c5);
#pragma unroll
  for (int k = 0; k < 4; ++k) z[k] = c5[k] * (1.f / SPLIT_SCALE) + w.b5[k];
}

// ---- 1D Euler: one fused pass per right-hand side -------------------------------------
// Tiles of 64 consecutive faces g = 63 t + lane of the batch, one wave each,
// overlapping by one face (lane 63's face is lane 0 of the next tile).  Lane
// l < 63 owns the cell between its face and the next when both are faces of
// one line, so a tile holds every flux its cells need and no data moves
// between waves; lane 63 only completes lane 62's cell.  Faces (their
// fluxes in OUT_FACES mode, their labels) are written by lanes 0..62, and by
// lane 63 in the last tile.  A face computed by two tiles gets the same bits
// in both: its arithmetic does not depend on the lane it runs in.
//
// Near-cutoff evaluations (smallest |logit| below the margin) are evaluated
// again before the combine, in the tile itself: they are listed in LDS, form
// their features from the stash in passes of 16 (FP32 MFMA) or, with SPLIT
// (FP16 operands), of 32 (two-part FP16, remainder table read through the
// caches), and the re-check's labels replace the reduced-precision ones.  A few tenths
// of a percent of the evaluations are near, about one per tile.

// Output of cell kc of the line of fa, between fluxes Fl (left face) and Fr.
// What cell_out needs from memory besides the fluxes: the line's spacing and
// time step, its frozen flag and (RK3 stages 2 and 3) the cell's state at
// the start of the step; loaded by the lanes that own a cell, early, so that
// the loads' latency overlaps the combine.
struct CellIn {
  float dx = 1.f, dt = 0.f, u0[3] = {0.f, 0.f, 0.f};
  bool frozen = false;
};
N6_DEV CellIn cell_in(const Line1D &ln, const Out1D &out, const Face1 &fa, int kc) {
  CellIn ci;
  if (out.mode == OUT_FACES) return ci;
  const int64_t c = (int64_t)fa.o + kc;
  ci.dx = (float)ln.dx[fa.p];
  if (out.mode == OUT_RHS) return ci;
  ci.frozen = out.frozen[fa.p] != 0;
  ci.dt = (float)out.dt[fa.p];
  if (out.stage != 1) {
#pragma unroll
    for (int v = 0; v < 3; ++v) ci.u0[v] = out.u0[v * ln.total + c];
  }
  return ci;
}

N6_DEV void cell_out(const Line1D &ln, const Out1D &out, const Face1 &fa, int kc, const CellIn &ci,
                     const float qc[3], float pc, const float Fl[3], const float Fr[3]) {
#pragma clang fp contract(off)
  if (out.mode == OUT_FACES) return;
  const int64_t c = (int64_t)fa.o + kc;
  if (out.mode == OUT_RHS) {
#pragma unroll
    for (int v = 0; v < 3; ++v) out.dst[v * ln.total + c] = (Fl[v] - Fr[v]) / ci.dx;
    if (out.status && !physical<float>(qc[0], pc)) out.status[fa.p] = ST_NONPHYSICAL;
    return;
  }
#pragma unroll
  for (int v = 0; v < 3; ++v) {
    const float L = (Fl[v] - Fr[v]) / ci.dx;
    const float u0 = out.stage == 1 ? qc[v] : ci.u0[v];
    out.dst[v * ln.total + c] = ci.frozen ? u0 : rk3<float>(out.stage, qc[v], u0, L, ci.dt);
  }
}

// Counters of re-checked evaluations (diagnostic): a wave adds its count to
// slot (workgroup * waves + wave) % NRECHECK_SLOTS, so few waves share one.
constexpr int NRECHECK_SLOTS = QCOUNTERS;

// The fused 1D Euler pass.  Three waves per SIMD (168 registers; one value
// used only after the tile loop waits in scratch; the third wave hides more
// of the MFMA -> convert -> MFMA latency).  With FP16 operands the two
// tiles' classifier chains are interleaved (mlp_front2).  The
// cell's line data and the stage's u0 are loaded before the combine, so their
// latency overlaps it.
//
// Flat faces (six equal cells): every split stencil is constant, and the
// re-normalised combination of a constant stencil is that constant for every
// selection (the weights sum to one); the difference form of the combine
// gives it exactly (h = s_2), so the flux does not depend on the labels.  Near-cutoff
// evaluations of flat faces are then re-checked only when the caller asks
// for the labels (out.masks); they are most of the near evaluations of
// piecewise-constant data.
template <int PREC, int W, bool MLP, bool SPLIT>
__global__ void __launch_bounds__(W * 64) __attribute__((amdgpu_waves_per_eu(3)))
k_euler1d(Line1D ln, int selector, const void *__restrict__ prepared, float margin,
          const float *__restrict__ q, const uint8_t *__restrict__ min, Out1D out, int xcd) {
  // stash slots per lane: the six split stencils, the Roe average, the
  // state and pressure of the cell to the right, the line and the flat flag
  constexpr int NE = 6, S_ROE = NE * 6, S_QC = S_ROE + 4, S_LINE = S_QC + 4, NS = S_LINE + 1;
  __shared__ float stash[W][NS][64];
  // re-check list (lane << 3 | kind) and the re-checked labels (kind, lane)
  __shared__ uint16_t relist[W][MLP ? NE * 64 : 1];
  __shared__ uint8_t relab[W][MLP ? NE : 1][64];
  __shared__ CombTab ctab;
  comb_fill(ctab);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t nf = ln.faces();
  const int64_t ntile = (nf + 61) / 63;  // faces 63 t .. 63 t + 63 cover 0 .. nf - 1
  const int64_t nb = gridDim.x;
  const int64_t lb = xcd ? (int64_t)(blockIdx.x % 8) * (nb / 8) + blockIdx.x / 8 : blockIdx.x;
  Wts w;
  const float *b5 = (const float *)((const char *)prepared + PREP_B5_OFF);
  const float *f4tab = (const float *)((const char *)prepared + PREP_F4_OFF);
  const bool need_labels = out.masks != nullptr;
  if constexpr (MLP) load_wts<PREC>(prepared, lane, w);
  u32 nre = 0u;  // evaluations this wave re-checked
  for (int64_t t = lb * W + wv; t < ntile; t += nb * W) {
    const int64_t g = t * 63 + lane;
    const bool valid = g < nf;
    {
      // the face's line and geometry wait in LDS with the stencils: nothing
      // but the classifier's operands holds registers through the MFMA phase
      const Face1 fa = face1(ln, valid ? g : nf - 1);
      float s[NE][6], qc[3], pc;
      Roe1 rw;
      bool flat;
      setup1d(ln, q, fa, s, rw, qc, pc, &flat);
#pragma unroll
      for (int e = 0; e < NE; ++e)
#pragma unroll
        for (int j = 0; j < 6; ++j) stash[wv][e * 6 + j][lane] = s[e][j];
      stash[wv][S_ROE][lane] = rw.ut;
      stash[wv][S_ROE + 1][lane] = rw.ct;
      stash[wv][S_ROE + 2][lane] = rw.Ht;
      stash[wv][S_ROE + 3][lane] = rw.q2;
#pragma unroll
      for (int v = 0; v < 3; ++v) stash[wv][S_QC + v][lane] = qc[v];
      stash[wv][S_QC + 3][lane] = pc;
      stash[wv][S_LINE][lane] = __builtin_bit_cast(float, flat ? -1 - fa.p : fa.p);
    }
    u32 sel[NE], near = 0u;
    // the classifier phase at raised wave priority: its MFMA -> convert
    // chains are issued as soon as they are ready, and the other waves'
    // set-up and combine work fills the gaps
    if constexpr (MLP) __builtin_amdgcn_s_setprio(1);
    // each evaluation's features are formed from its stashed stencil right
    // before it is classified; the next stencil is read meanwhile
    float sn[6];
    if constexpr (MLP) {
#pragma unroll
      for (int j = 0; j < 6; ++j) sn[j] = stash[wv][j][lane];
    }
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      if constexpr (MLP) {
        u32 xe[6];
        feature_pack<PREC>(sn, xe);
        if (e + 1 < NE) {
#pragma unroll
          for (int j = 0; j < 6; ++j) sn[j] = stash[wv][(e + 1) * 6 + j][lane];
        }
        const u32 mk = classify_packed<PREC, PREC == 3>(w, xe, margin, nullptr);
        sel[e] = mk & 15u;
        near |= (mk >> 4) << e;
      } else if (selector == 1) {
        sel[e] = 15u;
      } else if (selector == 2) {
        sel[e] = 0u;
      } else if (selector == 4) {  // TENO6-opt, decided in FP64
        float se[6];
#pragma unroll
        for (int j = 0; j < 6; ++j) se[j] = stash[wv][e * 6 + j][lane];
        sel[e] = teno_mask_of<float>(se);
      } else {
        sel[e] = (min[(e >> 1) * nf + (valid ? g : nf - 1)] >> ((e & 1) * 4)) & 15u;
      }
    }
    __builtin_amdgcn_sched_barrier(0);
    const int pl = __builtin_bit_cast(int, stash[wv][S_LINE][lane]);
    const bool flat = pl < 0;
    if constexpr (MLP) {
      __builtin_amdgcn_s_setprio(0);
      near = valid ? near : 0u;
      // labels of flat faces do not change the flux (see above)
      const u32 want = (flat && !need_labels) ? 0u : near;
      if (__ballot(want != 0u) != 0ull) {  // wave-uniform
        // list the evaluations: lane l's entries after those of lanes < l
        const u32 c = (u32)__popc(want);
        u32 inc = c;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
          const u32 tt = __shfl_up(inc, o);
          inc += lane >= o ? tt : 0u;
        }
        const int nnear = (int)__shfl(inc, 63);
        u32 pos = inc - c, m = want;
        while (m) {
          relist[wv][pos++] = (uint16_t)(((u32)lane << 3) | (u32)(__ffs(m) - 1));
          m &= m - 1u;
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        if constexpr (SPLIT) {
          const u32 *lot = (const u32 *)((const char *)prepared + PREP_LO_OFF);
          const int jcol = lane & 31;
          for (int b0 = 0; b0 < nnear; b0 += 32) {
            const int i = b0 + jcol;
            const bool ok = i < nnear;
            const u32 ent = relist[wv][ok ? i : b0];
            const int src = (int)(ent >> 3), e = (int)(ent & 7u);
            float se[6], z[4];
#pragma unroll
            for (int j = 0; j < 6; ++j) se[j] = stash[wv][e * 6 + j][src];
            mlp_split32(w, lot, lane, split_input(se, lane), z);
            if (lane < 32 && ok) relab[wv][e][src] = (uint8_t)mask_from_logits<float>(z);
          }
        } else {
          const int jcol = lane & 15;
          for (int b0 = 0; b0 < nnear; b0 += 16) {
            const int i = b0 + jcol;
            const bool ok = i < nnear;
            const u32 ent = relist[wv][ok ? i : b0];
            const int src = (int)(ent >> 3), e = (int)(ent & 7u);
            float se[6], x[6], z[4];
#pragma unroll
            for (int j = 0; j < 6; ++j) se[j] = stash[wv][e * 6 + j][src];
            features<float>(se, x);
            mlp_f32_16(f4tab, b5, lane, x, z);
            if (lane < 16 && ok) relab[wv][e][src] = (uint8_t)mask_from_logits<float>(z);
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll
        for (int e = 0; e < NE; ++e)
          if ((want >> e) & 1u) sel[e] = relab[wv][e][lane];
        nre += (u32)nnear;
      }
    }
    Face1 fa;
    fa.p = flat ? -1 - pl : pl;
    {
      const int64_t o = ln.offsets[fa.p];
      fa.o = (uint32_t)o;
      fa.n = (int)(ln.offsets[fa.p + 1] - o);
      fa.k = (int)((valid ? g : nf - 1) - o - fa.p);
    }
    const bool own_cell = valid && lane < 63 && fa.k < fa.n;
    CellIn ci;
    if (own_cell) ci = cell_in(ln, out, fa, fa.k);
    float hs[3], F[3], R[3][3];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      float sp[6], sm[6];
#pragma unroll
      for (int j = 0; j < 6; ++j) {
        sp[j] = stash[wv][(2 * m) * 6 + j][lane];
        sm[j] = stash[wv][(2 * m + 1) * 6 + j][lane];
      }
      // a flat face's combine is its constant (the value the combine gives):
      // waves whose faces are all flat skip the combine
      hs[m] = flat ? sp[2] + sm[2] : comb_pair_tab(ctab, sp, sel[2 * m], sm, sel[2 * m + 1]);
    }
    roe_R1(Roe1{stash[wv][S_ROE][lane], stash[wv][S_ROE + 1][lane], stash[wv][S_ROE + 2][lane],
                stash[wv][S_ROE + 3][lane]},
           R);
    back_project<3>(R, hs, F);
    float qc[3];
#pragma unroll
    for (int v = 0; v < 3; ++v) qc[v] = stash[wv][S_QC + v][lane];
    const float pc = stash[wv][S_QC + 3][lane];
    // the next face's flux: every lane takes part in the shuffle (a lane
    // outside a conditional would supply no value)
    float Fr[3];
#pragma unroll
    for (int v = 0; v < 3; ++v) Fr[v] = __shfl_down(F[v], 1);
    const bool own_face = valid && (lane < 63 || t == ntile - 1);
    if (own_cell) cell_out(ln, out, fa, fa.k, ci, qc, pc, F, Fr);
    if (own_face) {
      if (out.mode == OUT_FACES) {
#pragma unroll
        for (int v = 0; v < 3; ++v) out.dst[v * nf + g] = F[v];
      }
      if (out.masks) {
#pragma unroll
        for (int m = 0; m < 3; ++m) out.masks[m * nf + g] = (uint8_t)(sel[2 * m] | (sel[2 * m + 1] << 4));
      }
    }
  }
  if (MLP && out.nrecheck && lane == 0 && nre)
    atomicAdd(out.nrecheck + (blockIdx.x * W + wv) % NRECHECK_SLOTS, nre);
}

// Scalar stencils (reconstruction, advection, classifier on its own): one
// lane per stencil, re-check done in place (these are the small cases).
// mode 0: stencils from f[k..k+5] (sign) ; mode 1: advection lines (ghosts);
// mode 2: raw stencils sten[n][6] -> logits.
// LDS of one wave for the two-part re-check of the scalar kernels.
struct WaveRecheck {
  float s[6][64];   // the wave's stencils
  float z[4][64];   // re-check logits
  uint8_t list[64];
  uint8_t lab[64];
};

// MLP label of the stencil s of every lane of the wave (all 64 lanes call
// it together): the BF16/FP16 classifier, then the re-check of evaluations
// within the margin -- FP32 on the vector units, or with SPLIT two-part FP16
// passes of 32 (lot: the remainder table, in LDS).  With z, the lane's
// logits (the re-check's where it ran).
template <int PREC, bool SPLIT>
N6_DEV u32 mlp_select(const Wts &w, const void *prepared, const u32 *lot, WaveRecheck &L,
                      float margin, const float s[6], bool valid, float *z) {
  float zl[4];
  const u32 mk = classify_wave<PREC>(w, s, margin, zl);
  const bool near = valid && (mk & 16u);
  u32 sel = mk & 15u;
  if constexpr (SPLIT) {
    const uint64_t bal = __ballot(near);
    if (bal != 0ull) {  // wave-uniform
      const int lane = threadIdx.x & 63;
#pragma unroll
      for (int j = 0; j < 6; ++j) L.s[j][lane] = s[j];
      const int nnear = __popcll(bal);
      if (near) L.list[__builtin_amdgcn_mbcnt_hi((u32)(bal >> 32), __builtin_amdgcn_mbcnt_lo((u32)bal, 0u))] = (uint8_t)lane;
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      for (int b0 = 0; b0 < nnear; b0 += 32) {
        const int i = b0 + (lane & 31);
        const bool ok = i < nnear;
        const int src = L.list[ok ? i : b0];
        float se[6], zz[4];
#pragma unroll
        for (int j = 0; j < 6; ++j) se[j] = L.s[j][src];
        mlp_split32(w, lot, lane, split_input(se, lane), zz);
        if (lane < 32 && ok) {
          L.lab[src] = (uint8_t)mask_from_logits<float>(zz);
#pragma unroll
          for (int k = 0; k < 4; ++k) L.z[k][src] = zz[k];
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      if (near) {
        sel = L.lab[lane];
#pragma unroll
        for (int k = 0; k < 4; ++k) zl[k] = L.z[k][lane];
      }
    }
  } else if (near) {
    float x[6];
    features<float>(s, x);
    mlp_logits<float>(uniform_f32(prepared), x, zl);
    sel = mask_from_logits<float>(zl);
  }
  if (z) {
#pragma unroll
    for (int k = 0; k < 4; ++k) z[k] = zl[k];
  }
  return sel;
}

// The two-part re-check's LDS of a scalar kernel: the remainder table,
// staged once per workgroup, and one WaveRecheck per wave.
#define N6_SCALAR_RECHECK_LDS(SPLIT, selector, prepared)                                          \
  __shared__ u32 lot[(SPLIT) ? LO_REGS * 64 : 1];                                                \
  __shared__ WaveRecheck wrl[(SPLIT) ? WPB : 1];                                                 \
  if ((SPLIT) && (selector) == 0) {                                                              \
    const u32 *g_ = (const u32 *)((const char *)(prepared) + PREP_LO_OFF);                       \
    for (int i_ = threadIdx.x; i_ < LO_REGS * 64; i_ += TPB) lot[i_] = g_[i_];                   \
    __syncthreads();                                                                             \
  }                                                                                              \
  WaveRecheck &wr = wrl[(SPLIT) ? (threadIdx.x >> 6) : 0];

template <int PREC, bool SPLIT>
__global__ void __launch_bounds__(TPB)
k_fast_scalar(int mode, Line1D ln, const void *__restrict__ prepared, float margin,
              const float *__restrict__ src, int64_t n, int sign, int selector,
              const uint8_t *__restrict__ min, float *__restrict__ out, uint8_t *__restrict__ mout,
              float *__restrict__ zout) {
  const int lane = threadIdx.x & 63;
  const int64_t nchunk = (n + 63) / 64;
  N6_SCALAR_RECHECK_LDS(SPLIT, selector, prepared)
  Wts w;
  if (selector == 0) load_wts<PREC>(prepared, lane, w);
  for (int64_t ch = (int64_t)blockIdx.x * WPB + (threadIdx.x >> 6); ch < nchunk;
       ch += (int64_t)gridDim.x * WPB) {
    const int64_t k = ch * 64 + lane;
    const bool valid = k < n;
    const int64_t kc = valid ? k : n - 1;
    float s[6];
    if (mode == 0) {
#pragma unroll
      for (int j = 0; j < 6; ++j) s[j] = sign > 0 ? src[kc + j] : src[kc + 5 - j];
    } else if (mode == 1) {
      const int p = line_of_face(ln, kc);
      const int64_t o = ln.offsets[p], nn = ln.offsets[p + 1] - o, kk = kc - o - p;
#pragma unroll
      for (int j = 0; j < 6; ++j) s[j] = src[o + ghost(kk - 3 + j, nn, ln.bc)];
    } else {
#pragma unroll
      for (int j = 0; j < 6; ++j) s[j] = src[6 * kc + j];
    }
    u32 sel;
    float z[4];
    if (selector == 0) {
      sel = mlp_select<PREC, SPLIT>(w, prepared, lot, wr, margin, s, valid, mode == 2 ? z : nullptr);
    } else if (selector == 1) {
      sel = 15u;
    } else if (selector == 2) {
      sel = 0u;
    } else if (selector == 4) {
      sel = teno_mask_of<float>(s);
    } else {
      sel = min[kc] & 15u;
    }
    if (!valid) continue;
    if (mode == 2) {
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) zout[4 * k + kk] = z[kk];
    } else {
      out[k] = combine_fast(s, sel);
    }
    if (mout) mout[k] = (uint8_t)sel;
  }
}

// Label of one scalar stencil by the selector; the MFMA classification is a
// wave-wide operation, so every lane of the wave calls this together.
template <int PREC, bool SPLIT>
N6_DEV u32 scalar_select(const Wts &w, int selector, const void *prepared, const u32 *lot,
                         WaveRecheck &wr, float margin, const float s[6], bool valid, u32 mask_in) {
  if (selector == 0) return mlp_select<PREC, SPLIT>(w, prepared, lot, wr, margin, s, valid, nullptr);
  if (selector == 1) return 15u;
  if (selector == 2) return 0u;
  if (selector == 4) return teno_mask_of<float>(s);
  return mask_in & 15u;
}

// Burgers faces (Sec. 4.3): one lane per face; f = u^2/2, Rusanov speed
// alpha = max |u| over the six cells, f+- = (f +- alpha u)/2 ('-' mirrored);
// both split stencils classified (re-check in place), face flux = sum of the
// two reconstructions.
template <int PREC, bool SPLIT>
__global__ void __launch_bounds__(TPB)
k_fast_burgers(Line1D ln, const void *__restrict__ prepared, float margin, int selector,
               const float *__restrict__ u, const uint8_t *__restrict__ min,
               float *__restrict__ Fh, uint8_t *__restrict__ mout) {
  const int lane = threadIdx.x & 63;
  const int64_t nf = ln.faces(), nchunk = (nf + 63) / 64;
  N6_SCALAR_RECHECK_LDS(SPLIT, selector, prepared)
  Wts w;
  if (selector == 0) load_wts<PREC>(prepared, lane, w);
  for (int64_t ch = (int64_t)blockIdx.x * WPB + (threadIdx.x >> 6); ch < nchunk;
       ch += (int64_t)gridDim.x * WPB) {
    const int64_t g = ch * 64 + lane;
    const bool valid = g < nf;
    const int64_t gc = valid ? g : nf - 1;
    const int p = line_of_face(ln, gc);
    const int64_t o = ln.offsets[p], n = ln.offsets[p + 1] - o, k = gc - o - p;
    float us[6], alpha = 0.f;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      us[j] = u[o + ghost(k - 3 + j, n, ln.bc)];
      alpha = fmaxf(alpha, fabsf(us[j]));
    }
    float sp[6], sm[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      const float f = 0.5f * (us[j] * us[j]);
      const float t = alpha * us[j];
      sp[j] = 0.5f * (f + t);
      sm[5 - j] = 0.5f * (f - t);
    }
    const u32 mi = min ? min[gc] : 0u;
    const u32 selp = scalar_select<PREC, SPLIT>(w, selector, prepared, lot, wr, margin, sp, valid, mi);
    const u32 selm = scalar_select<PREC, SPLIT>(w, selector, prepared, lot, wr, margin, sm, valid, mi >> 4);
    if (!valid) continue;
    Fh[g] = combine_fast(sp, selp) + combine_fast(sm, selm);
    if (mout) mout[g] = (uint8_t)(selp | (selm << 4));
  }
}

// Clears the re-check counters (one per evaluation kind and sweep direction).
__global__ void k_zero_u32(u32 *p) {
  if (threadIdx.x < QCOUNTERS) p[threadIdx.x] = 0u;
}

__global__ void __launch_bounds__(TPB) k_copy_u8(const uint8_t *__restrict__ a, uint8_t *__restrict__ b, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TPB) b[i] = a[i];
}

hipError_t copy_bytes(const uint8_t *a, uint8_t *b, int64_t n, hipStream_t s) {
  const int64_t blocks = (n + TPB - 1) / TPB;
  hipLaunchKernelGGL(k_copy_u8, dim3((unsigned)(blocks < 4096 ? blocks : 4096)), dim3(TPB), 0, s, a, b, n);
  return hipGetLastError();
}

// Prepared block: FP32 copy of the parameters, the BF16 and FP16 per-lane
// operand tables, b5 in FP32, the per-neuron scales of the hidden layers, the
// FP32 operand table of the BF16 re-check and the FP16 remainder table.
constexpr int PREP_THREADS = (TAB_REGS > F4_REGS ? TAB_REGS : F4_REGS) * 64;
static_assert(NPARAM <= PREP_THREADS, "k_prepare covers every element");
// Scales of hidden layers 1..4 (64 + 32 + 16 + 8 values, FP64).
constexpr int SC1 = 0, SC2 = 64, SC3 = 96, SC4 = 112, NSCALE = 120;
static_assert(PREP_B5_OFF + 16 <= PREP_SCALE_OFF && PREP_SCALE_OFF + NSCALE * 8 <= PREP_F4_OFF,
              "prepared block layout");

// A-priori activation scales (one workgroup of 64 threads).  With inputs
// |x_i| <= 1 (eq. normalizainput) the pre-activation z_o of a first-layer
// neuron is at most b_o + sum_i |W_oi|; a deeper neuron, whose inputs are
// ReLU outputs in [0, U_i], at most b_o + sum_i max(W_oi, 0) U_i.  The scale
// s_o adds 1/32 of the neuron's absolute sum (|b_o| + sum_i |W_oi| U_i) to
// that bound, so the BF16/FP16 rounding of the scaled products (a few 2^-8
// of the absolute sum) cannot push a scaled pre-activation above 1.  A
// neuron whose bound is <= 0 never fires; its scale is 1.
__global__ void __launch_bounds__(64) k_prepare_scales(const double *__restrict__ P,
                                                       double *__restrict__ S) {
  __shared__ double U[64];
  const int o = threadIdx.x;
  double u = P[OB1 + o], a = fabs(P[OB1 + o]);
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    u += fabs(P[OW1 + o * 6 + i]);
    a += fabs(P[OW1 + o * 6 + i]);
  }
  S[SC1 + o] = u > 0.0 ? u + a / 32.0 : 1.0;
  U[o] = u > 0.0 ? u : 0.0;
  __syncthreads();
  const int nin[3] = {64, 32, 16}, nout[3] = {32, 16, 8};
  const int ow[3] = {OW2, OW3, OW4}, ob[3] = {OB2, OB3, OB4}, so[3] = {SC2, SC3, SC4};
  for (int l = 0; l < 3; ++l) {
    double ul = 0.0;
    if (o < nout[l]) {
      ul = P[ob[l] + o];
      a = fabs(P[ob[l] + o]);
      for (int i = 0; i < nin[l]; ++i) {
        const double w = P[ow[l] + o * nin[l] + i];
        ul += (w > 0.0 ? w : 0.0) * U[i];
        a += fabs(w) * U[i];
      }
      S[so[l] + o] = ul > 0.0 ? ul + a / 32.0 : 1.0;
    }
    __syncthreads();
    if (o < nout[l]) U[o] = ul > 0.0 ? ul : 0.0;
    __syncthreads();
  }
}

// Entry t of the prepared block (FP32 copy, FP32 and BF16/FP16 operand
// tables).  With S (the scales above), the BF16/FP16 tables hold the scaled
// network: hidden neuron o of layer l computes z_o / s_o, so its inputs'
// weights are W_oi s_i / s_o (s_i = 1 for the six features), its bias b_o /
// s_o, and the output layer's weights W5_ki s_i; without S (the training
// tables) the plain weights.
// FP64 value of element q2 (0, 1) of weight register reg (reg < 36 or 84 <=
// reg < R_C3; the bias registers excluded) of lane `lane` of the BF16/FP16
// operand table, scaled by S (nullptr: unscaled).
N6_DEV double tab_value(const double *__restrict__ P, const double *__restrict__ S, int reg, int lane,
                        int q2) {
  auto sc = [&](int base, int i) { return S ? S[base + i] : 1.0; };
  const int i = lane % 32, h = lane / 32;
  if (reg >= 84 && reg < R_T3) {
    // L1 with K = 16: lanes (i, 0) slots 0..7 = W1 row o on the leading
    // parts, b1 on the bias input; lanes (i, 1) slots 8..15 = W1 row o on the
    // trailing parts
    const int tt = (reg - 84) / 4, k = 2 * ((reg - 84) % 4) + q2, o = 32 * tt + i;
    const double x = k < 6 ? P[OW1 + o * 6 + k] : (k == 6 && h == 0 ? P[OB1 + o] : 0.0);
    return x / sc(SC1, o);
  }
  if (reg < 4) {  // L1: tile reg/2, elements e = 2*(reg%2) + q2, K slot 4h + e
    const int tt = reg / 2, e = 2 * (reg % 2) + q2, kk = 4 * h + e, o = 32 * tt + i;
    const double x = kk < 6 ? P[OW1 + o * 6 + kk] : (kk == 6 ? P[OB1 + o] : 0.0);
    return x / sc(SC1, o);
  }
  if (reg < 20) {  // L2 step s
    const int s = (reg - 4) / 4, e = 2 * ((reg - 4) % 4) + q2;
    const int n1 = 32 * (s / 2) + 16 * (s % 2) + 8 * (e / 4) + 4 * h + e % 4;
    return P[OW2 + i * 64 + n1] * sc(SC1, n1) / sc(SC2, i);
  }
  if (reg < 28) {  // L3 step s
    const int s = (reg - 20) / 4, e = 2 * ((reg - 20) % 4) + q2;
    const int n2 = 8 * (2 * s + e / 4) + 4 * h + e % 4;
    return i < 16 ? P[OW3 + i * 32 + n2] * sc(SC2, n2) / sc(SC3, i) : 0.0;
  }
  if (reg < 32) {  // L4
    const int e = 2 * (reg - 28) + q2;
    const int n3 = 8 * (e / 4) + 4 * h + e % 4;
    return i < 8 ? P[OW4 + i * 16 + n3] * sc(SC3, n3) / sc(SC4, i) : 0.0;
  }
  if (reg < 36) {  // L5: K slots e < 4 carry tile 0 (rows 0..3), e >= 4 tile 1 (rows 4..7)
    const int e = 2 * (reg - 32) + q2, t5 = e / 4, n4 = 4 * h + e % 4;
    return i / 4 == t5 ? P[OW5 + (i % 4) * 8 + n4] * sc(SC4, n4) : 0.0;
  }
  // inference L3..L5 on 16x16x32: lane (m, G) = (lane % 16, lane / 16), K
  // slot 8G + tt of the A operand, tt = 2 (reg % 4) + q2
  const int m = lane % 16, G = lane / 16, tt = 2 * ((reg - R_T3) % 4) + q2;
  if (reg < R_T4) {  // L3: row m; K slot -> L2 row of X / Y of h = G / 2
    const int ii = tt + 8 * (G % 2), n2 = 8 * (ii / 4) + 4 * (G / 2) + ii % 4;
    return P[OW3 + m * 32 + n2] * sc(SC2, n2) / sc(SC3, m);
  }
  if (reg < R_T5) {  // L4, both blocks: rows m < 8 block A, m >= 8 block B
    const int n3 = 4 * G + tt % 4;
    return (tt < 4) == (m < 8) ? P[OW4 + (m % 8) * 16 + n3] * sc(SC3, n3) / sc(SC4, m % 8) : 0.0;
  }
  // L5, four blocks: row m = 4 B + k, block B = 2 tile + half; K slot 8G + tt
  // holds tile tt / 4, half G / 2, L4 neuron 4 (G % 2) + tt % 4
  const int blk = m / 4, n4 = 4 * (G % 2) + tt % 4;
  return (tt / 4 == blk / 2 && G / 2 == blk % 2) ? P[OW5 + (m % 4) * 8 + n4] * sc(SC4, n4) : 0.0;
}

// FP16 value of x and what that rounding leaves, rounded to FP16 again.
N6_DEV f32x2 f16_parts(double x) {
  const float hi = (float)(_Float16)(float)x;
  return f32x2{hi, (float)(_Float16)(float)(x - (double)hi)};
}

// Register reg of lane `lane` of the remainder table (LO_* layout): the
// FP16 remainders of the scaled weights, in the operand order of the FP16
// table's register it pairs with (L1, L2, and L3 / L4 on 16x16x32); LO_S5A /
// LO_S5B the output layer of one 32-evaluation tile on 16x16x32: K slots
// 8G..8G+3 the leading parts, 8G+4..8G+7 the trailing parts of lane group
// G's L4 rows (block G / 2, neurons 4 (G % 2)..), output rows 4B..4B+3 the
// logits of block B % 2; S5A the FP16 weights on both parts, S5B the
// remainder weights on the leading parts.
N6_DEV u32 lo_table_value(const double *__restrict__ P, const double *__restrict__ S, int reg,
                          int lane) {
  float v[2];
  for (int q2 = 0; q2 < 2; ++q2) {
    if (reg < LO_S5A) {
      const int m = reg < LO_A2 ? 84 + reg : (reg < LO_T3 ? 4 + reg - LO_A2 : (reg < LO_T4 ? R_T3 + reg - LO_T3 : R_T4 + reg - LO_T4));
      v[q2] = f16_parts(tab_value(P, S, m, lane, q2))[1];
    } else {
      const int m = lane % 16, G = lane / 16, tt = 2 * (reg % 4) + q2, n4 = 4 * (G % 2) + tt % 4;
      const f32x2 w = (G / 2 == (m / 4) % 2) ? f16_parts(P[OW5 + (m % 4) * 8 + n4] * S[SC4 + n4])
                                             : f32x2{0.f, 0.f};
      v[q2] = reg < LO_S5B ? w[0] : (tt < 4 ? w[1] : 0.f);
    }
  }
  return pack2<3>(v[0], v[1]);
}

// Entry t of the prepared block (FP32 copy, FP32 and BF16/FP16 operand
// tables).  With S (the scales above), the BF16/FP16 tables hold the scaled
// network: hidden neuron o of layer l computes z_o / s_o, so its inputs'
// weights are W_oi s_i / s_o (s_i = 1 for the six features), its bias b_o /
// s_o, and the output layer's weights W5_ki s_i; without S (the training
// tables) the plain weights and no remainder table.
N6_DEV void prepare_entry(const double *__restrict__ P, const double *__restrict__ S,
                          char *__restrict__ prep, int t) {
  if (t < NPARAM) ((float *)prep)[t] = (float)P[t];
  if (t < 4) ((float *)(prep + PREP_B5_OFF))[t] = (float)P[OB5 + t];
  if (t < F4_REGS * 64) ((float *)(prep + PREP_F4_OFF))[t] = f4_table_value(P, t / 64, t % 64);
  if (S && t < LO_REGS * 64) {
    const int reg = t / 64, lane = t % 64;
    ((u32 *)(prep + PREP_LO_OFF))[((reg / 4) * 64 + lane) * 4 + reg % 4] = lo_table_value(P, S, reg, lane);
  }
  if (t >= TAB_REGS * 64) return;
  const int reg = t / 64, lane = t % 64, h = lane / 32;
  u32 wb, wh;
  if (reg < 36 || (reg >= 84 && reg < R_C3)) {
    const float v0 = (float)tab_value(P, S, reg, lane, 0), v1 = (float)tab_value(P, S, reg, lane, 1);
    wb = pack2<2>(v0, v1);
    wh = pack2<3>(v0, v1);
  } else if (reg >= R_C3) {
    // biases of the 16x16 tiles: register r of lane group G is row 4G + r
    auto sc = [&](int base, int i) { return S ? S[base + i] : 1.0; };
    const int row = 4 * (lane / 16) + (reg - R_C3) % 4;
    const double x = reg < R_C4 ? P[OB3 + row] / sc(SC3, row) : P[OB4 + row % 8] / sc(SC4, row % 8);
    wb = wh = __builtin_bit_cast(u32, (float)x);
  } else {
    // bias tuples: C register r of lane (j, h) is row 8(r/4) + 4h + r%4
    auto sc = [&](int base, int i) { return S ? S[base + i] : 1.0; };
    const int blk = (reg - 36) / 16, r = (reg - 36) % 16;
    const int row = 8 * (r / 4) + 4 * h + r % 4;
    double x;
    if (blk == 0) x = P[OB2 + row] / sc(SC2, row);
    else if (blk == 1) x = row < 16 ? P[OB3 + row] / sc(SC3, row) : 0.0;
    else x = row < 8 ? P[OB4 + row] / sc(SC4, row) : 0.0;
    wb = wh = __builtin_bit_cast(u32, (float)x);
  }
  ((u32 *)(prep + PREP_BF16_OFF))[reg * 64 + lane] = wb;
  ((u32 *)(prep + PREP_F16_OFF))[reg * 64 + lane] = wh;
}

__global__ void __launch_bounds__(TPB) k_prepare(const double *__restrict__ P, char *__restrict__ prep) {
  prepare_entry(P, (const double *)(prep + PREP_SCALE_OFF), prep, blockIdx.x * TPB + threadIdx.x);
}

inline unsigned grid_for(int64_t items_per_wave_chunks) {
  const int64_t blocks = (items_per_wave_chunks + WPB - 1) / WPB;
  return (unsigned)(blocks < 2048 ? (blocks > 0 ? blocks : 1) : 2048);
}

// Launch shape of the fused face kernel and of the re-check pair.
struct FaceLaunch {
  unsigned grid;
  int waves, xcd;
};

FaceLaunch face_launch(const FastArgs &fa, int64_t nchunk) {
  FaceLaunch L;
  L.waves = (fa.face_waves == 2 || fa.face_waves == 8) ? fa.face_waves : 4;
  const int64_t need = (nchunk + L.waves - 1) / L.waves;
  const int64_t cap = fa.face_blocks > 0 ? fa.face_blocks : 2048;
  const int64_t g = need < cap ? need : cap;
  L.grid = (unsigned)(g > 0 ? g : 1);
  L.xcd = (fa.xcd_order && L.grid % 8 == 0) ? 1 : 0;
  return L;
}

// ---- classifier training on MFMA (BF16, FP32 accumulation) ------------------
// Tiles of 32 samples per wave, persistent over the mini-batch.  Forward: the
// inference tiles (activations kept, as packed BF16, for the backward pass).
// Backward: delta_{l-1} = (W_l^T delta_l) o [h_{l-1} > 0] on MFMA with the
// transposed weights as the A operand, K order permuted exactly like the
// forward chaining, so deltas stay in the lanes.  Weight gradients
// dW_l = sum over samples of delta_l h_{l-1}^T are MFMA products with K =
// samples: delta and activation tiles go through a lane-private LDS transpose
// ([neuron][sample], BF16), 16 samples per instruction.  Bias gradients of
// L2..L5 are lane sums reduced across the 32 lanes of each half at the end;
// b1 comes out of the L1 product through the constant input slot.
constexpr int BT_REGS = 24;  // backward A tables: L5 2, L4 2, L3 4, L2 16

// Entry t of the backward operand tables.
N6_DEV void prepare_bwd_entry(const double *__restrict__ P, u32 *__restrict__ tab, int t) {
  if (t >= BT_REGS * 64) return;
  const int reg = t / 64, lane = t % 64, i = lane % 32, h = lane / 32;
  float v[2];
  for (int q2 = 0; q2 < 2; ++q2) {
    double x = 0.0;
    if (reg < 2) {  // L5^T, 32x32x8: K slot 4h + e = output neuron of L5
      const int e = 2 * reg + q2, k = 4 * h + e;
      x = (k < 4 && i < 8) ? P[OW5 + k * 8 + i] : 0.0;
    } else if (reg < 4) {  // L4^T, 32x32x8
      const int e = 2 * (reg - 2) + q2, k = 4 * h + e;
      x = (i < 16) ? P[OW4 + k * 16 + i] : 0.0;
    } else if (reg < 8) {  // L3^T, 32x32x16: K slot = L3 output row 8(e/4)+4h+e%4
      const int e = 2 * (reg - 4) + q2, n3 = 8 * (e / 4) + 4 * h + e % 4;
      x = P[OW3 + n3 * 32 + i];
    } else {  // L2^T, output tile t (L1 neurons 32t..32t+31), K step s
      const int r = reg - 8, tt = r / 8, s = (r % 8) / 4, e = 2 * (r % 4) + q2;
      const int n2 = 8 * (2 * s + e / 4) + 4 * h + e % 4;
      x = P[OW2 + n2 * 64 + 32 * tt + i];
    }
    v[q2] = (float)x;
  }
  tab[reg * 64 + lane] = pack2<2>(v[0], v[1]);
}

// Both tables of a training step in one launch: the first PREP_BLOCKS
// workgroups build the forward block, the rest the backward tables.
constexpr int PREP_BLOCKS = (PREP_THREADS + TPB - 1) / TPB;
__global__ void __launch_bounds__(TPB) k_prepare_train(const double *__restrict__ P, char *__restrict__ prep,
                                                       u32 *__restrict__ tab) {
  if ((int)blockIdx.x < PREP_BLOCKS)
    prepare_entry(P, nullptr, prep, blockIdx.x * TPB + threadIdx.x);
  else
    prepare_bwd_entry(P, tab, ((int)blockIdx.x - PREP_BLOCKS) * TPB + threadIdx.x);
}

// Writes rows [0, nrows) of a C-layout FP32 tile (lane (j, h), register r =
// row 8(r/4) + 4h + r%4) as BF16 into T[row][j].
N6_DEV void tile_to_lds(const f32x16 &c, int nrows, int row0, __bf16 (*T)[32], int j, int h) {
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int row = 8 * (r / 4) + 4 * h + r % 4;
    if (row < nrows) T[row0 + row][j] = (__bf16)c[r];
  }
}
// Same for a packed BF16 tile (registers p hold C registers 2p, 2p+1).
template <int NPACKED>
N6_DEV void packed_to_lds(const u32 *hp, int nrows, int row0, __bf16 (*T)[32], int j, int h) {
#pragma unroll
  for (int p = 0; p < NPACKED; ++p) {
    const bf16x2 v = __builtin_bit_cast(bf16x2, hp[p]);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int r = 2 * p + q, row = 8 * (r / 4) + 4 * h + r % 4;
      if (row < nrows) T[row0 + row][j] = v[q];
    }
  }
}
// MFMA operand of 8 consecutive samples of one neuron: rows >= nrows are zero.
N6_DEV u32x4 lds_operand(__bf16 (*T)[32], int row, int nrows, int k0) {
  if (row >= nrows) return u32x4{0u, 0u, 0u, 0u};
  return *(const u32x4 *)&T[row][k0];
}
N6_DEV float bf16_pos(u32 packed, int half) {  // ReLU derivative of a stored activation
  const bf16x2 v = __builtin_bit_cast(bf16x2, packed);
  return (float)v[half] > 0.f ? 1.f : 0.f;
}

__global__ void __launch_bounds__(TPB)
k_grad_mfma(const void *__restrict__ prepared, const u32 *__restrict__ btab,
            const float *__restrict__ s, const uint8_t *__restrict__ y,
            const int64_t *__restrict__ idx, int64_t m, float inv_m, int nwaves,
            float *__restrict__ part, double *__restrict__ lpart) {
  __shared__ __attribute__((aligned(16))) __bf16 Td[WPB][64][32];
  __shared__ __attribute__((aligned(16))) __bf16 Ta[WPB][64][32];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, j = lane & 31, h = lane >> 5;
  const int wid = blockIdx.x * WPB + wv;
  WtsT w;
  load_wts_train(prepared, lane, w);
  u32x2 bt5, bt4;
  u32x4 bt3, bt2[2][2];
  bt5 = u32x2{btab[0 * 64 + lane], btab[1 * 64 + lane]};
  bt4 = u32x2{btab[2 * 64 + lane], btab[3 * 64 + lane]};
  bt3 = u32x4{btab[4 * 64 + lane], btab[5 * 64 + lane], btab[6 * 64 + lane], btab[7 * 64 + lane]};
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int st = 0; st < 2; ++st) {
      const int b = 8 + 8 * t + 4 * st;
      bt2[t][st] = u32x4{btab[(b + 0) * 64 + lane], btab[(b + 1) * 64 + lane],
                         btab[(b + 2) * 64 + lane], btab[(b + 3) * 64 + lane]};
    }
  const f32x16 zero = {};
  f32x16 g1a = zero, g1b = zero, g2a = zero, g2b = zero, g3 = zero, g4 = zero, g5 = zero;
  float db2[16], db3[8], db4[4], db5[4], lsum = 0.f;
#pragma unroll
  for (int r = 0; r < 16; ++r) db2[r] = 0.f;
#pragma unroll
  for (int r = 0; r < 8; ++r) db3[r] = 0.f;
#pragma unroll
  for (int r = 0; r < 4; ++r) db4[r] = db5[r] = 0.f;
  const int64_t ntile = (m + 31) / 32;
  for (int64_t tile = wid; tile < ntile; tile += nwaves) {
    const int64_t smp = tile * 32 + j;
    const bool valid = smp < m;
    float x[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    unsigned lab = 0;
    if (valid) {
      const int64_t id = idx ? idx[smp] : smp;
      float st6[6];
#pragma unroll
      for (int k = 0; k < 6; ++k) st6[k] = s[6 * id + k];
      features<float>(st6, x);
      lab = y[id];
    }
    const float one = valid ? 1.f : 0.f;
    const u32x2 bin = h == 0 ? u32x2{pack2<2>(x[0], x[1]), pack2<2>(x[2], x[3])}
                             : u32x2{pack2<2>(x[4], x[5]), pack2<2>(one, 0.f)};
    // forward
    const f32x16 c1a = mma8<2>(w.a1[0], bin, zero);
    const f32x16 c1b = mma8<2>(w.a1[1], bin, zero);
    u32 h1a[8], h1b[8];
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      h1a[p] = relu_pack<2>(c1a[2 * p], c1a[2 * p + 1]);
      h1b[p] = relu_pack<2>(c1b[2 * p], c1b[2 * p + 1]);
    }
    f32x16 c2 = mma16<2>(w.a2[0], u32x4{h1a[0], h1a[1], h1a[2], h1a[3]}, w.b2);
    c2 = mma16<2>(w.a2[1], u32x4{h1a[4], h1a[5], h1a[6], h1a[7]}, c2);
    c2 = mma16<2>(w.a2[2], u32x4{h1b[0], h1b[1], h1b[2], h1b[3]}, c2);
    c2 = mma16<2>(w.a2[3], u32x4{h1b[4], h1b[5], h1b[6], h1b[7]}, c2);
    u32 h2[8];
#pragma unroll
    for (int p = 0; p < 8; ++p) h2[p] = relu_pack<2>(c2[2 * p], c2[2 * p + 1]);
    f32x16 c3 = mma16<2>(w.a3[0], u32x4{h2[0], h2[1], h2[2], h2[3]}, w.b3);
    c3 = mma16<2>(w.a3[1], u32x4{h2[4], h2[5], h2[6], h2[7]}, c3);
    u32 h3[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) h3[p] = relu_pack<2>(c3[2 * p], c3[2 * p + 1]);
    const f32x16 c4 = mma16<2>(w.a4, u32x4{h3[0], h3[1], h3[2], h3[3]}, w.b4);
    // L4 rows 8..31 are padding; the L5 K slots of the second tile stay zero
    u32 h4[2];
#pragma unroll
    for (int p = 0; p < 2; ++p) h4[p] = relu_pack<2>(c4[2 * p], c4[2 * p + 1]);
    const f32x16 c5 = mma16<2>(w.a5, u32x4{h4[0], h4[1], 0u, 0u}, zero);
    // loss and output deltas (lanes of the first half hold the four logits)
    float d5[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float z = c5[k] + w.b5[k];
      const float yk = (float)((lab >> k) & 1u);
      const bool act = valid && h == 0;
      const float sp = z > 0.f ? z + log1pf(expf(-z)) : log1pf(expf(z));  // softplus(z)
      lsum += act ? 0.25f * (sp - yk * z) : 0.f;
      d5[k] = act ? (1.f / (1.f + expf(-z)) - yk) * 0.25f * inv_m : 0.f;
      db5[k] += d5[k];
    }
    // backward through L5 (K = 4 output neurons, 32x32x8)
    const u32x2 D5 = u32x2{pack2<2>(d5[0], d5[1]), pack2<2>(d5[2], d5[3])};
    const f32x16 e4 = mma8<2>(bt5, D5, zero);
    float d4[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      d4[r] = e4[r] * bf16_pos(h4[r >> 1], r & 1);
      db4[r] += d4[r];
    }
    const u32x2 D4 = u32x2{pack2<2>(d4[0], d4[1]), pack2<2>(d4[2], d4[3])};
    const f32x16 e3 = mma8<2>(bt4, D4, zero);
    float d3[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      d3[r] = e3[r] * bf16_pos(h3[r >> 1], r & 1);
      db3[r] += d3[r];
    }
    const u32x4 D3 = u32x4{pack2<2>(d3[0], d3[1]), pack2<2>(d3[2], d3[3]), pack2<2>(d3[4], d3[5]),
                           pack2<2>(d3[6], d3[7])};
    const f32x16 e2 = mma16<2>(bt3, D3, zero);
    f32x16 d2;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      d2[r] = e2[r] * bf16_pos(h2[r >> 1], r & 1);
      db2[r] += d2[r];
    }
    const u32x4 D2a = u32x4{pack2<2>(d2[0], d2[1]), pack2<2>(d2[2], d2[3]), pack2<2>(d2[4], d2[5]),
                            pack2<2>(d2[6], d2[7])};
    const u32x4 D2b = u32x4{pack2<2>(d2[8], d2[9]), pack2<2>(d2[10], d2[11]),
                            pack2<2>(d2[12], d2[13]), pack2<2>(d2[14], d2[15])};
    f32x16 e1a = mma16<2>(bt2[0][0], D2a, zero);
    e1a = mma16<2>(bt2[0][1], D2b, e1a);
    f32x16 e1b = mma16<2>(bt2[1][0], D2a, zero);
    e1b = mma16<2>(bt2[1][1], D2b, e1b);
    f32x16 d1a, d1b, d5t = zero, d4t = zero, d3t = zero;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      d1a[r] = e1a[r] * bf16_pos(h1a[r >> 1], r & 1);
      d1b[r] = e1b[r] * bf16_pos(h1b[r >> 1], r & 1);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      d5t[r] = d5[r];
      d4t[r] = d4[r];
    }
#pragma unroll
    for (int r = 0; r < 8; ++r) d3t[r] = d3[r];
    // weight gradients: transpose through LDS, K = 32 samples in two steps
    __bf16(*TD)[32] = Td[wv];
    __bf16(*TA)[32] = Ta[wv];
    auto wgrad = [&](f32x16 &acc, int nout, int nin, int drow0, int arow0) {
#pragma unroll
      for (int kk = 0; kk < 2; ++kk) {
        const u32x4 A = lds_operand(TD, drow0 + j, drow0 + nout, 16 * kk + 8 * h);
        const u32x4 B = lds_operand(TA, arow0 + j, arow0 + nin, 16 * kk + 8 * h);
        acc = mma16<2>(A, B, acc);
      }
    };
    // L5 and L4: deltas rows 0..3 / 4..11, activations h4 rows 0..7 / h3 rows 8..23
    tile_to_lds(d5t, 4, 0, TD, j, h);
    tile_to_lds(d4t, 8, 4, TD, j, h);
    packed_to_lds<4>(h4, 8, 0, TA, j, h);
    packed_to_lds<4>(h3, 16, 8, TA, j, h);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    wgrad(g5, 4, 8, 0, 0);
    wgrad(g4, 8, 16, 4, 8);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    // L3: delta3 rows 0..15, h2 rows 0..31
    tile_to_lds(d3t, 16, 0, TD, j, h);
    packed_to_lds<8>(h2, 32, 0, TA, j, h);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    wgrad(g3, 16, 32, 0, 0);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    // L2: delta2 rows 0..31, h1 rows 0..63 (two output-column tiles)
    tile_to_lds(d2, 32, 0, TD, j, h);
    packed_to_lds<8>(h1a, 32, 0, TA, j, h);
    packed_to_lds<8>(h1b, 32, 32, TA, j, h);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    wgrad(g2a, 32, 32, 0, 0);
    wgrad(g2b, 32, 32, 0, 32);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    // L1: delta1 rows 0..63, inputs x0..x5 and the constant slot (rows 0..6)
    tile_to_lds(d1a, 32, 0, TD, j, h);
    tile_to_lds(d1b, 32, 32, TD, j, h);
    if (h == 0) {
#pragma unroll
      for (int k = 0; k < 6; ++k) TA[k][j] = (__bf16)x[k];
      TA[6][j] = (__bf16)one;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    wgrad(g1a, 32, 7, 0, 0);
    wgrad(g1b, 32, 7, 32, 0);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  }
  // partial gradient of this wave in the parameter layout
  float *gp = part + (int64_t)wid * NPARAM;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int o = 8 * (r / 4) + 4 * h + r % 4, in = j;
    if (o < 4 && in < 8) gp[OW5 + o * 8 + in] = g5[r];
    if (o < 8 && in < 16) gp[OW4 + o * 16 + in] = g4[r];
    if (o < 16) gp[OW3 + o * 32 + in] = g3[r];
    gp[OW2 + o * 64 + in] = g2a[r];
    gp[OW2 + o * 64 + 32 + in] = g2b[r];
    if (in < 6) {
      gp[OW1 + o * 6 + in] = g1a[r];
      gp[OW1 + (32 + o) * 6 + in] = g1b[r];
    } else if (in == 6) {
      gp[OB1 + o] = g1a[r];
      gp[OB1 + 32 + o] = g1b[r];
    }
  }
  // bias gradients: sum over the 32 samples of each lane half
  auto half_sum = [&](float v) {
#pragma unroll
    for (int off = 16; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
  };
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const float v = half_sum(db2[r]);
    if (j == 0) gp[OB2 + 8 * (r / 4) + 4 * h + r % 4] = v;
  }
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const float v = half_sum(db3[r]);
    if (j == 0) gp[OB3 + 8 * (r / 4) + 4 * h + r % 4] = v;
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const float v4 = half_sum(db4[r]);
    if (j == 0) gp[OB4 + 4 * h + r] = v4;
    const float v5 = half_sum(db5[r]);
    if (j == 0 && h == 0) gp[OB5 + r] = v5;
  }
  float l = lsum;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) l += __shfl_xor(l, off);
  if (lane == 0) lpart[wid] = (double)l;
}

}  // namespace

// Gradient partials of one mini-batch on MFMA: one partial per wave.
int train_mfma_waves(int64_t m) {
  const int64_t t = (m + 31) / 32;
  const int64_t nw = t < 1024 ? t : 1024;
  return (int)((nw + WPB - 1) / WPB * WPB);
}
size_t train_mfma_tab_bytes() { return PREP_BYTES + BT_REGS * 64 * 4; }

hipError_t launch_grad_mfma(const double *P, void *tabs, const float *s, const uint8_t *y,
                            const int64_t *idx, int64_t m, float *part, double *lpart,
                            hipStream_t st) {
  char *prep = (char *)tabs;
  u32 *btab = (u32 *)(prep + PREP_BYTES);
  hipLaunchKernelGGL(k_prepare_train, dim3(PREP_BLOCKS + (BT_REGS * 64 + TPB - 1) / TPB), dim3(TPB), 0,
                     st, P, prep, btab);
  const int nw = train_mfma_waves(m);
  hipLaunchKernelGGL(k_grad_mfma, dim3(nw / WPB), dim3(TPB), 0, st, prep, btab, s, y, idx, m,
                     (float)(1.0 / (double)m), nw, part, lpart);
  return hipGetLastError();
}

size_t fast_prepared_bytes() { return PREP_BYTES; }
const void *fast_prepared_f32(const void *prepared) { return prepared; }

hipError_t launch_fast_prepare(const double *P, void *prepared, hipStream_t s) {
  hipLaunchKernelGGL(k_prepare_scales, dim3(1), dim3(64), 0, s, P,
                     (double *)((char *)prepared + PREP_SCALE_OFF));
  hipLaunchKernelGGL(k_prepare, dim3((PREP_THREADS + TPB - 1) / TPB), dim3(TPB), 0, s, P,
                     (char *)prepared);
  return hipGetLastError();
}

// The scalar kernel of an operand precision and re-check arithmetic.
#define N6_SCALAR(precision, split, ...)                                                        \
  do {                                                                                        \
    if ((precision) == 2)                                                                     \
      hipLaunchKernelGGL((k_fast_scalar<2, false>), __VA_ARGS__);                             \
    else if (split)                                                                           \
      hipLaunchKernelGGL((k_fast_scalar<3, true>), __VA_ARGS__);                              \
    else                                                                                      \
      hipLaunchKernelGGL((k_fast_scalar<3, false>), __VA_ARGS__);                             \
  } while (0)

hipError_t launch_fast_logits(const void *prepared, int precision, bool split, float margin,
                              const float *sten, int64_t n, float *z, uint8_t *masks,
                              hipStream_t s) {
  if (n == 0) return hipSuccess;
  Line1D ln{};
  const unsigned grid = grid_for((n + 63) / 64);
  N6_SCALAR(precision, split, dim3(grid), dim3(TPB), 0, s, 2, ln, prepared, margin, sten, n, 1, 0,
            nullptr, nullptr, masks, z);
  return hipGetLastError();
}

hipError_t launch_fast_reconstruct(const void *prepared, int precision, bool split, float margin,
                                   const float *f, int64_t n_faces, int sign, int selector,
                                   const uint8_t *masks_in, float *fhat, uint8_t *masks_out,
                                   hipStream_t s) {
  if (n_faces == 0) return hipSuccess;
  Line1D ln{};
  const unsigned grid = grid_for((n_faces + 63) / 64);
  N6_SCALAR(precision, split, dim3(grid), dim3(TPB), 0, s, 0, ln, prepared, margin, f, n_faces,
            sign, selector, masks_in, fhat, masks_out, nullptr);
  return hipGetLastError();
}

// 2D sweep: the fused face kernel in the tuned shape (four or eight waves),
// or the selector-only instantiation.
hipError_t launch_faces2d_kernel(const FaceLaunch &L, const FastArgs &fa, hipStream_t s,
                                 const Grid2D &g, int dir, const float *q, const uint8_t *mi,
                                 float *F, uint8_t *m) {
#define N6_FACES(P, W, SPLIT)                                                                 \
  hipLaunchKernelGGL((k_fast_faces<P, W, true, SPLIT>), dim3(L.grid), dim3(W * 64), 0, s, g,   \
                     dir, fa.selector, fa.prepared, fa.margin, q, mi, F, m, nrc, L.xcd)
  // re-check counters of this sweep (diagnostic), only while a margin is set
  u32 *nrc = fa.margin > 0.f && fa.scr.qcount ? fa.scr.qcount + 8 * dir : nullptr;
  if (fa.selector != 0) {  // the other selectors: no classifier, one instantiation
    hipLaunchKernelGGL((k_fast_faces<2, 4, false, false>), dim3(L.grid), dim3(256), 0, s, g, dir,
                       fa.selector, fa.prepared, fa.margin, q, mi, F, m, nullptr, L.xcd);
    return hipGetLastError();
  }
  if (fa.precision == 2) {
    if (L.waves == 8) N6_FACES(2, 8, false);
    else N6_FACES(2, 4, false);
  } else if (fa.split) {
    if (L.waves == 8) N6_FACES(3, 8, true);
    else N6_FACES(3, 4, true);
  } else {
    if (L.waves == 8) N6_FACES(3, 8, false);
    else N6_FACES(3, 4, false);
  }
#undef N6_FACES
  return hipGetLastError();
}

hipError_t launch_fast_pass1d(const Line1D &ln, const FastArgs &fa, const float *q,
                              const uint8_t *masks_in, const Out1D &out, hipStream_t s) {
  const int64_t tf = ln.faces();
  const unsigned grid = grid_for((tf + 63) / 64);
  if (fa.equation == 0 || fa.equation == 1) {  // scalar laws: face fluxes, re-check in place
    if (out.mode != OUT_FACES) return hipErrorInvalidValue;
    if (fa.equation == 0) {
      N6_SCALAR(fa.precision, fa.split, dim3(grid), dim3(TPB), 0, s, 1, ln, fa.prepared, fa.margin,
                q, tf, 1, fa.selector, masks_in, out.dst, out.masks, nullptr);
    } else if (fa.precision == 2) {
      hipLaunchKernelGGL((k_fast_burgers<2, false>), dim3(grid), dim3(TPB), 0, s, ln, fa.prepared,
                         fa.margin, fa.selector, q, masks_in, out.dst, out.masks);
    } else if (fa.split) {
      hipLaunchKernelGGL((k_fast_burgers<3, true>), dim3(grid), dim3(TPB), 0, s, ln, fa.prepared,
                         fa.margin, fa.selector, q, masks_in, out.dst, out.masks);
    } else {
      hipLaunchKernelGGL((k_fast_burgers<3, false>), dim3(grid), dim3(TPB), 0, s, ln, fa.prepared,
                         fa.margin, fa.selector, q, masks_in, out.dst, out.masks);
    }
    return hipGetLastError();
  }
  const FaceLaunch L = face_launch(fa, (tf + 61) / 63);
#define N6_EULER1D(P, W, MLP, SPLIT)                                                           \
  hipLaunchKernelGGL((k_euler1d<P, W, MLP, SPLIT>), dim3(L.grid), dim3(W * 64), 0, s, ln,        \
                     fa.selector, fa.prepared, fa.margin, q, masks_in, out, L.xcd)
  if (fa.selector != 0) {
    N6_EULER1D(2, 4, false, false);
  } else if (fa.precision == 2) {
    if (L.waves == 2) N6_EULER1D(2, 2, true, false);
    else if (L.waves == 8) N6_EULER1D(2, 8, true, false);
    else N6_EULER1D(2, 4, true, false);
  } else if (fa.split) {
    if (L.waves == 2) N6_EULER1D(3, 2, true, true);
    else if (L.waves == 8) N6_EULER1D(3, 8, true, true);
    else N6_EULER1D(3, 4, true, true);
  } else {
    if (L.waves == 2) N6_EULER1D(3, 2, true, false);
    else if (L.waves == 8) N6_EULER1D(3, 8, true, false);
    else N6_EULER1D(3, 4, true, false);
  }
#undef N6_EULER1D
  return hipGetLastError();
}

hipError_t launch_fast_reset(const FastArgs &fa, hipStream_t s) {
  if (!(fa.selector == 0 && fa.margin > 0.f) || !fa.scr.qcount) return hipSuccess;
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, fa.scr.qcount);
  return hipGetLastError();
}

hipError_t launch_fast_faces2d(const Grid2D &g, const FastArgs &fa, const float *q,
                               const uint8_t *masks_in, uint8_t *masks_out, float *Fx, float *Gy,
                               hipStream_t s) {
  const int64_t nfx = (g.nx + 1) * g.ny, nfy = g.nx * (g.ny + 1);
  uint8_t *masks = fa.scr.masks;  // both sweeps' labels (copied out if asked for)
  const bool recheck = fa.selector == 0 && fa.margin > 0.f;
  for (int dir = 0; dir < 2; ++dir) {
    const int64_t nf = dir == 0 ? nfx : nfy;
    uint8_t *md = masks + (dir == 0 ? 0 : 4 * nfx);
    const uint8_t *mi = masks_in ? masks_in + (dir == 0 ? 0 : 4 * nfx) : nullptr;
    float *Fd = dir == 0 ? Fx : Gy;
    u32 *qc = fa.scr.qcount + 8 * dir;  // eight counters (kinds) per sweep direction
    const FaceLaunch L = face_launch(fa, (nf + 63) / 64);
    hipError_t e = launch_faces2d_kernel(L, fa, s, g, dir, q, mi, Fd, md);
    if (e != hipSuccess) return e;
  }
  if (masks_out) return copy_bytes(masks, masks_out, 4 * (nfx + nfy), s);
  return hipSuccess;
}

hipError_t launch_fast_rhs2d(const Grid2D &g, const FastArgs &fa, const float *q, float *rhs,
                             const uint8_t *masks_in, uint8_t *masks_out, int32_t *status,
                             float *Fx, float *Gy, const Stage *st, hipStream_t s) {
  hipError_t e = launch_fast_faces2d(g, fa, q, masks_in, masks_out, Fx, Gy, s);
  if (e != hipSuccess) return e;
  return launch_diff2d<float>(g, Fx, Gy, q, rhs, st, status, s, fa.scr.qcount);
}

}  // namespace n6
