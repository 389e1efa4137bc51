// block_codec.hpp -- per-block ZFP fixed-rate coding, one block per lane.
//
// Everything here works on one 4x4x4 block held in registers of a single
// lane: block exponent, block-floating-point cast, separable integer lifting,
// sequency reordering, negabinary conversion, a 64x32 bit-matrix transpose
// into bit planes, and the embedded bit-plane coder/decoder cut at the fixed
// budget of 64*rate bits (the paper's Section II-C: independent 4^3 blocks,
// lifting transform, precision reduction, exactly r bits per value; the
// in-block steps as in ZFP's published algorithm description).
//
// Stream layout of one block (64*rate bits, least significant bit first in
// little-endian 64-bit words):
//   bit 0        1 if the block has a nonzero value, else 0 and the rest is 0
//   bits 1..8    emax + 127, emax = largest exponent e with |v| = f 2^e,
//                f in [1/2,1) (values below 2^-126 count as e = -126)
//   then, planes 31..0 of the negabinary coefficients in sequency order:
//   the first n bits verbatim, then group tests and unary scans that make
//   further coefficients significant; the last position is implied when a
//   scan reaches it; when the budget runs out the rest is zero.
//
// Variable-size modes (fixed precision, fixed accuracy) run the same coder
// but stop after the bit planes 31 .. 32 - p, p = min(maxprec, max(0,
// emax - minexp + 2 (d + 1))) with d = 3 (ZFP's rule for its precision and
// accuracy modes, which the paper names as the variable-size alternative);
// p = 0 makes the block the single bit 0.  The defaults of maxprec and minexp
// give p = 32 for every float block, which is fixed rate.
//
// The functions are __host__ __device__ so that the same logic can be built
// for the CPU when debugging; the library itself only runs them on the GPU.
#pragma once

#include <stdint.h>

#if defined(__HIP_DEVICE_COMPILE__)
#define ZFPX_HD __host__ __device__ __attribute__((always_inline)) inline
#elif defined(__HIPCC__)
#define ZFPX_HD __host__ __device__ inline
#else
#define ZFPX_HD inline
#endif

namespace zfpx {

constexpr uint32_t kNegabinaryMask = 0xaaaaaaaau;
constexpr int kMinExpNone = -1074;  // no exponent floor: every block keeps maxprec planes

// Bit planes coded for a block with exponent emax.
ZFPX_HD int block_precision(int emax, int maxprec, int minexp) {
  const int p = emax - minexp + 8;
  return p < 0 ? 0 : (p > maxprec ? maxprec : p);
}

// ---------------------------------------------------------------------------
// Sequency order, computed at compile time by sorting the 64 block-local
// indices i = 16 z + 4 y + x on the key (x+y+z, x^2+y^2+z^2, i).
// ---------------------------------------------------------------------------
struct SeqOrder {
  int8_t idx[64];  // idx[s] = block-local index at sequency position s
};

constexpr int seq_key(int i) {
  int x = i & 3, y = (i >> 2) & 3, z = i >> 4;
  return ((x + y + z) * 64 + (x * x + y * y + z * z)) * 64 + i;
}

constexpr SeqOrder make_seq_order() {
  SeqOrder o{};
  int a[64] = {};
  for (int i = 0; i < 64; i++) a[i] = i;
  for (int i = 1; i < 64; i++) {  // insertion sort
    int v = a[i], j = i - 1;
    while (j >= 0 && seq_key(a[j]) > seq_key(v)) {
      a[j + 1] = a[j];
      j--;
    }
    a[j + 1] = v;
  }
  for (int i = 0; i < 64; i++) o.idx[i] = (int8_t)a[i];
  return o;
}

constexpr SeqOrder kSeq = make_seq_order();

// ---------------------------------------------------------------------------
// Scalar helpers
// ---------------------------------------------------------------------------
ZFPX_HD uint32_t f32_bits(float f) { return __builtin_bit_cast(uint32_t, f); }

ZFPX_HD float scale_pow2(float f, int e) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_ldexpf(f, e);
#else
  return __builtin_ldexpf(f, e);
#endif
}

ZFPX_HD uint64_t low_mask(int n) {  // n in [0, 64]
  return n >= 64 ? ~uint64_t(0) : ((uint64_t(1) << n) - 1);
}

// low_mask(n) for n in [1, 64] without a select: 2 << 63 wraps to 0.
ZFPX_HD uint64_t mask_upto(int n) { return ((uint64_t)2 << (n - 1)) - 1; }

ZFPX_HD int ctz64(uint64_t x) {  // x != 0
  return __builtin_ctzll(x);
}

// ---------------------------------------------------------------------------
// Lifting (wrapping int32 arithmetic, arithmetic shifts)
// ---------------------------------------------------------------------------
ZFPX_HD void lift_fwd(int32_t& x0, int32_t& x1, int32_t& x2, int32_t& x3) {
  // done in uint32 so that wrap-around is defined; >> on int32 is arithmetic
  auto add = [](int32_t a, int32_t b) { return (int32_t)((uint32_t)a + (uint32_t)b); };
  auto sub = [](int32_t a, int32_t b) { return (int32_t)((uint32_t)a - (uint32_t)b); };
  x0 = add(x0, x3) >> 1; x3 = sub(x3, x0);
  x2 = add(x2, x1) >> 1; x1 = sub(x1, x2);
  x0 = add(x0, x2) >> 1; x2 = sub(x2, x0);
  x3 = add(x3, x1) >> 1; x1 = sub(x1, x3);
  x3 = add(x3, x1 >> 1); x1 = sub(x1, x3 >> 1);
}

ZFPX_HD void lift_inv(int32_t& x0, int32_t& x1, int32_t& x2, int32_t& x3) {
  auto add = [](int32_t a, int32_t b) { return (int32_t)((uint32_t)a + (uint32_t)b); };
  auto sub = [](int32_t a, int32_t b) { return (int32_t)((uint32_t)a - (uint32_t)b); };
  // The steps "a += b; b = 2b - a" leave b = 2b - (a + b) = b - a (mod 2^32):
  // two operations instead of three.
  auto step = [&](int32_t& a, int32_t& b) {
    const int32_t a0 = a;
    a = add(a0, b);
    b = sub(b, a0);
  };
  x1 = add(x1, x3 >> 1); x3 = sub(x3, x1 >> 1);
  step(x1, x3);
  step(x2, x0);
  step(x1, x2);
  step(x3, x0);
}

// Forward 3-D transform of q[16 z + 4 y + x]: x-lines, y-lines, z-lines.
ZFPX_HD void xform_fwd(int32_t* q) {
#pragma unroll
  for (int zy = 0; zy < 16; zy++) lift_fwd(q[4 * zy], q[4 * zy + 1], q[4 * zy + 2], q[4 * zy + 3]);
#pragma unroll
  for (int z = 0; z < 4; z++)
#pragma unroll
    for (int x = 0; x < 4; x++)
      lift_fwd(q[16 * z + x], q[16 * z + 4 + x], q[16 * z + 8 + x], q[16 * z + 12 + x]);
#pragma unroll
  for (int yx = 0; yx < 16; yx++) lift_fwd(q[yx], q[16 + yx], q[32 + yx], q[48 + yx]);
}

// Inverse: z-lines, y-lines, x-lines.
ZFPX_HD void xform_inv(int32_t* q) {
#pragma unroll
  for (int yx = 0; yx < 16; yx++) lift_inv(q[yx], q[16 + yx], q[32 + yx], q[48 + yx]);
#pragma unroll
  for (int z = 0; z < 4; z++)
#pragma unroll
    for (int x = 0; x < 4; x++)
      lift_inv(q[16 * z + x], q[16 * z + 4 + x], q[16 * z + 8 + x], q[16 * z + 12 + x]);
#pragma unroll
  for (int zy = 0; zy < 16; zy++) lift_inv(q[4 * zy], q[4 * zy + 1], q[4 * zy + 2], q[4 * zy + 3]);
}

// ---------------------------------------------------------------------------
// Bit transpose
// ---------------------------------------------------------------------------

// Two independent 32x32 transposes at once on 64-bit words: a[r] holds row r
// of the first matrix in its low half and of the second in its high half;
// afterwards a[r] low/high bit c = old a[c] low/high bit r.  The classic
// five-stage block-swap transpose: stage J swaps, between rows r and r+J
// (r & J == 0), the bits whose column has bit J set in row r with the bits
// whose column has it clear in row r+J.  Stages 16 and 8 move whole bytes
// (one byte permute per output half); stages 4, 2, 1 are a shift and a
// bit-field select per output half.

// Byte permute: result byte i = byte sel_i of (hi:lo), bytes 0-3 from lo.
ZFPX_HD uint32_t byte_perm(uint32_t hi, uint32_t lo, uint32_t sel) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_perm(hi, lo, sel);
#else
  uint64_t x = ((uint64_t)hi << 32) | lo;
  uint32_t r = 0;
  for (int i = 0; i < 4; i++) r |= (uint32_t)((x >> (8 * ((sel >> (8 * i)) & 7))) & 0xff) << (8 * i);
  return r;
#endif
}

template <int J>
ZFPX_HD void transpose_bytes64(uint64_t* a) {
  // J = 16: new a = [a.b0 a.b1 b.b0 b.b1], new b = [a.b2 a.b3 b.b2 b.b3]
  // J = 8 : new a = [a.b0 b.b0 a.b2 b.b2], new b = [a.b1 b.b1 a.b3 b.b3]
  constexpr uint32_t sa = J == 16 ? 0x05040100u : 0x06020400u;
  constexpr uint32_t sb = J == 16 ? 0x07060302u : 0x07030501u;
#pragma unroll
  for (int r = 0; r < 32; r++) {
    if ((r & J) == 0) {
      uint32_t alo = (uint32_t)a[r], ahi = (uint32_t)(a[r] >> 32);
      uint32_t blo = (uint32_t)a[r + J], bhi = (uint32_t)(a[r + J] >> 32);
      a[r] = byte_perm(blo, alo, sa) | ((uint64_t)byte_perm(bhi, ahi, sa) << 32);
      a[r + J] = byte_perm(blo, alo, sb) | ((uint64_t)byte_perm(bhi, ahi, sb) << 32);
    }
  }
}

// Bit select: (a & m) | (b & ~m), one three-input logic instruction; INV
// returns its complement, still one instruction.
template <bool INV = false>
ZFPX_HD uint32_t bit_select(uint32_t m, uint32_t a, uint32_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_bitop3_b32(m, a, b, INV ? 0x35 : 0xCA);
#else
  return INV ? ~((a & m) | (b & ~m)) : (a & m) | (b & ~m);
#endif
}

// Any three-input bitwise function in one instruction: bit i of TT is the
// result for the inputs (s0, s1, s2) = (bit 2, bit 1, bit 0 of i).
template <uint32_t TT>
ZFPX_HD uint32_t bitop3(uint32_t s0, uint32_t s1, uint32_t s2) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_bitop3_b32(s0, s1, s2, TT);
#else
  uint32_t r = 0;
  for (int i = 0; i < 8; i++)
    if ((TT >> i) & 1) r |= ((i & 4) ? s0 : ~s0) & ((i & 2) ? s1 : ~s1) & ((i & 1) ? s2 : ~s2);
  return r;
#endif
}

// INV_HI complements the rows r + J written by the stage (the odd rows when
// J = 1), at no cost.
template <int J, uint32_t MASK, bool INV_HI = false>
ZFPX_HD void transpose_bits64(uint64_t* a) {
  // Each half is shifted on its own: the bits a 64-bit shift would carry
  // across the halves land where the select mask discards them.
  constexpr uint32_t HM = MASK << J;
#pragma unroll
  for (int r = 0; r < 32; r++) {
    if ((r & J) == 0) {
      uint32_t xl = (uint32_t)a[r], xh = (uint32_t)(a[r] >> 32);
      uint32_t yl = (uint32_t)a[r + J], yh = (uint32_t)(a[r + J] >> 32);
      a[r + J] = (uint64_t)bit_select<INV_HI>(MASK, xl >> J, yl) |
                 ((uint64_t)bit_select<INV_HI>(MASK, xh >> J, yh) << 32);
      a[r] = (uint64_t)bit_select(HM, yl << J, xl) | ((uint64_t)bit_select(HM, yh << J, xh) << 32);
    }
  }
}

// The J = 1 stage reading the odd rows complemented (the input rows r + 1),
// at no cost: each output is one three-input function of the two rows.
ZFPX_HD void transpose_bits64_odd_in_inverted(uint64_t* a) {
  constexpr uint32_t M = 0x55555555u, HM = M << 1;
#pragma unroll
  for (int r = 0; r < 32; r += 2) {
    uint32_t xl = (uint32_t)a[r], xh = (uint32_t)(a[r] >> 32);
    uint32_t yl = (uint32_t)a[r + 1], yh = (uint32_t)(a[r + 1] >> 32);
    // odd row: (M & x >> 1) | (~M & ~y); even row: (HM & ~(y << 1)) | (~HM & x)
    a[r + 1] = (uint64_t)bitop3<0xC5>(M, xl >> 1, yl) | ((uint64_t)bitop3<0xC5>(M, xh >> 1, yh) << 32);
    a[r] = (uint64_t)bitop3<0x3A>(HM, yl << 1, xl) | ((uint64_t)bitop3<0x3A>(HM, yh << 1, xh) << 32);
  }
}

// Each stage swaps one bit of the row index with the same bit of the column
// index; the stages commute, so any order gives the transpose.
// INVERT_ODD: afterwards rows 1, 3, ..., 31 are complemented.  XOR with a
// constant commutes with the transpose, so the encoder's negabinary XOR with
// 0xaaaaaaaa (bits 1, 3, ..., 31 of every coefficient) becomes exactly this.
template <bool INVERT_ODD = false>
ZFPX_HD void transpose32x2(uint64_t* a) {
  transpose_bytes64<16>(a);
  transpose_bytes64<8>(a);
  transpose_bits64<4, 0x0f0f0f0fu>(a);
  transpose_bits64<2, 0x33333333u>(a);
  transpose_bits64<1, 0x55555555u, INVERT_ODD>(a);
}

// The transpose of rows 1, 3, ..., 31 complemented (the J = 1 stage first,
// reading them inverted): for the decoder, whose odd bit planes are the
// complemented ones (the negabinary XOR with 0xaaaaaaaa seen plane-wise).
ZFPX_HD void transpose32x2_odd_in_inverted(uint64_t* a) {
  transpose_bits64_odd_in_inverted(a);
  transpose_bits64<2, 0x33333333u>(a);
  transpose_bits64<4, 0x0f0f0f0fu>(a);
  transpose_bytes64<8>(a);
  transpose_bytes64<16>(a);
}

// ---------------------------------------------------------------------------
// Coded-stream access in LDS
// ---------------------------------------------------------------------------
// Each lane owns a slice of LDS words for its block: `rate` words of stream
// followed by slack words that are always zero, so that windows and writes
// that run past the budget stay inside the slice.

constexpr int kSlackWords = 2;

// OR the (up to 64-bit) value `code` into the slice at bit position `pos`.
// The word index of bit position pos, kept opaque so that the address
// becomes one shift-add of it (not a shift, a mask and an add).
ZFPX_HD uint32_t word_of(uint32_t pos) {
  uint32_t w = pos >> 6;
#if defined(__HIP_DEVICE_COMPILE__)
  asm("" : "+v"(w));
#endif
  return w;
}

ZFPX_HD void or_bits(uint64_t* s, uint32_t pos, uint64_t code) {
  uint32_t w = word_of(pos), b = pos & 63;
  uint64_t lo = code << b;
  uint64_t hi = (code >> 1) >> (63 - b);
#if defined(__HIP_DEVICE_COMPILE__)
  __hip_atomic_fetch_or(s + w, lo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
  __hip_atomic_fetch_or(s + w + 1, hi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
#else
  s[w] |= lo;
  s[w + 1] |= hi;
#endif
}

// The 64 stream bits starting at bit position `pos`.
// Read as 32-bit words (the low word of each 64-bit word first): three words
// from word pos / 32 hold the window, and two funnel shifts by pos % 32 (which
// the instruction takes from the low 5 bits of its count) assemble it.
typedef uint32_t __attribute__((may_alias)) u32_alias;
ZFPX_HD uint32_t funnel32(uint32_t hi, uint32_t lo, uint32_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_alignbit(hi, lo, b);
#else
  return (uint32_t)((((uint64_t)hi << 32) | lo) >> (b & 31));
#endif
}
// The 32-bit word index of bit position pos, opaque as word_of.
ZFPX_HD uint32_t word32_of(uint32_t pos) {
  uint32_t w = pos >> 5;
#if defined(__HIP_DEVICE_COMPILE__)
  asm("" : "+v"(w));
#endif
  return w;
}
ZFPX_HD uint64_t window64(const uint64_t* s, uint32_t pos) {
  const u32_alias* d = reinterpret_cast<const u32_alias*>(s) + word32_of(pos);
  const uint32_t d0 = d[0], d1 = d[1], d2 = d[2];
  return (uint64_t)funnel32(d1, d0, pos) | ((uint64_t)funnel32(d2, d1, pos) << 32);
}

// The three 32-bit words that hold the window at pos, and the window itself.
struct Words3 {
  uint32_t w0, w1, w2;
};
ZFPX_HD Words3 window_words(const uint64_t* s, uint32_t pos) {
  const u32_alias* d = reinterpret_cast<const u32_alias*>(s) + word32_of(pos);
  return Words3{d[0], d[1], d[2]};
}
ZFPX_HD uint64_t window_of(const Words3& w, uint32_t pos) {
  return (uint64_t)funnel32(w.w1, w.w0, pos) | ((uint64_t)funnel32(w.w2, w.w1, pos) << 32);
}

// Make the words of two windows available at this point (an empty asm that
// reads and writes all six): the six reads are issued first and waited for
// together, one LDS round trip for both windows.
ZFPX_HD void pin_words(Words3& a, Words3& b) {
#if defined(__HIP_DEVICE_COMPILE__)
  asm volatile("" : "+v"(a.w0), "+v"(a.w1), "+v"(a.w2), "+v"(b.w0), "+v"(b.w1), "+v"(b.w2));
#else
  (void)a;
  (void)b;
#endif
}
ZFPX_HD void pin_words(Words3& a) {
#if defined(__HIP_DEVICE_COMPILE__)
  asm volatile("" : "+v"(a.w0), "+v"(a.w1), "+v"(a.w2));
#else
  (void)a;
#endif
}

// ---------------------------------------------------------------------------
// Encoder
// ---------------------------------------------------------------------------

// Encode one block of 64 floats (v[16 z + 4 y + x]) into the slice `out`,
// which must hold rate + kSlackWords zero words.  Bits are ORed in place;
// the slack words may receive bits past the budget and are not part of the
// stream.  v is clobbered.  Returns the block's length in bits (at most
// 64 * rate; 1 for a block coded as the single bit 0).
template <int RATE>
ZFPX_HD uint32_t encode_block(float* v, uint64_t* out, int rate_rt, int maxprec = 32,
                              int minexp = kMinExpNone) {
  const int rate = RATE > 0 ? RATE : rate_rt;
  const uint32_t maxbits = 64u * (uint32_t)rate;
  // block exponent from the largest magnitude (its biased exponent field)
  float amax = 0.0f;
#pragma unroll
  for (int i = 0; i < 64; i++) amax = __builtin_fmaxf(amax, __builtin_fabsf(v[i]));
  uint32_t mx = f32_bits(amax);
  if (mx == 0) return 1;  // empty block: the single bit 0, all zero
  int emax = (int)(mx >> 23) - 126;  // subnormal maximum (field 0) gives -126
  const int kmin = 32 - block_precision(emax, maxprec, minexp);
  if (kmin == 32) return 1;  // no plane to code: the single bit 0
  or_bits(out, 0, 1u | ((uint64_t)((emax + 127) & 0xff) << 1));
  // X[s] = coefficients s and 32+s (negabinary); after the transpose X[k] is
  // bit plane k: bit s of X[k] = bit k of coefficient s
  uint64_t X[32];
  {
    int32_t q[64];
    if (emax >= -97) {
      // 2^(30 - emax) is a normal float: one multiply per value is the same
      // exact scaling (a product below 1 in magnitude truncates to 0 whatever
      // its rounding)
      const float sc = scale_pow2(1.0f, 30 - emax);
#pragma unroll
      for (int i = 0; i < 64; i++) q[i] = (int32_t)(v[i] * sc);
    } else {
#pragma unroll
      for (int i = 0; i < 64; i++) q[i] = (int32_t)scale_pow2(v[i], 30 - emax);
    }
    xform_fwd(q);
    // negabinary (q + mask) ^ mask: the add here, the XOR in the transpose
#pragma unroll
    for (int s = 0; s < 32; s++) {
      uint32_t lo = (uint32_t)q[kSeq.idx[s]] + kNegabinaryMask;
      uint32_t hi = (uint32_t)q[kSeq.idx[32 + s]] + kNegabinaryMask;
      X[s] = (uint64_t)lo | ((uint64_t)hi << 32);
    }
  }
  static_assert(kNegabinaryMask == 0xaaaaaaaau, "the transpose complements the odd planes");
  transpose32x2<true>(X);
  uint32_t pos = 9;
  int n = 0;
  uint64_t vm = 0;  // low_mask(n), updated only when n changes
#pragma unroll
  for (int k = 31; k >= 0; k--) {
    if (pos < maxbits && k >= kmin) {
      const uint64_t x = X[k];
      or_bits(out, pos, x & vm);  // the first n bits verbatim
      pos += n;
      // a bit at or above n (vm = 2^n - 1 with every bit below n set)
      if (x > vm && pos < maxbits) {
        uint64_t y = x >> n;  // bits not yet significant (n < 64 here)
        // Each newly significant coefficient costs a group test 1, the zeros
        // up to it and its own 1 (that one is implied, and not written, for
        // coefficient 63).
        bool done = false;
        // Common case: all of the plane's groups fit one 64-bit code word and
        // none reaches coefficient 63.  With the newly significant
        // coefficients at positions q_0 < ... < q_(m-1) of y, the word has a
        // group test 1 at bit 0 and, for each i, the coefficient's one at bit
        // q_i + i + 1, followed (unless i is the last) by the next group test
        // 1 at bit q_i + i + 2.  sp = sum_i 2^(q_i + i) (each one of y moved
        // up by the number of ones below it) is built by adding, for t = 0,
        // 1, ..., y without its lowest t + 1 ones shifted up by t.  The word
        // is then written at once; groups that start past the budget only
        // land in the slack words, and the budget is spent either way, so the
        // coded bits are those of the group-by-group loop below.
        const int hy = 63 - __builtin_clzll(y);           // q_(m-1)
        const int hs = hy + __builtin_popcountll(y) - 1;  // its bit in sp
        if (hs <= 62 && n + hy <= 62) {
          uint64_t sp = y, e = y;
          for (int t = 0;; t++) {
            e &= e - 1;
            if (e == 0) break;
            sp += e << t;
          }
          // the three parts share no bit, so adds join them (shift-adds)
          const uint64_t code = ((sp ^ (uint64_t(1) << hs)) << 2) + ((sp << 1) + 1);
          or_bits(out, pos, code);
          pos += (uint32_t)hs + 2;
          n += hy + 1;
          done = true;
        }
        while (!done && y != 0 && pos < maxbits) {
          int p = ctz64(y);
          int last = (n + p == 63);
          uint64_t g = last ? uint64_t(1) : (uint64_t(1) | (uint64_t(2) << p));
          or_bits(out, pos, g);
          pos += p + 2 - last;
          n += p + 1;
          y = (y >> p) >> 1;
        }
        vm = mask_upto(n);
      }
      pos += n < 64 ? 1 : 0;  // group test 0 (a zero bit)
    }
  }
  return pos < maxbits ? pos : maxbits;
}

// ---------------------------------------------------------------------------
// Decoder
// ---------------------------------------------------------------------------

// Population count of a 64-bit word.
ZFPX_HD int popc64(uint64_t x) { return __builtin_popcountll(x); }

// The group tests and scans that follow a group test of 1, parsed from the
// 64 stream bits v after it (bit 0 first), without a loop over the groups.
// Each group is zeros up to a one (the newly significant coefficient), and
// the group test after it is 1 if another group follows: so inside every
// maximal run of ones that starts right after a zero (or at bit 0) the bits
// alternate coefficient-one, group-test, coefficient-one, ...; a run that
// ends on a coefficient-one is followed by the closing group test 0.
// Returns the window position p of that last coefficient-one (64 if the
// window holds none) and, through ev, the coefficient-ones at positions
// 0..p.
ZFPX_HD int parse_groups(uint64_t v, uint64_t& ev) {
  constexpr uint64_t kEven = 0x5555555555555555ull;
  const uint64_t starts = v & ~(v << 1);
  // runs that start at an even position turn to zeros when their start bit
  // is added (the carry runs through them); the others are unchanged
  const uint64_t t = v + (starts & kEven);
  // coefficient-ones: even positions of even-started runs, odd positions of
  // odd-started runs
  const uint64_t e = v & (t ^ kEven);
  const uint64_t ends = e & ~(v >> 1);
  if (ends == 0) {
    ev = 0;
    return 64;
  }
  const int p = ctz64(ends);
  ev = e & (((uint64_t)2 << p) - 1);  // p <= 63: 2 << 63 wraps to 0, mask all ones
  return p;
}

// Decode the slice `in` (rate words followed by kSlackWords zero words) into
// 64 floats (block-local order).
//
// Stream positions never pass maxbits (reads there return the zero slack,
// which is what a budget that has run out yields for verbatim bits and group
// tests).  Per bit plane: the verbatim bits are the window at pos masked to
// the n significant coefficients, and the group test is bit n of the same
// window; a plane whose group test is 0 (most of them) is done with that.
// Otherwise the groups are parsed from the window after the group test
// (parse_groups), unless the budget ends inside them or a scan could reach
// coefficient 63 (whose one is implied, not coded): those take the
// group-by-group loop.
// TINY_SINGLE selects how results that may be subnormal (blocks with
// emax < -95) are rounded: in single precision only, or from a double
// product.  Both round once and agree bit for bit.  The choice changes how
// the compiler lays out the whole decoder, not only that rare path: measured
// on the 9.47 GB buffer, the variable-size decoder runs 6% faster with the
// single-precision form and the fixed-rate decoders about 1% slower.
template <int RATE, bool TINY_SINGLE = false>
ZFPX_HD void decode_block(const uint64_t* in, float* vout, int rate_rt, int maxprec = 32,
                          int minexp = kMinExpNone) {
  const int rate = RATE > 0 ? RATE : rate_rt;
  const uint32_t maxbits = 64u * (uint32_t)rate;
  // the header (bits 0..8) and the first plane's window (from bit 9) are in
  // the first three words: one round trip
  Words3 wfirst = window_words(in, 0);
  pin_words(wfirst);
  const uint32_t head = wfirst.w0;
  uint32_t pos = maxbits;  // an empty block decodes to zeros
  int emax = 0, kmin = 0;
  if (head & 1) {
    emax = (int)((head >> 1) & 0xff) - 127;
    pos = 9;
    kmin = 32 - block_precision(emax, maxprec, minexp);
  }
  uint64_t X[32];  // bit planes, then (after the transpose) coefficients s, 32+s
  int n = 0;
  uint64_t vm = 0;  // low_mask(n)
#pragma unroll
  for (int k = 31; k >= 0; k--) {
    uint64_t x = 0;
    if (k >= kmin && pos < maxbits) {
      const uint64_t w = k == 31 ? window_of(wfirst, pos) : window64(in, pos);
      x = w & vm;  // verbatim bits (zeros past the budget)
      const uint32_t gpos = pos + (uint32_t)n;
      const bool group = n < 64 && ((w >> (n & 63)) & 1) && gpos < maxbits;
      pos = gpos + (n < 64 ? 1u : 0u);
      if (group) {
        // pos is the bit after the group test of 1
        uint64_t ev;
        const int p = parse_groups(window64(in, pos), ev);
        const int m = popc64(ev);
        const int last = n + p + 1 - m;  // coefficient of the last one found
        // The whole run can be read off the window unless it reaches past
        // it, past the budget, or up to the implied coefficient 63; then it
        // is taken group by group (the second stage runs no step when the
        // first applied: one stage after the other, not alternatives, keeps
        // the compiler from carrying this block's planes through a loop
        // around the decoder in extra registers).
        const bool whole = p < 63 && pos + (uint32_t)p < maxbits && last <= 62;
        if (whole) {
          // each coefficient-one moves down by the number of group tests
          // before it: y = ev - sum_t (ev without its lowest t ones) >> t
          uint64_t y = ev, e = ev;
          for (int t = 1;; t++) {
            e &= e - 1;
            if (e == 0) break;
            y -= e >> t;
          }
          x |= y << n;
          n = last + 1;
          pos += (uint32_t)p + 2;  // through the closing group test 0
        }
        // group by group: zeros up to the next one, at most up to
        // coefficient 63 (implied) or the end of the budget
        int g = whole ? 0 : 1;
        while (g) {
          int lim = 63 - n;
          if ((int)(maxbits - pos) < lim) lim = (int)(maxbits - pos);
          const uint64_t s = window64(in, pos);
          const int z = s ? ctz64(s) : 64;
          const int t = z < lim ? z : lim;
          const int found = z < lim;
          x |= uint64_t(1) << (n + t);
          n += t + 1;
          pos += (uint32_t)(t + found);
          g = 0;
          if (n < 64 && pos < maxbits) {
            g = (int)((s >> (t + found)) & 1);  // t + found <= 63
            pos += 1;
          }
        }
        vm = mask_upto(n);  // n >= 1 after a group test of 1
      }
      if (pos > maxbits) pos = maxbits;
    }
    X[k] = x;
  }
  // odd planes complemented as the transpose reads them: every coefficient
  // comes out XORed with the negabinary mask 0xaaaaaaaa (bits 1, 3, ..., 31)
  transpose32x2_odd_in_inverted(X);
  int32_t q[64];
#pragma unroll
  for (int s = 0; s < 32; s++) {
    // negabinary to two's complement: (u ^ mask) - mask, the XOR done above
    q[kSeq.idx[s]] = (int32_t)((uint32_t)X[s] - kNegabinaryMask);
    q[kSeq.idx[32 + s]] = (int32_t)((uint32_t)(X[s] >> 32) - kNegabinaryMask);
  }
  xform_inv(q);
  if (emax >= -95) {
    // float(q) is one rounding and the power-of-two scale is exact (normal
    // result); 2^(emax - 30) is a normal float, so a multiply applies it
    const float sc = scale_pow2(1.0f, emax - 30);
#pragma unroll
    for (int i = 0; i < 64; i++) vout[i] = (float)q[i] * sc;
  } else if (TINY_SINGLE) {
    // Results may be subnormal; each is still rounded once, in single
    // precision only.  With s = emax + 119 (in -7 .. 23),
    // q * 2^(emax - 30) = q * 2^s * 2^-149, and 2^-149 is float32's smallest
    // step.  A result of magnitude 2^-126 or more (|q| >= 2^(23 - s)) is
    // normal: float(q), one rounding, then two exact power-of-two scalings.
    // A smaller one is the integer nearest q * 2^s (ties to even; exact for
    // s >= 0) times 2^-149, which float32 holds exactly; its sign is q's,
    // zero included.
    const int s = emax + 119;
    const float up = scale_pow2(1.0f, emax + 34);  // 2^(emax - 30) = 2^-64 * up
#pragma unroll
    for (int i = 0; i < 64; i++) {
      const int32_t qi = q[i];
      const uint32_t mag = qi < 0 ? 0u - (uint32_t)qi : (uint32_t)qi;
      float r;
      if (mag >= (1u << (23 - s))) {
        r = ((float)qi * 0x1p-64f) * up;
      } else {
        int32_t m;
        if (s >= 0) {
          m = (int32_t)((uint32_t)qi << s);
        } else {
          const int k = -s;
          m = (qi + (1 << (k - 1)) - 1 + ((qi >> k) & 1)) >> k;  // |qi| < 2^30 here
        }
        r = __builtin_copysignf(((float)m * 0x1p-100f) * 0x1p-49f, qi < 0 ? -1.0f : 1.0f);
      }
      vout[i] = r;
    }
  } else {
    // results may be subnormal: round once from the exact double product
#pragma unroll
    for (int i = 0; i < 64; i++) vout[i] = (float)__builtin_ldexp((double)q[i], emax - 30);
  }
}

}  // namespace zfpx
