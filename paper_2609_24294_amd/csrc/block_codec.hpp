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
  auto dbl_sub = [](int32_t a, int32_t b) { return (int32_t)(((uint32_t)a << 1) - (uint32_t)b); };
  x1 = add(x1, x3 >> 1); x3 = (int32_t)((uint32_t)x3 - (uint32_t)(x1 >> 1));
  x1 = add(x1, x3); x3 = dbl_sub(x3, x1);
  x2 = add(x2, x0); x0 = dbl_sub(x0, x2);
  x1 = add(x1, x2); x2 = dbl_sub(x2, x1);
  x3 = add(x3, x0); x0 = dbl_sub(x0, x3);
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
// 32x32 bit-matrix transpose in place: afterwards a[r] bit c = old a[c] bit r.
// ---------------------------------------------------------------------------
template <int J, uint32_t MASK>
ZFPX_HD void transpose_stage(uint32_t* a) {
#pragma unroll
  for (int r = 0; r < 32; r++) {
    if ((r & J) == 0) {
      uint32_t t = ((a[r] >> J) ^ a[r + J]) & MASK;
      a[r + J] ^= t;
      a[r] ^= t << J;
    }
  }
}

ZFPX_HD void transpose32(uint32_t* a) {
  transpose_stage<16, 0x0000ffffu>(a);
  transpose_stage<8, 0x00ff00ffu>(a);
  transpose_stage<4, 0x0f0f0f0fu>(a);
  transpose_stage<2, 0x33333333u>(a);
  transpose_stage<1, 0x55555555u>(a);
}

// ---------------------------------------------------------------------------
// Encoder
// ---------------------------------------------------------------------------

// Bit writer: a 64-bit accumulator flushed word by word to `out`.
struct BitWriter {
  uint64_t acc;
  int na;  // bits held in acc, 0..63
  int wi;  // words written
  uint64_t* out;

  ZFPX_HD void put(uint64_t v, int l) {  // 0 <= l <= 64, v < 2^l
    acc |= v << na;
    int t = na + l;
    if (t >= 64) {
      out[wi++] = acc;
      acc = na ? (v >> (64 - na)) : 0;
      t -= 64;
    }
    na = t;
  }
};

// Encode one block of 64 floats (v[16 z + 4 y + x]) into exactly `rate`
// 64-bit words written to out[0..rate-1].  v is clobbered.
template <int RATE>
ZFPX_HD void encode_block(float* v, uint64_t* out, int rate_rt) {
  const int rate = RATE > 0 ? RATE : rate_rt;
  const int maxbits = 64 * rate;
  // block exponent: the largest biased exponent field over |v|
  uint32_t mx = 0;
#pragma unroll
  for (int i = 0; i < 64; i++) {
    uint32_t m = f32_bits(v[i]) & 0x7fffffffu;
    mx = m > mx ? m : mx;
  }
  BitWriter w{0, 0, 0, out};
  int bits;
  uint32_t pl[64];  // becomes the plane words: pl[k] low half, pl[32+k] high half
  if (mx == 0) {
    w.na = 1;  // single 0 bit
    bits = 0;
#pragma unroll
    for (int i = 0; i < 64; i++) pl[i] = 0;
  } else {
    int emax = (int)(mx >> 23) - 126;  // subnormal maximum (field 0) gives -126
    w.acc = 1u | ((uint64_t)((emax + 127) & 0xff) << 1);
    w.na = 9;
    bits = maxbits - 9;
    int32_t q[64];
#pragma unroll
    for (int i = 0; i < 64; i++) q[i] = (int32_t)scale_pow2(v[i], 30 - emax);
    xform_fwd(q);
#pragma unroll
    for (int s = 0; s < 64; s++)
      pl[s] = ((uint32_t)q[kSeq.idx[s]] + kNegabinaryMask) ^ kNegabinaryMask;
    transpose32(pl);
    transpose32(pl + 32);
  }
  int n = 0;
#pragma unroll
  for (int k = 31; k >= 0; k--) {
    if (bits > 0) {
      uint64_t x = (uint64_t)pl[k] | ((uint64_t)pl[32 + k] << 32);
      int m = n < bits ? n : bits;
      w.put(x & low_mask(m), m);
      bits -= m;
      uint64_t y = n < 64 ? (x >> n) : 0;
      while (n < 64 && bits > 0) {
        if (y == 0) {  // group test 0: nothing more in this plane
          w.put(0, 1);
          bits -= 1;
          break;
        }
        int p = ctz64(y);
        int last = (n + p == 63);  // the bit at position 63 is implied
        int len = p + 2 - last;
        uint64_t code = last ? uint64_t(1) : (uint64_t(1) | (uint64_t(2) << p));
        if (len > bits) {
          len = bits;
          code &= low_mask(len);
        }
        w.put(code, len);
        bits -= len;
        n += p + 1;
        y = (p >= 63) ? 0 : (y >> (p + 1));
      }
    }
  }
  if (w.na > 0) out[w.wi++] = w.acc;
  for (int i = w.wi; i < rate; i++) out[i] = 0;
}

// ---------------------------------------------------------------------------
// Decoder
// ---------------------------------------------------------------------------

// Bit reader over `rate` words with a 64..128-bit window (w0 = next 64 bits).
struct BitReader {
  uint64_t w0, w1;
  int v;   // valid bits in (w0, w1), kept >= 64
  int ri;  // next word to fetch
  int nw;  // words in the block
  const uint64_t* in;

  ZFPX_HD void init(const uint64_t* src, int words) {
    in = src;
    nw = words;
    w0 = src[0];
    w1 = words > 1 ? src[1] : 0;
    v = 128;
    ri = 2;
  }
  ZFPX_HD void consume(int l) {  // 0 <= l <= 64
    if (l == 0) return;
    if (l < 64) {
      w0 = (w0 >> l) | (w1 << (64 - l));
      w1 >>= l;
    } else {
      w0 = w1;
      w1 = 0;
    }
    v -= l;
    if (v < 64) {
      uint64_t nx = ri < nw ? in[ri] : 0;
      ri++;
      w0 |= nx << v;  // v in [0, 63]
      w1 = v ? (nx >> (64 - v)) : 0;
      v += 64;
    }
  }
};

// Decode `rate` words into 64 floats (block-local order).
template <int RATE>
ZFPX_HD void decode_block(const uint64_t* in, float* vout, int rate_rt) {
  const int rate = RATE > 0 ? RATE : rate_rt;
  const int maxbits = 64 * rate;
  BitReader r;
  r.init(in, rate);
  uint64_t head = r.w0;
  int bits = 0, emax = 0;
  if (head & 1) {
    emax = (int)((head >> 1) & 0xff) - 127;
    bits = maxbits - 9;
    r.consume(9);
  }
  uint32_t pl[64];
  int n = 0;
#pragma unroll
  for (int k = 31; k >= 0; k--) {
    uint64_t x = 0;
    if (bits > 0) {
      int m = n < bits ? n : bits;
      x = r.w0 & low_mask(m);
      r.consume(m);
      bits -= m;
      while (n < 64 && bits > 0) {
        uint64_t win = r.w0;
        bits -= 1;  // the group test
        if (!(win & 1)) {
          r.consume(1);
          break;
        }
        int lim = 63 - n < bits ? 63 - n : bits;
        uint64_t s = win >> 1;
        int z = s ? ctz64(s) : 64;
        int t = z < lim ? z : lim;
        int found = z < lim;
        r.consume(1 + t + found);
        bits -= t + found;
        n += t;
        x |= uint64_t(1) << n;
        n++;
      }
    }
    pl[k] = (uint32_t)x;
    pl[32 + k] = (uint32_t)(x >> 32);
  }
  transpose32(pl);
  transpose32(pl + 32);
  int32_t q[64];
#pragma unroll
  for (int s = 0; s < 64; s++)
    q[kSeq.idx[s]] = (int32_t)((pl[s] ^ kNegabinaryMask) - kNegabinaryMask);
  xform_inv(q);
  if (emax >= -95) {
    // float(q) is one rounding and the power-of-two scale is exact (normal result)
#pragma unroll
    for (int i = 0; i < 64; i++) vout[i] = scale_pow2((float)q[i], emax - 30);
  } else {
    // results may be subnormal: round once from the exact double product
#pragma unroll
    for (int i = 0; i < 64; i++) vout[i] = (float)__builtin_ldexp((double)q[i], emax - 30);
  }
}

}  // namespace zfpx
