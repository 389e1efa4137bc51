/*
 * zfp_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, deliberately unoptimised CPU implementation of ZFP coding of
 * 3-D float32 arrays (fixed rate, and the variable-size modes), used to check the HIP library bit for bit.
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it; the product path never does, and it shares no code,
 * header, table or helper with the HIP library.
 *
 * What is computed, and where it comes from:
 *  - The paper (Section II-C, "ZFP Fixed-Rate Compression"; Section IV-B,
 *    "Compression Configuration") fixes the method: ZFP in fixed-rate mode,
 *    arrays cut into independent 4x4x4 blocks, a lifting decorrelating
 *    transform, precision reduction, exactly r compressed bits per value,
 *    rates 16 and 8.
 *  - The steps inside a block follow ZFP's published algorithm description
 *    (Lindstrom 2014, cited by the paper): block-floating-point conversion to a
 *    common exponent, the separable 4-point integer lifting transform,
 *    sequency ordering, negabinary conversion, and embedded bit-plane coding
 *    with group tests, cut off at the fixed bit budget.
 *  - Conventions the description leaves open are fixed as follows (each is a
 *    reading, not a claim of byte compatibility with the ZFP library):
 *      header   : 1 bit "non-empty" flag, then 8 bits of emax+127, LSB first;
 *                 an all-zero block is the single bit 0;
 *      bit order: bits appended least-significant first into little-endian
 *                 64-bit words; block b occupies bits [64 r b, 64 r (b+1));
 *      padding  : partial blocks are completed by clamp-to-edge replication
 *                 and padded positions are never written on decode;
 *      cast     : q = trunc(v 2^(30-emax)), an exact real product;
 *      inverse  : v = RNE_float32(q 2^(emax-30)), one rounding;
 *      ordering : sequency key (i+j+k, i^2+j^2+k^2, 16k+4j+i);
 *      budget   : all 32 bit planes eligible; when the budget runs out in the
 *                 middle of a scan the decoder still sets the bit at the
 *                 current scan position.
 *  - The variable-size modes (fixed precision, fixed accuracy) that the paper
 *    names as future work (Sections II-C and IV-B) are the same coder
 *    stopped after a block-dependent number of bit planes; see "Variable-size
 *    blocks" below for the rule and the stream layout used for them.
 *  - "Parity unpinned": byte compatibility with the ZFP library itself (no
 *    library is available to compare against), and the paper's measured error
 *    values (its input data are not available).
 *
 * Floating point is done in double precision where it occurs (cast and
 * inverse cast); everything after the cast is 32-bit two's-complement integer
 * arithmetic that wraps modulo 2^32, done here through 64-bit intermediates so
 * that no C signed-overflow rule is involved.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NVAL 64 /* values in a 4x4x4 block */

/* ------------------------------------------------------------------------- */
/* 32-bit wrapping integer helpers                                            */
/* ------------------------------------------------------------------------- */

/* Reduce any integer modulo 2^32 into the int32 range [-2^31, 2^31). */
static int32_t wrap32(int64_t x) {
  uint32_t u = (uint32_t)((uint64_t)x & 0xffffffffu);
  return u >= 0x80000000u ? (int32_t)((int64_t)u - 4294967296LL) : (int32_t)u;
}

/* floor(a / 2) for a signed integer (an arithmetic shift right by one). */
static int64_t half_floor(int64_t a) {
  int64_t r = a % 2;
  if (r < 0) r += 2;
  return (a - r) / 2;
}

/* ------------------------------------------------------------------------- */
/* Bit stream: one bit at a time                                              */
/* ------------------------------------------------------------------------- */

typedef struct {
  uint64_t *words;
  int64_t pos; /* next bit position */
} bitwriter;

static void put_bit(bitwriter *w, int bit) {
  if (bit) w->words[w->pos >> 6] |= (uint64_t)1 << (w->pos & 63);
  w->pos++;
}

typedef struct {
  const uint64_t *words;
  int64_t pos;
} bitreader;

static int get_bit(bitreader *r) {
  int b = (int)((r->words[r->pos >> 6] >> (r->pos & 63)) & 1u);
  r->pos++;
  return b;
}

/* ------------------------------------------------------------------------- */
/* Block exponent and block-floating-point cast (precision reduction)         */
/* ------------------------------------------------------------------------- */

/*
 * Common block exponent.  For nonzero v, e(v) is the exponent in
 * |v| = f 2^e with f in [1/2, 1); values below the smallest normal float use
 * e = -126.  emax is the largest e over the block's nonzero values.  Returns 0
 * when every value is +0 or -0 (an "empty" block), 1 otherwise.
 */
int orc_block_exponent(const float v[NVAL], int *emax) {
  int any = 0, em = -126;
  for (int i = 0; i < NVAL; i++) {
    if (v[i] != 0.0f) {
      int e;
      frexp(fabs((double)v[i]), &e);
      if (e < -126) e = -126;
      if (e > em) em = e;
      any = 1;
    }
  }
  *emax = em;
  return any;
}

/* q_i = trunc(v_i 2^(30 - emax)); the product is exact in double. */
void orc_cast_forward(const float v[NVAL], int emax, int32_t q[NVAL]) {
  for (int i = 0; i < NVAL; i++) {
    double s = ldexp((double)v[i], 30 - emax);
    q[i] = (int32_t)trunc(s);
  }
}

/* v_i = q_i 2^(emax - 30) rounded once to float32 (nearest, ties to even). */
void orc_cast_inverse(const int32_t q[NVAL], int emax, float v[NVAL]) {
  for (int i = 0; i < NVAL; i++) v[i] = (float)ldexp((double)q[i], emax - 30);
}

/* ------------------------------------------------------------------------- */
/* Decorrelating transform: 4-point integer lifting, separable in 3-D        */
/* ------------------------------------------------------------------------- */

/*
 * Forward lifting of the four values p[0], p[s], p[2s], p[3s].  Without the
 * floor roundings it is the matrix (1/16)[[4,4,4,4],[5,1,-1,-5],[-4,4,4,-4],
 * [-2,6,-6,2]] applied to (x0, x1, x2, x3); x0 becomes the mean (DC) term.
 */
void orc_lift_forward(int32_t *p, int s) {
  int64_t x0 = p[0], x1 = p[s], x2 = p[2 * s], x3 = p[3 * s];
  x0 = wrap32(half_floor(wrap32(x0 + x3)));
  x3 = wrap32(x3 - x0);
  x2 = wrap32(half_floor(wrap32(x2 + x1)));
  x1 = wrap32(x1 - x2);
  x0 = wrap32(half_floor(wrap32(x0 + x2)));
  x2 = wrap32(x2 - x0);
  x3 = wrap32(half_floor(wrap32(x3 + x1)));
  x1 = wrap32(x1 - x3);
  x3 = wrap32(x3 + half_floor(x1));
  x1 = wrap32(x1 - half_floor(x3));
  p[0] = (int32_t)x0;
  p[s] = (int32_t)x1;
  p[2 * s] = (int32_t)x2;
  p[3 * s] = (int32_t)x3;
}

/* Inverse lifting: undoes the forward steps in reverse order. */
void orc_lift_inverse(int32_t *p, int s) {
  int64_t x0 = p[0], x1 = p[s], x2 = p[2 * s], x3 = p[3 * s];
  x1 = wrap32(x1 + half_floor(x3));
  x3 = wrap32(x3 - half_floor(x1));
  x1 = wrap32(x1 + x3);
  x3 = wrap32(2 * x3 - x1);
  x2 = wrap32(x2 + x0);
  x0 = wrap32(2 * x0 - x2);
  x1 = wrap32(x1 + x2);
  x2 = wrap32(2 * x2 - x1);
  x3 = wrap32(x3 + x0);
  x0 = wrap32(2 * x0 - x3);
  p[0] = (int32_t)x0;
  p[s] = (int32_t)x1;
  p[2 * s] = (int32_t)x2;
  p[3 * s] = (int32_t)x3;
}

/* Block-local index of (x, y, z) is 16 z + 4 y + x.  Forward: x-lines, then
 * y-lines, then z-lines. */
void orc_transform_forward(int32_t q[NVAL]) {
  for (int z = 0; z < 4; z++)
    for (int y = 0; y < 4; y++) orc_lift_forward(q + 16 * z + 4 * y, 1);
  for (int z = 0; z < 4; z++)
    for (int x = 0; x < 4; x++) orc_lift_forward(q + 16 * z + x, 4);
  for (int y = 0; y < 4; y++)
    for (int x = 0; x < 4; x++) orc_lift_forward(q + 4 * y + x, 16);
}

/* Inverse: z-lines, then y-lines, then x-lines. */
void orc_transform_inverse(int32_t q[NVAL]) {
  for (int y = 0; y < 4; y++)
    for (int x = 0; x < 4; x++) orc_lift_inverse(q + 4 * y + x, 16);
  for (int z = 0; z < 4; z++)
    for (int x = 0; x < 4; x++) orc_lift_inverse(q + 16 * z + x, 4);
  for (int z = 0; z < 4; z++)
    for (int y = 0; y < 4; y++) orc_lift_inverse(q + 16 * z + 4 * y, 1);
}

/* ------------------------------------------------------------------------- */
/* Sequency ordering                                                          */
/* ------------------------------------------------------------------------- */

static int seq_key_cmp(const void *a, const void *b) {
  int ia = *(const int *)a, ib = *(const int *)b;
  int xa = ia & 3, ya = (ia >> 2) & 3, za = ia >> 4;
  int xb = ib & 3, yb = (ib >> 2) & 3, zb = ib >> 4;
  int sa = xa + ya + za, sb = xb + yb + zb;
  if (sa != sb) return sa - sb;
  int qa = xa * xa + ya * ya + za * za, qb = xb * xb + yb * yb + zb * zb;
  if (qa != qb) return qa - qb;
  return ia - ib;
}

/* perm[s] = block-local index of the coefficient at sequency position s. */
void orc_sequency_order(int perm[NVAL]) {
  for (int i = 0; i < NVAL; i++) perm[i] = i;
  qsort(perm, NVAL, sizeof(int), seq_key_cmp);
}

/* ------------------------------------------------------------------------- */
/* Negabinary conversion                                                      */
/* ------------------------------------------------------------------------- */

#define NBMASK 0xaaaaaaaau

uint32_t orc_to_negabinary(int32_t q) {
  uint32_t t = (uint32_t)(((uint64_t)(int64_t)q + NBMASK) & 0xffffffffu);
  return t ^ NBMASK;
}

int32_t orc_from_negabinary(uint32_t u) {
  return wrap32((int64_t)(u ^ NBMASK) - (int64_t)NBMASK);
}

/* ------------------------------------------------------------------------- */
/* Embedded bit-plane coding under a fixed bit budget                         */
/* ------------------------------------------------------------------------- */

/* Bit s of the plane word is bit k of u[s]. */
static uint64_t plane_word(const uint32_t u[NVAL], int k) {
  uint64_t x = 0;
  for (int s = 0; s < NVAL; s++) x |= (uint64_t)((u[s] >> k) & 1u) << s;
  return x;
}

/*
 * Code the 64 negabinary coefficients, most significant plane first, writing
 * at most `budget` bits.  n counts the leading sequency positions already
 * known to be significant.  For each plane: the first n bits verbatim, then
 * repeated group tests ("is any bit at position >= n set?"), each positive
 * test followed by a unary scan to the next set bit; position 63 is implied
 * when the scan reaches it.  Returns the number of bits written.
 */
int64_t orc_encode_planes_from(const uint32_t u[NVAL], int kmin, int64_t budget,
                               uint64_t *words, int64_t bitpos) {
  bitwriter w = {words, bitpos};
  int64_t bits = budget;
  int n = 0;
  for (int k = 31; k >= kmin && bits > 0; k--) {
    uint64_t x = plane_word(u, k);
    int64_t m = n < bits ? n : bits;
    for (int64_t i = 0; i < m; i++) put_bit(&w, (int)((x >> i) & 1u));
    bits -= m;
    while (n < 64 && bits > 0) {
      int group = (x >> n) != 0;
      put_bit(&w, group);
      bits--;
      if (!group) break;
      while (n < 63 && bits > 0) {
        int b = (int)((x >> n) & 1u);
        put_bit(&w, b);
        bits--;
        if (b) break;
        n++;
      }
      n++;
    }
  }
  return w.pos - bitpos;
}

/* All 32 planes (fixed-rate mode). */
int64_t orc_encode_planes(const uint32_t u[NVAL], int64_t budget, uint64_t *words,
                          int64_t bitpos) {
  return orc_encode_planes_from(u, 0, budget, words, bitpos);
}

/* Mirror image of orc_encode_planes_from; returns the number of bits read. */
int64_t orc_decode_planes_from(const uint64_t *words, int64_t bitpos, int kmin, int64_t budget,
                               uint32_t u[NVAL]) {
  bitreader r = {words, bitpos};
  int64_t bits = budget;
  int n = 0;
  for (int s = 0; s < NVAL; s++) u[s] = 0;
  for (int k = 31; k >= kmin && bits > 0; k--) {
    uint64_t x = 0;
    int64_t m = n < bits ? n : bits;
    for (int64_t i = 0; i < m; i++) x |= (uint64_t)get_bit(&r) << i;
    bits -= m;
    while (n < 64 && bits > 0) {
      bits--;
      if (!get_bit(&r)) break;
      while (n < 63 && bits > 0) {
        bits--;
        if (get_bit(&r)) break;
        n++;
      }
      x |= (uint64_t)1 << n;
      n++;
    }
    for (int s = 0; s < NVAL; s++) u[s] |= (uint32_t)((x >> s) & 1u) << k;
  }
  return r.pos - bitpos;
}

int64_t orc_decode_planes(const uint64_t *words, int64_t bitpos, int64_t budget,
                          uint32_t u[NVAL]) {
  return orc_decode_planes_from(words, bitpos, 0, budget, u);
}

/* ------------------------------------------------------------------------- */
/* One block                                                                  */
/* ------------------------------------------------------------------------- */

/* Encode 64 values into exactly `rate` 64-bit words (64 * rate bits). */
void orc_encode_block(const float v[NVAL], int rate, uint64_t *words) {
  int64_t maxbits = 64 * (int64_t)rate;
  memset(words, 0, (size_t)rate * sizeof(uint64_t));
  bitwriter w = {words, 0};
  int emax;
  if (!orc_block_exponent(v, &emax)) {
    put_bit(&w, 0); /* empty block; the rest stays zero */
    return;
  }
  put_bit(&w, 1);
  for (int i = 0; i < 8; i++) put_bit(&w, ((emax + 127) >> i) & 1);
  int32_t q[NVAL];
  orc_cast_forward(v, emax, q);
  orc_transform_forward(q);
  int perm[NVAL];
  orc_sequency_order(perm);
  uint32_t u[NVAL];
  for (int s = 0; s < NVAL; s++) u[s] = orc_to_negabinary(q[perm[s]]);
  orc_encode_planes(u, maxbits - 9, words, w.pos);
}

/* Decode `rate` words into 64 values. */
void orc_decode_block(const uint64_t *words, int rate, float v[NVAL]) {
  int64_t maxbits = 64 * (int64_t)rate;
  bitreader r = {words, 0};
  if (!get_bit(&r)) {
    for (int i = 0; i < NVAL; i++) v[i] = 0.0f;
    return;
  }
  int e = 0;
  for (int i = 0; i < 8; i++) e |= get_bit(&r) << i;
  int emax = e - 127;
  uint32_t u[NVAL];
  orc_decode_planes(words, r.pos, maxbits - 9, u);
  int perm[NVAL];
  orc_sequency_order(perm);
  int32_t q[NVAL];
  for (int s = 0; s < NVAL; s++) q[perm[s]] = orc_from_negabinary(u[s]);
  orc_transform_inverse(q);
  orc_cast_inverse(q, emax, v);
}

/* ------------------------------------------------------------------------- */
/* Variable-size blocks: fixed-precision and fixed-accuracy modes             */
/* ------------------------------------------------------------------------- */
/*
 * The paper (Sections II-C and IV-B) names ZFP's two variable-size modes as
 * the alternative to fixed rate that future work may take up: a fixed number
 * of bit planes (precision mode) and a fixed absolute error tolerance
 * (accuracy mode).  In ZFP's description both run the same block coder as
 * fixed rate but stop after fewer bit planes, with no rate budget:
 *   - a block with exponent emax codes planes 31 .. 32 - p, where
 *     p = min(maxprec, max(0, emax - minexp + 2 (d + 1))), d = 3 dimensions
 *     (the 2 (d + 1) planes cover the growth of the decorrelating transform
 *     so that the dropped planes stay below 2^minexp);
 *   - precision mode: maxprec = the precision, minexp unbounded;
 *   - accuracy mode: maxprec = 32, minexp = floor(log2 tolerance);
 *   - p = 0, like an all-zero block, is the single bit 0.
 * Here the block length is also capped at maxbits (ZFP's expert-mode bit
 * cap); a block that reaches the cap is cut there like a fixed-rate block
 * and loses the error guarantee.  The block's length is the number of bits
 * the coder wrote (header included).
 */

/* Bit planes coded for a block with exponent emax. */
int orc_block_precision(int emax, int maxprec, int minexp) {
  int64_t p = (int64_t)emax - (int64_t)minexp + 8;
  if (p < 0) p = 0;
  if (p > maxprec) p = maxprec;
  return (int)p;
}

/* Encode into zeroed words (at least maxbits / 64 + 1 of them); returns the
 * length in bits (1 .. maxbits). */
int64_t orc_encode_block_var(const float v[NVAL], int maxprec, int minexp, int64_t maxbits,
                             uint64_t *words) {
  bitwriter w = {words, 0};
  int emax;
  int prec = 0;
  if (orc_block_exponent(v, &emax)) prec = orc_block_precision(emax, maxprec, minexp);
  if (prec == 0) {
    put_bit(&w, 0);
    return 1;
  }
  put_bit(&w, 1);
  for (int i = 0; i < 8; i++) put_bit(&w, ((emax + 127) >> i) & 1);
  int32_t q[NVAL];
  orc_cast_forward(v, emax, q);
  orc_transform_forward(q);
  int perm[NVAL];
  orc_sequency_order(perm);
  uint32_t u[NVAL];
  for (int s = 0; s < NVAL; s++) u[s] = orc_to_negabinary(q[perm[s]]);
  return 9 + orc_encode_planes_from(u, 32 - prec, maxbits - 9, words, w.pos);
}

/* Decode a block made by orc_encode_block_var with the same parameters. */
void orc_decode_block_var(const uint64_t *words, int maxprec, int minexp, int64_t maxbits,
                          float v[NVAL]) {
  bitreader r = {words, 0};
  if (!get_bit(&r)) {
    for (int i = 0; i < NVAL; i++) v[i] = 0.0f;
    return;
  }
  int e = 0;
  for (int i = 0; i < 8; i++) e |= get_bit(&r) << i;
  int emax = e - 127;
  int prec = orc_block_precision(emax, maxprec, minexp);
  uint32_t u[NVAL];
  orc_decode_planes_from(words, r.pos, 32 - prec, maxbits - 9, u);
  int perm[NVAL];
  orc_sequency_order(perm);
  int32_t q[NVAL];
  for (int s = 0; s < NVAL; s++) q[perm[s]] = orc_from_negabinary(u[s]);
  orc_transform_inverse(q);
  orc_cast_inverse(q, emax, v);
}

/* ------------------------------------------------------------------------- */
/* Regular strided 3-D arrays                                                 */
/* ------------------------------------------------------------------------- */

static int64_t ceil4(int64_t n) { return (n + 3) / 4; }
static int64_t imin64(int64_t a, int64_t b) { return a < b ? a : b; }

/* Blocks of an nx x ny x nz array: ceil(nx/4) ceil(ny/4) ceil(nz/4). */
int64_t orc_regular_blocks(int64_t nx, int64_t ny, int64_t nz) {
  return ceil4(nx) * ceil4(ny) * ceil4(nz);
}

/* Gather block (bx, by, bz) with clamp-to-edge padding. */
static void gather_regular(const float *a, int64_t nx, int64_t ny, int64_t nz, int64_t sx,
                           int64_t sy, int64_t sz, int64_t bx, int64_t by, int64_t bz,
                           float v[NVAL]) {
  for (int z = 0; z < 4; z++)
    for (int y = 0; y < 4; y++)
      for (int x = 0; x < 4; x++) {
        int64_t i = imin64(4 * bx + x, nx - 1);
        int64_t j = imin64(4 * by + y, ny - 1);
        int64_t k = imin64(4 * bz + z, nz - 1);
        v[16 * z + 4 * y + x] = a[i * sx + j * sy + k * sz];
      }
}

/* Blocks are numbered with bx fastest, then by, then bz. */
void orc_encode_regular(const float *a, int64_t nx, int64_t ny, int64_t nz, int64_t sx,
                        int64_t sy, int64_t sz, int rate, uint64_t *out) {
  int64_t nbx = ceil4(nx), nby = ceil4(ny), nbz = ceil4(nz);
  int64_t nb = nbx * nby * nbz;
#pragma omp parallel for schedule(static)
  for (int64_t b = 0; b < nb; b++) {
    float v[NVAL];
    gather_regular(a, nx, ny, nz, sx, sy, sz, b % nbx, (b / nbx) % nby, b / (nbx * nby), v);
    orc_encode_block(v, rate, out + b * rate);
  }
}

/* Only positions inside the array are written. */
void orc_decode_regular(const uint64_t *in, int64_t nx, int64_t ny, int64_t nz, int64_t sx,
                        int64_t sy, int64_t sz, int rate, float *a) {
  int64_t nbx = ceil4(nx), nby = ceil4(ny), nbz = ceil4(nz);
  int64_t nb = nbx * nby * nbz;
#pragma omp parallel for schedule(static)
  for (int64_t b = 0; b < nb; b++) {
    float v[NVAL];
    int64_t bx = b % nbx, by = (b / nbx) % nby, bz = b / (nbx * nby);
    orc_decode_block(in + b * rate, rate, v);
    for (int z = 0; z < 4; z++)
      for (int y = 0; y < 4; y++)
        for (int x = 0; x < 4; x++) {
          int64_t i = 4 * bx + x, j = 4 * by + y, k = 4 * bz + z;
          if (i < nx && j < ny && k < nz) a[i * sx + j * sy + k * sz] = v[16 * z + 4 * y + x];
        }
  }
}

/* ------------------------------------------------------------------------- */
/* Per-destination chunks with ragged rows (pack + encode, decode + unpack)   */
/* ------------------------------------------------------------------------- */
/*
 * Chunk c is a 3-D view of a larger buffer: levels z = 0..levels[c]-1 at
 * element offset chunk_base[c] + z * level_stride[c]; rows
 * r = row_start[c]..row_start[c+1]-1 at further offset row_offset[r], each
 * row_len[r] points long and contiguous in x.  Rows are taken in groups of
 * four in order; a group is as wide as its longest row.  Each chunk is coded
 * as its own array: blocks are numbered (level block, row group, x block) with
 * the x block fastest, and chunk streams are concatenated in chunk order.
 */

typedef struct {
  int nchunks;
  const int64_t *chunk_base, *level_stride;
  const int32_t *levels, *row_start;
  const int64_t *row_offset;
  const int32_t *row_len;
} chunk_table;

static int64_t group_width(const chunk_table *t, int c, int64_t g) {
  int64_t r0 = t->row_start[c], r1 = t->row_start[c + 1];
  int64_t w = 0;
  for (int64_t r = r0 + 4 * g; r < r0 + 4 * g + 4 && r < r1; r++)
    if (t->row_len[r] > w) w = t->row_len[r];
  return w;
}

/* Blocks in chunk c: ceil(levels/4) * sum over row groups of ceil(width/4). */
static int64_t chunk_blocks(const chunk_table *t, int c) {
  int64_t nrows = t->row_start[c + 1] - t->row_start[c];
  int64_t per_level_block = 0;
  for (int64_t g = 0; g < ceil4(nrows); g++) per_level_block += ceil4(group_width(t, c, g));
  return ceil4(t->levels[c]) * per_level_block;
}

void orc_chunk_blocks(int nchunks, const int64_t *chunk_base, const int64_t *level_stride,
                      const int32_t *levels, const int32_t *row_start,
                      const int64_t *row_offset, const int32_t *row_len, int64_t *blocks) {
  chunk_table t = {nchunks, chunk_base, level_stride, levels, row_start, row_offset, row_len};
  for (int c = 0; c < nchunks; c++) blocks[c] = chunk_blocks(&t, c);
}

/* Locate block b of chunk c and gather its 64 values (clamp-to-edge). */
static void gather_chunk_block(const chunk_table *t, int c, int64_t b, const float *src,
                               float v[NVAL], int64_t *pos /* 64 element offsets or NULL */,
                               int *inside /* 64 flags or NULL */) {
  int64_t r0 = t->row_start[c], nrows = t->row_start[c + 1] - r0;
  int64_t ngroups = ceil4(nrows);
  int64_t per_level_block = 0;
  for (int64_t g = 0; g < ngroups; g++) per_level_block += ceil4(group_width(t, c, g));
  int64_t bz = b / per_level_block, rem = b % per_level_block;
  int64_t g = 0;
  while (rem >= ceil4(group_width(t, c, g))) {
    rem -= ceil4(group_width(t, c, g));
    g++;
  }
  int64_t bx = rem;
  for (int z = 0; z < 4; z++)
    for (int y = 0; y < 4; y++)
      for (int x = 0; x < 4; x++) {
        int64_t lz = 4 * bz + z, ry = 4 * g + y, px = 4 * bx + x;
        int64_t lzc = imin64(lz, t->levels[c] - 1);
        int64_t ryc = imin64(ry, nrows - 1);
        int64_t len = t->row_len[r0 + ryc];
        int64_t pxc = imin64(px, len - 1);
        int64_t off = t->chunk_base[c] + lzc * t->level_stride[c] + t->row_offset[r0 + ryc] + pxc;
        int i = 16 * z + 4 * y + x;
        if (v) v[i] = src[off];
        if (pos) pos[i] = off;
        if (inside) inside[i] = (lz < t->levels[c]) && (ry < nrows) && (px < len);
      }
}

void orc_pack_encode(int nchunks, const int64_t *chunk_base, const int64_t *level_stride,
                     const int32_t *levels, const int32_t *row_start,
                     const int64_t *row_offset, const int32_t *row_len, const float *src,
                     int rate, uint64_t *out) {
  chunk_table t = {nchunks, chunk_base, level_stride, levels, row_start, row_offset, row_len};
  int64_t first = 0;
  for (int c = 0; c < nchunks; c++) {
    int64_t nb = chunk_blocks(&t, c);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t b = 0; b < nb; b++) {
      float v[NVAL];
      gather_chunk_block(&t, c, b, src, v, NULL, NULL);
      orc_encode_block(v, rate, out + (first + b) * rate);
    }
    first += nb;
  }
}

void orc_decode_unpack(int nchunks, const int64_t *chunk_base, const int64_t *level_stride,
                       const int32_t *levels, const int32_t *row_start,
                       const int64_t *row_offset, const int32_t *row_len, const uint64_t *in,
                       int rate, float *dst) {
  chunk_table t = {nchunks, chunk_base, level_stride, levels, row_start, row_offset, row_len};
  int64_t first = 0;
  for (int c = 0; c < nchunks; c++) {
    int64_t nb = chunk_blocks(&t, c);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t b = 0; b < nb; b++) {
      float v[NVAL];
      int64_t pos[NVAL];
      int inside[NVAL];
      gather_chunk_block(&t, c, b, NULL, NULL, pos, inside);
      orc_decode_block(in + (first + b) * rate, rate, v);
      for (int i = 0; i < NVAL; i++)
        if (inside[i]) dst[pos[i]] = v[i];
    }
    first += nb;
  }
}

/*
 * Encode only the listed global block ids (numbered across all chunks in
 * chunk order), writing `rate` words per listed block into out[j * rate].
 * Used to check very large buffers on a sample of blocks.
 */
void orc_pack_encode_sample(int nchunks, const int64_t *chunk_base, const int64_t *level_stride,
                            const int32_t *levels, const int32_t *row_start,
                            const int64_t *row_offset, const int32_t *row_len,
                            const float *src, int rate, const int64_t *ids, int64_t nids,
                            uint64_t *out) {
  chunk_table t = {nchunks, chunk_base, level_stride, levels, row_start, row_offset, row_len};
  int64_t *first = (int64_t *)malloc(sizeof(int64_t) * ((size_t)nchunks + 1));
  first[0] = 0;
  for (int c = 0; c < nchunks; c++) first[c + 1] = first[c] + chunk_blocks(&t, c);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t j = 0; j < nids; j++) {
    int c = 0;
    while (c + 1 < nchunks && first[c + 1] <= ids[j]) c++;
    float v[NVAL];
    gather_chunk_block(&t, c, ids[j] - first[c], src, v, NULL, NULL);
    orc_encode_block(v, rate, out + j * rate);
  }
  free(first);
}

/* Decode the listed global block ids of a stream; writes 64 values per id
 * into vals[j * 64] and their element offsets / in-range flags. */
void orc_decode_sample(int nchunks, const int64_t *chunk_base, const int64_t *level_stride,
                       const int32_t *levels, const int32_t *row_start,
                       const int64_t *row_offset, const int32_t *row_len, const uint64_t *in,
                       int rate, const int64_t *ids, int64_t nids, float *vals, int64_t *pos,
                       int32_t *inside) {
  chunk_table t = {nchunks, chunk_base, level_stride, levels, row_start, row_offset, row_len};
  int64_t *first = (int64_t *)malloc(sizeof(int64_t) * ((size_t)nchunks + 1));
  first[0] = 0;
  for (int c = 0; c < nchunks; c++) first[c + 1] = first[c] + chunk_blocks(&t, c);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t j = 0; j < nids; j++) {
    int c = 0;
    while (c + 1 < nchunks && first[c + 1] <= ids[j]) c++;
    int ins[NVAL];
    gather_chunk_block(&t, c, ids[j] - first[c], NULL, NULL, pos + j * NVAL, ins);
    orc_decode_block(in + ids[j] * rate, rate, vals + j * NVAL);
    for (int i = 0; i < NVAL; i++) inside[j * NVAL + i] = ins[i];
  }
  free(first);
}

/* Decode many independent blocks (block j at in[j * rate]). */
void orc_decode_blocks(const uint64_t *in, int64_t nblocks, int rate, float *vals) {
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < nblocks; j++) orc_decode_block(in + j * rate, rate, vals + j * NVAL);
}

/* Encode many independent blocks (block j's values at vals[j * 64]). */
void orc_encode_blocks(const float *vals, int64_t nblocks, int rate, uint64_t *out) {
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < nblocks; j++) orc_encode_block(vals + j * NVAL, rate, out + j * rate);
}

/* ------------------------------------------------------------------------- */
/* Variable-size stream of a chunk set                                        */
/* ------------------------------------------------------------------------- */
/*
 * Layout of this library's variable-size mode (a convention of its own, not
 * ZFP's file format): blocks are numbered across chunks in chunk order as in
 * fixed rate; block b's bits, LSB first, padded with zeros to whole 32-bit
 * words, take nd[b] = ceil(len_b / 32) words starting at word
 * off(b) = nd[0] + ... + nd[b-1] of the output; tile_off[t] = off(64 t) for
 * t < ceil(nb / 64) and tile_off[ceil(nb / 64)] = the total word count.
 * Chunk c's message is the words from off(first block of c) to
 * off(first block of c+1); the per-block counts rebuild every offset.
 */

/* Dword i of a block coded into 64-bit words (low half first). */
static uint32_t block_dword(const uint64_t *w, int64_t i) {
  return (uint32_t)(w[i >> 1] >> (32 * (i & 1)));
}

void orc_pack_encode_var(int nchunks, const int64_t *chunk_base, const int64_t *level_stride,
                         const int32_t *levels, const int32_t *row_start,
                         const int64_t *row_offset, const int32_t *row_len, const float *src,
                         int maxprec, int minexp, int rate_cap, uint32_t *out, uint8_t *nd,
                         int64_t *tile_off) {
  chunk_table t = {nchunks, chunk_base, level_stride, levels, row_start, row_offset, row_len};
  int64_t *first = (int64_t *)malloc(sizeof(int64_t) * ((size_t)nchunks + 1));
  first[0] = 0;
  for (int c = 0; c < nchunks; c++) first[c + 1] = first[c] + chunk_blocks(&t, c);
  int64_t nb = first[nchunks];
  int64_t maxbits = 64 * (int64_t)rate_cap, stride = rate_cap + 1;
  uint64_t *tmp = (uint64_t *)calloc((size_t)(nb > 0 ? nb : 1) * (size_t)stride, 8);
  int64_t *len = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nb > 0 ? nb : 1));
  for (int c = 0; c < nchunks; c++) {
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t b = first[c]; b < first[c + 1]; b++) {
      float v[NVAL];
      gather_chunk_block(&t, c, b - first[c], src, v, NULL, NULL);
      len[b] = orc_encode_block_var(v, maxprec, minexp, maxbits, tmp + b * stride);
    }
  }
  int64_t off = 0;
  for (int64_t b = 0; b < nb; b++) {
    if (b % 64 == 0) tile_off[b / 64] = off;
    int64_t n = (len[b] + 31) / 32;
    nd[b] = (uint8_t)n;
    for (int64_t i = 0; i < n; i++) out[off + i] = block_dword(tmp + b * stride, i);
    off += n;
  }
  tile_off[(nb + 63) / 64] = off;
  free(len);
  free(tmp);
  free(first);
}

/* Decode with offsets rebuilt from nd alone; only chunk points are written. */
void orc_decode_unpack_var(int nchunks, const int64_t *chunk_base, const int64_t *level_stride,
                           const int32_t *levels, const int32_t *row_start,
                           const int64_t *row_offset, const int32_t *row_len,
                           const uint32_t *in, const uint8_t *nd, int maxprec, int minexp,
                           int rate_cap, float *dst) {
  chunk_table t = {nchunks, chunk_base, level_stride, levels, row_start, row_offset, row_len};
  int64_t *first = (int64_t *)malloc(sizeof(int64_t) * ((size_t)nchunks + 1));
  first[0] = 0;
  for (int c = 0; c < nchunks; c++) first[c + 1] = first[c] + chunk_blocks(&t, c);
  int64_t nb = first[nchunks];
  int64_t *off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nb + 1));
  off[0] = 0;
  for (int64_t b = 0; b < nb; b++) off[b + 1] = off[b] + nd[b];
  int64_t maxbits = 64 * (int64_t)rate_cap;
  for (int c = 0; c < nchunks; c++) {
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t b = first[c]; b < first[c + 1]; b++) {
      uint64_t w[64 + 2];
      memset(w, 0, sizeof w);
      for (int64_t i = 0; i < nd[b] && i < 2 * (int64_t)rate_cap; i++)
        w[i >> 1] |= (uint64_t)in[off[b] + i] << (32 * (i & 1));
      float v[NVAL];
      int64_t pos[NVAL];
      int inside[NVAL];
      gather_chunk_block(&t, c, b - first[c], NULL, NULL, pos, inside);
      orc_decode_block_var(w, maxprec, minexp, maxbits, v);
      for (int i = 0; i < NVAL; i++)
        if (inside[i]) dst[pos[i]] = v[i];
    }
  }
  free(off);
  free(first);
}


/* Encode only the listed global block ids in a variable-size mode: block
 * j's words (zero past its length) at out[j * (rate_cap + 1)], its length in
 * bits at len[j], and its element offsets / in-range flags at pos[j * 64] and
 * inside[j * 64].  Used to check very large buffers on a sample of blocks. */
void orc_pack_encode_var_sample(int nchunks, const int64_t *chunk_base,
                                const int64_t *level_stride, const int32_t *levels,
                                const int32_t *row_start, const int64_t *row_offset,
                                const int32_t *row_len, const float *src, int maxprec,
                                int minexp, int rate_cap, const int64_t *ids, int64_t nids,
                                uint64_t *out, int64_t *len, int64_t *pos, int32_t *inside) {
  chunk_table t = {nchunks, chunk_base, level_stride, levels, row_start, row_offset, row_len};
  int64_t *first = (int64_t *)malloc(sizeof(int64_t) * ((size_t)nchunks + 1));
  first[0] = 0;
  for (int c = 0; c < nchunks; c++) first[c + 1] = first[c] + chunk_blocks(&t, c);
  int64_t stride = rate_cap + 1;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t j = 0; j < nids; j++) {
    int c = 0;
    while (c + 1 < nchunks && first[c + 1] <= ids[j]) c++;
    float v[NVAL];
    int ins[NVAL];
    gather_chunk_block(&t, c, ids[j] - first[c], src, v, pos + j * NVAL, ins);
    memset(out + j * stride, 0, (size_t)stride * sizeof(uint64_t));
    len[j] = orc_encode_block_var(v, maxprec, minexp, 64 * (int64_t)rate_cap, out + j * stride);
    for (int i = 0; i < NVAL; i++) inside[j * NVAL + i] = ins[i];
  }
  free(first);
}

/* Threads used by the OpenMP loops above (for timing the oracle). */
void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }

