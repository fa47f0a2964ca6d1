// device_math.hpp -- integer arithmetic shared by the gfx950 kernels.
//
// Hash families over GF(p), p = 2^61 - 1 (Carter-Wegman polynomials; the
// paper asks for a 4-wise independent +-1 family xi and a bucket hash h per
// sketch row, Sections 4.1 and 4.2, and names no family):
//   x  = ((uint64)(int64)key) mod p
//   xi = +1 if (a0 + a1 x + a2 x^2 + a3 x^3 mod p) is even, else -1
//   h  = ((b0 + b1 x) mod p) mod w
//
// Evaluation is Horner's rule with lazy Mersenne reduction: intermediate
// values are only kept below 2^63 and congruent mod p; one canonical
// reduction at the end gives the exact residue.  Keys below 2^32 (all
// non-negative int32 keys) take the 61x32-bit path: two 32x32->64
// multiply-adds per Horner step (v_mad_u64_u32 on CDNA).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace compass {

constexpr uint64_t kP61 = (1ull << 61) - 1;

// r < 2^64  ->  r' == r (mod p), r' < 2^61 + 8
__device__ __forceinline__ uint64_t fold61(uint64_t r) {
  return (r & kP61) + (r >> 61);
}

// exact residue in [0, p) of any r < 2^64
__device__ __forceinline__ uint64_t canon61(uint64_t r) {
  r = fold61(r);
  return r >= kP61 ? r - kP61 : r;
}

// acc < 2^63, x < 2^32, c < 2^61:
// returns a value < 2^63 congruent to acc * x + c (mod p).
//   t0 = lo32(acc) * x                       (< 2^64)
//   t1 = hi32(acc) * x + hi32(t0)            (< 2^63 + 2^32)
//   acc * x = t1 * 2^32 + lo32(t0)
//   t1 * 2^32 = (t1 >> 29) * 2^61 + (t1 mod 2^29) * 2^32,  2^61 == 1 (mod p)
// so acc * x + c == (t1 mod 2^29) * 2^32 + lo32(t0) + (t1 >> 29) + c, a sum
// below 2^61 + 2^35 + 2^61.
__device__ __forceinline__ uint64_t madd61_x32_any(uint64_t acc, uint32_t x,
                                                   uint64_t c) {
  const uint64_t t0 = (uint64_t)(uint32_t)acc * x;
  const uint64_t t1 = (uint64_t)(uint32_t)(acc >> 32) * x + (t0 >> 32);
  const uint64_t low = ((t1 & 0x1FFFFFFFull) << 32) | (uint32_t)t0;
  return low + (t1 >> 29) + c;
}

// The Horner step of the hashes: acc < 2^62, x < 2^32, c < 2^61; returns a
// value below 2^61 + 2^34 (< 2^62, so steps chain) congruent to
// acc * x + c (mod p).  With l = lo32(acc), h = hi32(acc):
//   u = l * x + lo32(c)                      (< 2^64)
//   v = h * x + hi32(c) + hi32(u)            (< 2^63)
//   acc * x + c = v * 2^32 + lo32(u)
//   v * 2^32 == (v >> 29) + (v mod 2^29) * 2^32  (mod p)
// The two products take c's halves as their addends (scalar pairs), the
// low word of the result is lo32(u) and its high word (v mod 2^29), so the
// step is two v_mad_u64_u32, one 32-bit add with carry, one AND, one 64-bit
// shift and one 64-bit add.
__device__ __forceinline__ uint64_t madd61_x32(uint64_t acc, uint32_t x,
                                               uint64_t c) {
  const uint64_t u = (uint64_t)(uint32_t)acc * x + (uint32_t)c;
  const uint64_t v =
      (uint64_t)(uint32_t)(acc >> 32) * x + (c >> 32) + (u >> 32);
  uint64_t r0 = ((uint64_t)((uint32_t)v & 0x1FFFFFFFu) << 32) | (uint32_t)u;
  // a register pair as it stands (the AND writes its high word): keeps the
  // compiler from re-associating it into two 64-bit adds of zero-padded pairs
  __asm__("" : "+v"(r0));
  return r0 + (v >> 29);
}

// The same step for x < 2^31 (every non-negative int32 key): then
// l * x + c < 2^63 + 2^61 cannot wrap, so c enters whole as the first
// product's addend, and hi32(u) is the second one's:
//   u = l * x + c                            (< 2^64)
//   v = h * x + hi32(u)                      (< 2^61 + 2^32)
//   acc * x + c = v * 2^32 + lo32(u)
// Two v_mad_u64_u32 (and the move of hi32(u) into an addend pair), one AND,
// one 64-bit shift and one 64-bit add: one 64-bit add less than
// madd61_x32.  Result below 2^61 + 2^33.
__device__ __forceinline__ uint64_t madd61_x31(uint64_t acc, uint32_t x,
                                               uint64_t c) {
  const uint64_t u = (uint64_t)(uint32_t)acc * x + c;
  const uint64_t v = (uint64_t)(uint32_t)(acc >> 32) * x + (u >> 32);
  uint64_t r0 = ((uint64_t)((uint32_t)v & 0x1FFFFFFFu) << 32) | (uint32_t)u;
  __asm__("" : "+v"(r0));
  return r0 + (v >> 29);
}

// acc < 2^63, x < 2^61, c < 2^61: value < 2^63 congruent to acc * x + c.
//   acc * x = acc * lo32(x) + (acc * hi32(x)) * 2^32
__device__ __forceinline__ uint64_t madd61_x61(uint64_t acc, uint64_t x,
                                               uint64_t c) {
  const uint64_t r1 = madd61_x32_any(acc, (uint32_t)x, c);
  const uint64_t t = madd61_x32_any(acc, (uint32_t)(x >> 32), 0);
  // t * 2^32 == (t >> 29) + (t mod 2^29) * 2^32  (mod p)
  return fold61(r1) + (t >> 29) + ((t & 0x1FFFFFFFull) << 32);
}

// field element of a key: (uint64)(int64)key mod p
__device__ __forceinline__ uint64_t key_field(int64_t key) {
  return canon61((uint64_t)key);
}

// Row seeds of one sketch row.
struct RowSeeds {
  uint64_t a0, a1, a2, a3, b0, b1;
};

// bucket modulus: power of two -> mask; otherwise exact reduction of a
// 61-bit value via 2^32 mod w and a float64 quotient estimate.
struct BucketMod {
  uint32_t w;
  uint32_t mask;      // w - 1 when w is a power of two
  uint32_t r32;       // 2^32 mod w
  uint32_t pow2;
  double inv;         // 1 / w
};

__device__ __forceinline__ uint32_t bucket_of(uint64_t g, const BucketMod &m) {
  if (m.pow2) return (uint32_t)g & m.mask;
  // g < 2^61, w < 2^21: s = hi32(g) * (2^32 mod w) + lo32(g) < 2^50, s == g
  const uint64_t s = (uint64_t)(uint32_t)(g >> 32) * m.r32 + (uint32_t)g;
  int64_t q = (int64_t)((double)s * m.inv);  // off by at most one
  int64_t r = (int64_t)s - q * (int64_t)m.w;
  if (r < 0) r += m.w;
  if (r >= (int64_t)m.w) r -= m.w;
  return (uint32_t)r;
}

// Canonical residues are only needed through their low bits: for
// f = fold61(r) (< 2^61 + 8), the residue is f - p = f - 2^61 + 1 when
// f >= p, else f; 2^61 is a multiple of 2 and of any power-of-two w, so its
// low bits are those of f + (f >= p).
__device__ __forceinline__ uint32_t low_of_residue(uint64_t r) {
  const uint64_t f = fold61(r);
  return (uint32_t)f + (f >= kP61 ? 1u : 0u);
}

// sign (+1/-1) and bucket of one field element under one row's seeds.
template <bool X32>
__device__ __forceinline__ void hash_xi_h(uint64_t x, const RowSeeds &s,
                                          const BucketMod &m, int32_t &sign,
                                          uint32_t &bucket) {
  uint64_t v, g;
  if (X32) {
    const uint32_t x32 = (uint32_t)x;
    v = madd61_x32(s.a3, x32, s.a2);
    v = madd61_x32(v, x32, s.a1);
    v = madd61_x32(v, x32, s.a0);
    g = madd61_x32(s.b1, x32, s.b0);
  } else {
    v = madd61_x61(s.a3, x, s.a2);
    v = madd61_x61(v, x, s.a1);
    v = madd61_x61(v, x, s.a0);
    g = madd61_x61(s.b1, x, s.b0);
  }
  sign = 1 - 2 * (int32_t)(low_of_residue(v) & 1u);
  bucket = m.pow2 ? (low_of_residue(g) & m.mask) : bucket_of(canon61(g), m);
}

// Sign and power-of-two bucket of R keys (each below 2^32, or below 2^31
// with X31) under one row's seeds, step by step across the keys so that the
// R independent Horner chains interleave.
template <int R, bool X31 = false>
__device__ __forceinline__ void hash_many_pow2(const uint64_t (&x)[R],
                                               const RowSeeds &s, uint32_t mask,
                                               int32_t (&sign)[R],
                                               uint32_t (&bucket)[R]) {
  auto step = [](uint64_t acc, uint32_t xx, uint64_t c) {
    return X31 ? madd61_x31(acc, xx, c) : madd61_x32(acc, xx, c);
  };
  uint64_t v[R], g[R];
#pragma unroll
  for (int k = 0; k < R; ++k) v[k] = step(s.a3, (uint32_t)x[k], s.a2);
#pragma unroll
  for (int k = 0; k < R; ++k) g[k] = step(s.b1, (uint32_t)x[k], s.b0);
#pragma unroll
  for (int k = 0; k < R; ++k) v[k] = step(v[k], (uint32_t)x[k], s.a1);
#pragma unroll
  for (int k = 0; k < R; ++k) v[k] = step(v[k], (uint32_t)x[k], s.a0);
#pragma unroll
  for (int k = 0; k < R; ++k) {
    // +1 or -1 from the parity: bit 0 sign-extended (0 or -1), doubled, | 1
    // (opaque before and after the extract: the low bits stay one add with
    // carry, and the sign two instructions, instead of a compare of bit 0,
    // a mask xor and a select)
    uint32_t lr = low_of_residue(v[k]);
    __asm__("" : "+v"(lr));
    int32_t par = __builtin_amdgcn_sbfe((int32_t)lr, 0, 1);
    __asm__("" : "+v"(par));
    sign[k] = (int32_t)((uint32_t)par << 1) | 1;
    bucket[k] = low_of_residue(g[k]) & mask;
  }
}

// hash_many_pow2 of keys below 2^32 with the Horner step picked per wave:
// the shorter step when no key of the wave reaches 2^31.
template <int R>
__device__ __forceinline__ void hash_many_pow2_auto(const uint64_t (&x)[R],
                                                    const RowSeeds &s,
                                                    uint32_t mask,
                                                    int32_t (&sign)[R],
                                                    uint32_t (&bucket)[R]) {
  bool big = false;
#pragma unroll
  for (int k = 0; k < R; ++k) big = big || (x[k] >> 31) != 0;
  if (__any(big))
    hash_many_pow2<R, false>(x, s, mask, sign, bucket);
  else
    hash_many_pow2<R, true>(x, s, mask, sign, bucket);
}

// ---------------------------------------------------------------------
// 128-bit two's complement (wrapping) helpers
// ---------------------------------------------------------------------
typedef unsigned __int128 u128;

__device__ __forceinline__ u128 s64_to_u128(int64_t v) {
  return (u128)(__int128)v;
}

// 64 x 64 -> 128 unsigned product from four 32 x 32 -> 64 products.
__device__ __forceinline__ u128 mul_u64_full(uint64_t a, uint64_t b) {
  const uint64_t al = (uint32_t)a, ah = a >> 32;
  const uint64_t bl = (uint32_t)b, bh = b >> 32;
  const uint64_t ll = al * bl;
  const uint64_t lh = al * bh;
  const uint64_t hl = ah * bl;
  const uint64_t hh = ah * bh;
  const uint64_t mid = (ll >> 32) + (uint32_t)lh + (uint32_t)hl;
  const uint64_t lo = (mid << 32) | (uint32_t)ll;
  const uint64_t hi = hh + (lh >> 32) + (hl >> 32) + (mid >> 32);
  return ((u128)hi << 64) | lo;
}

// product mod 2^128
__device__ __forceinline__ u128 mul_u128(u128 a, u128 b) {
  const uint64_t al = (uint64_t)a, ah = (uint64_t)(a >> 64);
  const uint64_t bl = (uint64_t)b, bh = (uint64_t)(b >> 64);
  u128 r = mul_u64_full(al, bl);
  const uint64_t cross = al * bh + ah * bl;
  return r + ((u128)cross << 64);
}

// signed 64 x signed 64 -> exact signed 128-bit product
__device__ __forceinline__ u128 mul_s64_s64(int64_t a, int64_t b) {
  const u128 r = mul_u64_full((uint64_t)a, (uint64_t)b);
  uint64_t hi = (uint64_t)(r >> 64);
  if (a < 0) hi -= (uint64_t)b;
  if (b < 0) hi -= (uint64_t)a;
  return ((u128)hi << 64) | (uint64_t)r;
}

// 128-bit value times signed 64-bit value (sign-extended), mod 2^128
__device__ __forceinline__ u128 mul_u128_s64(u128 t, int64_t b) {
  const uint64_t tl = (uint64_t)t, th = (uint64_t)(t >> 64);
  const u128 r = mul_u64_full(tl, (uint64_t)b);
  uint64_t hi = (uint64_t)(r >> 64) + th * (uint64_t)b;
  if (b < 0) hi -= tl;
  return ((u128)hi << 64) | (uint64_t)r;
}

// signed 64-bit value times 128-bit value, mod 2^128
__device__ __forceinline__ u128 mul_s64_u128(int64_t a, u128 b) {
  return mul_u128(s64_to_u128(a), b);
}

// Round-to-nearest-even conversion of a signed 128-bit integer to double.
__device__ __forceinline__ double i128_to_double(u128 u) {
  const bool neg = (u >> 127) != 0;
  u128 m = neg ? (u128)(~u + 1) : u;  // |value|; -2^127 stays 2^127
  if (m == 0) return 0.0;
  const uint64_t hi = (uint64_t)(m >> 64), lo = (uint64_t)m;
  const int lz = hi ? __builtin_clzll(hi) : 64 + __builtin_clzll(lo);
  const int nbits = 128 - lz;  // position of the leading one + 1
  double r;
  if (nbits <= 53) {
    r = (double)(uint64_t)m;  // exact
  } else {
    const int sh = nbits - 53;
    u128 mant = m >> sh;
    const u128 rem = m & (((u128)1 << sh) - 1);
    const u128 half = (u128)1 << (sh - 1);
    if (rem > half || (rem == half && (mant & 1))) mant += 1;
    int e = sh;
    if (mant >> 53) {  // carried into a new bit
      mant >>= 1;
      e += 1;
    }
    r = ldexp((double)(uint64_t)mant, e);
  }
  return neg ? -r : r;
}

}  // namespace compass
