// Shared device/host helpers of the PT2 library (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#ifndef SHCI_DEV
#define SHCI_DEV __device__ __forceinline__
#endif
// pure bit manipulation, also usable in host code (unit tests)
#define SHCI_HD __host__ __device__ __forceinline__

namespace shci {

constexpr int WAVE = 64;

// ---------------------------------------------------------------------------
// Hashing: murmur3's 64-bit finaliser chained over the key words.  Used for
// the bucket id (top bits), the in-bucket sort key (next 32 bits) and the
// variational-space hash set.
// ---------------------------------------------------------------------------
SHCI_HD uint64_t fmix64(uint64_t k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdull;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ull;
  k ^= k >> 33;
  return k;
}

template <int KW>
SHCI_HD uint64_t hash_key(const uint64_t (&k)[KW]) {
  uint64_t h = 0x243f6a8885a308d3ull;
#pragma unroll
  for (int w = 0; w < KW; ++w) h = fmix64(h ^ k[w]);
  return h;
}

// ---------------------------------------------------------------------------
// Packed keys.  A determinant (alpha, beta; 128 bits each) is packed as
// bits [0,n) alpha, [n,2n) beta, then the sample id in [2n, 2n+sbits), then
// one auxiliary flag bit at 2n+sbits.  KW 64-bit words hold it.
// ---------------------------------------------------------------------------
template <int KW>
SHCI_HD void put_bits(uint64_t (&k)[KW], uint64_t v0, uint64_t v1, int off) {
  // OR the 128-bit value (v0 | v1<<64) into k at bit offset off
  const int w = off >> 6, b = off & 63;
#pragma unroll
  for (int j = 0; j < KW; ++j) {
    uint64_t add = 0;
    if (j == w) add = v0 << b;
    if (j == w + 1) add = (b ? (v0 >> (64 - b)) : 0ull) | (v1 << b);
    if (j == w + 2) add = b ? (v1 >> (64 - b)) : 0ull;
    k[j] |= add;
  }
}

template <int KW>
SHCI_HD void get_bits(const uint64_t (&k)[KW], int off, int nbits, uint64_t& v0, uint64_t& v1) {
  // extract nbits (<= 128) starting at bit off
  const int w = off >> 6, b = off & 63;
  uint64_t x0 = 0, x1 = 0, x2 = 0;
#pragma unroll
  for (int j = 0; j < KW; ++j) {
    if (j == w) x0 = k[j];
    if (j == w + 1) x1 = k[j];
    if (j == w + 2) x2 = k[j];
  }
  v0 = b ? ((x0 >> b) | (x1 << (64 - b))) : x0;
  v1 = b ? ((x1 >> b) | (x2 << (64 - b))) : x1;
  if (nbits < 64) {
    v0 &= (1ull << nbits) - 1ull;
    v1 = 0;
  } else if (nbits < 128) {
    v1 &= (nbits == 64) ? 0ull : ((1ull << (nbits - 64)) - 1ull);
  }
}

// key = alpha | beta << n, in closed form (1 <= n <= 127; the branch on
// n >= 64 is uniform across a wavefront)
template <int KW>
SHCI_HD void pack_det(uint64_t (&k)[KW], uint64_t a0, uint64_t a1, uint64_t b0, uint64_t b1,
                       int n) {
  uint64_t o0, o1, o2, o3;
  if (n < 64) {
    o0 = b0 << n;
    o1 = (b1 << n) | (b0 >> (64 - n));
    o2 = b1 >> (64 - n);
    o3 = 0ull;
  } else {
    const int t = n - 64;
    o0 = 0ull;
    o1 = b0 << t;
    o2 = t ? ((b1 << t) | (b0 >> (64 - t))) : b1;
    o3 = t ? (b1 >> (64 - t)) : 0ull;
  }
  const uint64_t w[4] = {a0 | o0, a1 | o1, o2, o3};
#pragma unroll
  for (int j = 0; j < KW; ++j) k[j] = w[j];
}

template <int KW>
SHCI_HD void unpack_det(const uint64_t (&k)[KW], int n, uint64_t& a0, uint64_t& a1, uint64_t& b0,
                         uint64_t& b1) {
  uint64_t w[4] = {0ull, 0ull, 0ull, 0ull};
#pragma unroll
  for (int j = 0; j < KW; ++j) w[j] = k[j];
  const uint64_t m0 = (n >= 64) ? ~0ull : ((1ull << n) - 1ull);
  const uint64_t m1 = (n <= 64) ? 0ull : ((n >= 128) ? ~0ull : ((1ull << (n - 64)) - 1ull));
  a0 = w[0] & m0;
  a1 = w[1] & m1;
  uint64_t r0, r1;
  if (n < 64) {
    r0 = (w[0] >> n) | (w[1] << (64 - n));
    r1 = (w[1] >> n) | (w[2] << (64 - n));
  } else {
    const int t = n - 64;
    r0 = t ? ((w[1] >> t) | (w[2] << (64 - t))) : w[1];
    r1 = t ? ((w[2] >> t) | (w[3] << (64 - t))) : w[2];
  }
  b0 = r0 & m0;
  b1 = r1 & m1;
}

// the determinant bits of a key (bits below 2n), other bits cleared
template <int KW>
SHCI_HD void mask_det(uint64_t (&k)[KW], int n) {
#pragma unroll
  for (int j = 0; j < KW; ++j) {
    const int lim = 2 * n - 64 * j;
    k[j] &= (lim >= 64) ? ~0ull : (lim <= 0 ? 0ull : ((1ull << lim) - 1ull));
  }
}

// Hash of the determinant a key holds: the chained finaliser over the
// ceil(2n/64) words of alpha | beta << n (sample id and flag excluded), so the
// value depends on the determinant and n only, not on the key width.
// Buckets, in-bucket order, the V lookup and the hash batches of P all use it.
template <int KW>
SHCI_HD uint64_t det_hash(const uint64_t (&k)[KW], int n) {
  uint64_t m[KW];
#pragma unroll
  for (int j = 0; j < KW; ++j) m[j] = k[j];
  mask_det<KW>(m, n);
  const int dw = (2 * n + 63) >> 6;
  uint64_t h = 0x243f6a8885a308d3ull;
#pragma unroll
  for (int j = 0; j < KW; ++j) h = (j < dw) ? fmix64(h ^ m[j]) : h;
  return h;
}

// mask of the grouping bits (everything below the auxiliary flag)
// (per-word masks selected by value, so the word index never becomes a
// dynamic index into the key array)
template <int KW>
SHCI_HD void clear_aux(uint64_t (&k)[KW], int auxbit) {
  const int w = auxbit >> 6;
  const uint64_t m = ~(1ull << (auxbit & 63));
#pragma unroll
  for (int j = 0; j < KW; ++j) k[j] &= (j == w) ? m : ~0ull;
}

template <int KW>
SHCI_HD bool aux_set(const uint64_t (&k)[KW], int auxbit) {
  const int w = auxbit >> 6;
  const uint64_t m = 1ull << (auxbit & 63);
  uint64_t r = 0;
#pragma unroll
  for (int j = 0; j < KW; ++j) r |= (j == w) ? (k[j] & m) : 0ull;
  return r != 0ull;
}

// k -> (hi, lo) with k = hi (hi + 1) / 2 + lo, 0 <= lo <= hi (the triangle
// with its diagonal); the square root only seeds hi, integer steps make it exact
SHCI_HD void tri_split(int64_t k, int64_t& hi, int64_t& lo) {
  int64_t h = (int64_t)((sqrt(8.0 * (double)k + 1.0) - 1.0) * 0.5);
  while (h * (h + 1) / 2 > k) --h;
  while ((h + 1) * (h + 2) / 2 <= k) ++h;
  hi = h;
  lo = k - h * (h + 1) / 2;
}

// ---------------------------------------------------------------------------
// Spin strings (2 words) and fermion signs.
// ---------------------------------------------------------------------------
SHCI_HD void low_mask(int x, uint64_t& m0, uint64_t& m1) {
  // bits [0, x), 0 <= x <= 128
  if (x >= 64) {
    m0 = ~0ull;
    m1 = (x >= 128) ? ~0ull : ((1ull << (x - 64)) - 1ull);
  } else {
    m0 = (1ull << x) - 1ull;
    m1 = 0ull;
  }
}

// occupied orbitals of (s0,s1) strictly between p and r
SHCI_HD int between(uint64_t s0, uint64_t s1, int p, int r) {
  int lo = p < r ? p : r, hi = p < r ? r : p;
  uint64_t h0, h1, l0, l1;
  low_mask(hi, h0, h1);
  low_mask(lo + 1, l0, l1);
  return __builtin_popcountll(s0 & h0 & ~l0) + __builtin_popcountll(s1 & h1 & ~l1);
}

SHCI_HD bool occ(uint64_t s0, uint64_t s1, int p) {
  return ((p < 64 ? s0 : s1) >> (p & 63)) & 1ull;
}

SHCI_HD void flip(uint64_t& s0, uint64_t& s1, int p) {
  const uint64_t b = 1ull << (p & 63);
  s0 ^= (p < 64) ? b : 0ull;
  s1 ^= (p < 64) ? 0ull : b;
}

// ---------------------------------------------------------------------------
// Wave helpers
// ---------------------------------------------------------------------------
SHCI_DEV int lane_id() { return __lane_id(); }

SHCI_DEV uint64_t ballot(bool p) { return __ballot(p); }

// number of set bits of m below this lane
SHCI_DEV int rank_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// compensated addition (Knuth TwoSum) in binary32
SHCI_DEV void two_sum_f32(float& s, float& comp, float x) {
  float t = s + x;
  float bp = t - s;
  float err = (s - (t - bp)) + (x - bp);
  s = t;
  comp += err;
}

}  // namespace shci
