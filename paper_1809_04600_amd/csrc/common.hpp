// Shared device/host helpers of the PT2 library (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define SHCI_DEV __device__ __forceinline__

namespace shci {

constexpr int WAVE = 64;

// ---------------------------------------------------------------------------
// Hashing: murmur3's 64-bit finaliser chained over the key words.  Used for
// the bucket id (top bits), the in-bucket sort key (next 32 bits) and the
// variational-space hash set.
// ---------------------------------------------------------------------------
SHCI_DEV uint64_t fmix64(uint64_t k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdull;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ull;
  k ^= k >> 33;
  return k;
}

template <int KW>
SHCI_DEV uint64_t hash_key(const uint64_t (&k)[KW]) {
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
SHCI_DEV void put_bits(uint64_t (&k)[KW], uint64_t v0, uint64_t v1, int off) {
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
SHCI_DEV void get_bits(const uint64_t (&k)[KW], int off, int nbits, uint64_t& v0, uint64_t& v1) {
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

template <int KW>
SHCI_DEV void pack_det(uint64_t (&k)[KW], uint64_t a0, uint64_t a1, uint64_t b0, uint64_t b1,
                       int n) {
#pragma unroll
  for (int j = 0; j < KW; ++j) k[j] = 0;
  put_bits<KW>(k, a0, a1, 0);
  put_bits<KW>(k, b0, b1, n);
}

template <int KW>
SHCI_DEV void unpack_det(const uint64_t (&k)[KW], int n, uint64_t& a0, uint64_t& a1, uint64_t& b0,
                         uint64_t& b1) {
  get_bits<KW>(k, 0, n, a0, a1);
  get_bits<KW>(k, n, n, b0, b1);
}

// mask of the grouping bits (everything below the auxiliary flag)
template <int KW>
SHCI_DEV void clear_aux(uint64_t (&k)[KW], int auxbit) {
#pragma unroll
  for (int j = 0; j < KW; ++j)
    if (j == (auxbit >> 6)) k[j] &= ~(1ull << (auxbit & 63));
}

template <int KW>
SHCI_DEV bool aux_set(const uint64_t (&k)[KW], int auxbit) {
  bool r = false;
#pragma unroll
  for (int j = 0; j < KW; ++j)
    if (j == (auxbit >> 6)) r = (k[j] >> (auxbit & 63)) & 1ull;
  return r;
}

// ---------------------------------------------------------------------------
// Spin strings (2 words) and fermion signs.
// ---------------------------------------------------------------------------
SHCI_DEV void low_mask(int x, uint64_t& m0, uint64_t& m1) {
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
SHCI_DEV int between(uint64_t s0, uint64_t s1, int p, int r) {
  int lo = p < r ? p : r, hi = p < r ? r : p;
  uint64_t h0, h1, l0, l1;
  low_mask(hi, h0, h1);
  low_mask(lo + 1, l0, l1);
  return __popcll(s0 & h0 & ~l0) + __popcll(s1 & h1 & ~l1);
}

SHCI_DEV bool occ(uint64_t s0, uint64_t s1, int p) {
  return ((p < 64 ? s0 : s1) >> (p & 63)) & 1ull;
}

SHCI_DEV void flip(uint64_t& s0, uint64_t& s1, int p) {
  if (p < 64)
    s0 ^= 1ull << p;
  else
    s1 ^= 1ull << (p - 64);
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
