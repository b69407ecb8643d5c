// Sampling of variational determinants with p_i = |c_i| / sum_j |c_j>
// (paper, section II.B, sampling-probability equation) by the alias method,
// built and drawn on the device.
//
// The table is defined on exact integers so that it does not depend on the
// order of any sum (and equals, bit for bit, what a sequential construction
// gives):
//   - weights W_i = floor(|c_i| 2^(K - E)), with 2^(E-1) <= max|c| < 2^E and
//     K = 127 - 2 bits(N - 1): an exact scaling of the binary64 value,
//     truncated below 2^(E - K); masses a_i = N W_i, bucket capacity
//     T = sum W_i; every prefix sum of masses or deficits stays below
//     N T < 2^127 (128-bit unsigned);
//   - Vose's method in sweep order: lights (a_i < T) and heavies in index
//     order; the current heavy covers lights until its remaining mass is no
//     longer above T, then its own bucket keeps that remainder and aliases the
//     next heavy.  With D_k the deficit T - a of the first k lights summed and
//     X_j the excess a - T of heavies 0..j summed, light k is aliased to the
//     first heavy j with X_j > D_k, and heavy j keeps X_j + T - D_m with m the
//     first index where D_m >= X_j; so the table comes from two prefix sums and
//     binary searches;
//   - threshold P_k = floor(own_k 2^64 / T) (all ones when own_k = T; such a
//     bucket aliases itself);
//   - draw k of sample s: t = s N_d + k, r1 = SplitMix64 output 2t + 1 picks
//     bucket floor(r1 N / 2^64), r2 = output 2t + 2 keeps it when r2 < P.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace shci {

typedef unsigned __int128 u128;

// SplitMix64 (Steele, Lea and Flood 2014): output number m of the generator
// seeded with `seed`
SHCI_HD uint64_t splitmix64_out(uint64_t seed, uint64_t m) {
  uint64_t z = seed + m * 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

// exact floor(|x| 2^sh) of a finite double, from its exponent and mantissa bits
SHCI_HD u128 alias_weight(double x, int sh) {
  const uint64_t b = __builtin_bit_cast(uint64_t, x) & 0x7fffffffffffffffull;
  if (b == 0) return 0;
  const int ebits = (int)(b >> 52);
  uint64_t mant = b & ((1ull << 52) - 1);
  int e2;  // x = mant 2^e2 with mant an integer
  if (ebits == 0) {
    e2 = -1074;
  } else {
    mant |= 1ull << 52;
    e2 = ebits - 1075;
  }
  const int s = e2 + sh;
  if (s >= 0) return (u128)mant << s;
  if (s <= -64) return 0;
  return (u128)(mant >> (-s));
}

struct AliasArgs {
  const double* c;
  int64_t n;
  int K;              // 127 - 2 bits(n - 1)
  uint64_t* maxbits;  // [1] bits of max |c| (positive doubles order like their bits)
  u128* w;            // [n] weights
  u128* tsum;         // [nblk] partial sums of W
  u128* tot;          // [1] T
  uint32_t* isl;      // [n] 1 if light
  uint64_t* lpos;     // [n + 1] exclusive prefix of isl (rank among lights), lights at [n]
  uint32_t* hidx;     // [n] heavies in index order
  u128* dl;           // [n + 1] deficit of each light (0 for heavies), then its exclusive prefix
  u128* xh;           // [n + 1] excess of each heavy (0 for lights), then its exclusive prefix
  uint64_t* thr;      // [n] out: thresholds
  uint32_t* alias;    // [n] out
  uint32_t* flag;     // error bits: 2 non-finite c, 64 all zero
};
__global__ void k_alias_max(const double* c, int64_t n, uint64_t* maxbits, uint32_t* flag) {
  uint64_t m = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double v = c[i];
    if (!(v - v == 0.0)) atomicOr(flag, 2u);
    const uint64_t b = __builtin_bit_cast(uint64_t, v) & 0x7fffffffffffffffull;
    m = b > m ? b : m;
  }
  for (int o = 32; o > 0; o >>= 1) {
    const uint64_t x = __shfl_xor(m, o);
    m = x > m ? x : m;
  }
  if ((threadIdx.x & 63) == 0 && m) atomicMax((unsigned long long*)maxbits, (unsigned long long)m);
}

// weights and per-block partial sums of W (256 threads, 16 items each)
__global__ void __launch_bounds__(256) k_alias_weights(AliasArgs a) {
  __shared__ u128 sh[256];
  const uint64_t mb = *a.maxbits;
  const int emax = (int)(mb >> 52);  // biased exponent of max |c|
  // max|c| in [2^(E-1), 2^E): E = emax - 1022 for normal values
  int E;
  if (emax == 0) {
    const int lz = __clzll(mb);  // subnormal: value = mb 2^-1074, mb < 2^52
    E = (64 - lz) - 1074;
  } else {
    E = emax - 1022;
  }
  const int sh_bits = a.K - E;
  u128 s = 0;
  const int64_t base = (int64_t)blockIdx.x * 4096 + threadIdx.x;
  for (int j = 0; j < 16; ++j) {
    const int64_t i = base + (int64_t)j * 256;
    if (i < a.n) {
      const u128 w = alias_weight(a.c[i], sh_bits);
      a.w[i] = w;
      s += w;
    }
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) a.tsum[blockIdx.x] = sh[0];
}

__global__ void __launch_bounds__(256) k_alias_total(AliasArgs a, int64_t nblk) {
  __shared__ u128 sh[256];
  u128 s = 0;
  for (int64_t b = threadIdx.x; b < nblk; b += 256) s += a.tsum[b];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    *a.tot = sh[0];
    if (sh[0] == 0) atomicOr(a.flag, 64u);
  }
}

// light flags and, indexed by determinant, deficits of lights and excesses
// of heavies (prefix sums over the whole index range give the sweep's D and X)
__global__ void k_alias_classify(AliasArgs a) {
  const u128 T = *a.tot;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < a.n; i += (int64_t)gridDim.x * blockDim.x) {
    const u128 m = a.w[i] * (u128)(uint64_t)a.n;
    const bool light = m < T;
    a.isl[i] = light ? 1u : 0u;
    a.dl[i] = light ? T - m : (u128)0;
    a.xh[i] = light ? (u128)0 : m - T;
  }
}

// heavies in index order
__global__ void k_alias_heavies(AliasArgs a) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < a.n; i += (int64_t)gridDim.x * blockDim.x)
    if (!a.isl[i]) a.hidx[(uint64_t)i - a.lpos[i]] = (uint32_t)i;
}

SHCI_DEV uint64_t alias_threshold(u128 own, u128 T) {
  if (own >= T) return ~0ull;
  u128 rem = own;
  uint64_t q = 0;
  for (int k = 0; k < 64; ++k) {
    rem <<= 1;
    q <<= 1;
    if (rem >= T) {
      rem -= T;
      q |= 1;
    }
  }
  return q;
}

// assembles the table.  dl and xh hold exclusive prefix sums over the index
// range (entry n = total): the D of a light is dl at its index; X_j, the
// excess of heavies up to and including heavy i, is xh[i + 1].
__global__ void k_alias_assemble(AliasArgs a) {
  const u128 T = *a.tot;
  const int64_t n = a.n;
  const int64_t nh = n - (int64_t)a.lpos[n];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    u128 own;
    uint32_t al;
    if (a.isl[i]) {
      // the first heavy whose X exceeds this light's D: the first index h
      // with xh[h + 1] > D (the prefix only grows at heavies)
      const u128 d = a.dl[i];
      int64_t lo = 0, hi = n - 1;
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (a.xh[mid + 1] > d)
          hi = mid;
        else
          lo = mid + 1;
      }
      own = a.w[i] * (u128)(uint64_t)n;
      al = (uint32_t)lo;
    } else {
      // this heavy keeps X + T - D_m, D_m the first light prefix (or the
      // total) not below X: the first index m with dl[m] >= X
      const u128 x = a.xh[i + 1];
      int64_t lo = 0, hi = n;
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (a.dl[mid] >= x)
          hi = mid;
        else
          lo = mid + 1;
      }
      own = x + T - a.dl[lo];
      const int64_t j = i - (int64_t)a.lpos[i];  // rank among heavies
      al = (own >= T || j + 1 >= nh) ? (uint32_t)i : a.hidx[j + 1];
    }
    a.thr[i] = alias_threshold(own, T);
    a.alias[i] = al;
  }
}

// draws [ns][nd] from the table
__global__ void k_alias_draw(const uint64_t* thr, const uint32_t* alias, int64_t n, uint64_t seed, int32_t ns,
                             int32_t nd, uint32_t* draws) {
  const int64_t tot = (int64_t)ns * nd;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t r1 = splitmix64_out(seed, 2 * (uint64_t)t + 1);
    const uint64_t r2 = splitmix64_out(seed, 2 * (uint64_t)t + 2);
    const uint64_t b = __umul64hi(r1, (uint64_t)n);
    draws[t] = r2 < thr[b] ? (uint32_t)b : alias[b];
  }
}

}  // namespace shci
