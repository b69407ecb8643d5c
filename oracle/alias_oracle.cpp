// CPU reference for the sampling of variational determinants (TEST
// INFRASTRUCTURE): the alias table of p_i = |c_i| / sum_j |c_j| and the
// seeded draws of the stochastic PT2 samples.  Used only by the tests, the
// scripts that write stored expected values and the smoke check; shares no
// code with the GPU library.
//
// Paper, section II.B: determinants of V are drawn with replacement with
// probability p_i = |c_i| / sum_j |c_j| (sampling-probability equation), by
// the alias method (Walker; Kronmal and Peterson).  The paper gives no
// construction details; the readings used here:
//
//  1. Integer masses.  With m = max_i |c_i| = f 2^E (f in [0.5, 1)), b the
//     number of bits of N - 1 (0 for N = 1) and K = 127 - 2b, the weight of i
//     is the exact integer W_i = floor(|c_i| 2^(K - E)) (an exact scaling of
//     the binary64 value, truncated below 2^(E - K)).  Bucket capacity
//     T = sum W_i; item mass a_i = N W_i; sum a_i = N T.  All of it is exact in
//     128-bit unsigned arithmetic, and so is every sum of masses or of bucket
//     deficits (at most N T < 2^127), so the table does not depend on the
//     order of any sum.
//  2. Table (Vose's method, sweep order).  Items with a_i < T are light, the
//     others heavy; both in increasing index order.  The current heavy covers
//     the lights one after the other; whenever its remaining mass r is no
//     longer above T it becomes light: its own bucket keeps it with r and
//     aliases the next heavy, which first covers that bucket's deficit T - r.
//     The last heavy keeps r = T.  A bucket whose own mass is T aliases itself.
//  3. Thresholds.  Bucket k picks itself when a 64-bit uniform v satisfies
//     v < P_k = floor(prob_k 2^64 / T) (P_k = 2^64 - 1 when prob_k = T), else
//     its alias.
//  4. Draws.  SplitMix64 (Steele, Lea and Flood, 2014): output number m
//     (m >= 1) of the generator seeded with s is mix(s + m * 0x9e3779b97f4a7c15),
//     mix the published finaliser.  Draw k of sample j uses t = j N_d + k:
//     r1 = output 2t + 1 picks the bucket floor(r1 N / 2^64), r2 = output 2t + 2
//     is compared with its threshold.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

namespace {

typedef unsigned __int128 u128;

thread_local char a_err[256] = "";

uint64_t splitmix_output(uint64_t seed, uint64_t m) {
  uint64_t z = seed + m * 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

// exact floor(|x| * 2^sh) of a finite binary64 value, as an integer below 2^127
u128 scaled_weight(double x, int sh) {
  x = std::fabs(x);
  if (x == 0.0) return 0;
  int e;
  const double f = std::frexp(x, &e);  // x = f 2^e, f in [0.5, 1)
  const uint64_t mant = (uint64_t)std::ldexp(f, 53);  // exact 53-bit integer
  const int s = e - 53 + sh;  // x 2^sh = mant 2^s
  if (s >= 0) return (u128)mant << s;
  if (s <= -64) return 0;
  return (u128)(mant >> (-s));
}

int bits_of(int64_t n) {  // number of bits of n - 1
  int b = 0;
  while (((int64_t)1 << b) < n) ++b;
  return b;
}

struct Table {
  std::vector<u128> a;      // masses N W_i
  u128 T = 0;               // bucket capacity
  std::vector<u128> prob;   // own mass of each bucket
  std::vector<uint32_t> alias;
};

int build(const double* c, int64_t n, Table& t) {
  if (n < 1 || n >= ((int64_t)1 << 32) - 1) {
    snprintf(a_err, sizeof a_err, "n must be in [1, 2^32 - 1)");
    return -1;
  }
  double m = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    if (!std::isfinite(c[i])) {
      snprintf(a_err, sizeof a_err, "c[%lld] is not finite", (long long)i);
      return -5;
    }
    m = std::max(m, std::fabs(c[i]));
  }
  if (!(m > 0.0)) {
    snprintf(a_err, sizeof a_err, "all coefficients are zero");
    return -5;
  }
  int E;
  std::frexp(m, &E);
  const int K = 127 - 2 * bits_of(n);
  t.a.assign(n, 0);
  t.T = 0;
  for (int64_t i = 0; i < n; ++i) {
    const u128 w = scaled_weight(c[i], K - E);
    t.T += w;
    t.a[i] = w * (u128)n;
  }
  std::vector<int64_t> light, heavy;
  for (int64_t i = 0; i < n; ++i) (t.a[i] < t.T ? light : heavy).push_back(i);
  t.prob.assign(n, 0);
  t.alias.assign(n, 0);
  size_t j = 0;
  u128 r = t.a[heavy[0]];
  auto retire = [&]() {  // the current heavy is no longer above T
    t.prob[heavy[j]] = r;
    t.alias[heavy[j]] = (uint32_t)heavy[j + 1];
    const u128 deficit = t.T - r;
    ++j;
    r = t.a[heavy[j]] - deficit;
  };
  for (int64_t l : light) {
    while (r <= t.T && j + 1 < heavy.size()) retire();
    t.prob[l] = t.a[l];
    t.alias[l] = (uint32_t)heavy[j];
    r -= t.T - t.a[l];
  }
  while (j + 1 < heavy.size()) retire();
  t.prob[heavy[j]] = r;
  t.alias[heavy[j]] = (uint32_t)heavy[j];
  for (int64_t i = 0; i < n; ++i)
    if (t.prob[i] == t.T) t.alias[i] = (uint32_t)i;
  return 0;
}

uint64_t threshold(u128 prob, u128 T) {
  if (prob >= T) return ~0ull;
  u128 rem = prob;
  uint64_t q = 0;
  for (int k = 0; k < 64; ++k) {  // long division of prob 2^64 by T
    rem <<= 1;
    q <<= 1;
    if (rem >= T) {
      rem -= T;
      q |= 1;
    }
  }
  return q;
}

}  // namespace

extern "C" {

const char* oracle_alias_last_error() { return a_err; }

uint64_t oracle_splitmix64(uint64_t seed, uint64_t m) { return splitmix_output(seed, m); }

// Alias table of p_i = |c_i| / sum |c|: thresholds P [n] (u64), aliases [n];
// mass_lo/hi [n] receive the integer masses a_i and t_lohi[2] the capacity T
// (for the tests' exact checks); any of these three may be NULL.
int oracle_alias_table(const double* c, int64_t n, uint64_t* P, uint32_t* alias, uint64_t* mass_lo,
                       uint64_t* mass_hi, uint64_t* own_lo, uint64_t* own_hi, uint64_t* t_lohi) {
  Table t;
  const int st = build(c, n, t);
  if (st) return st;
  for (int64_t i = 0; i < n; ++i) {
    if (P) P[i] = threshold(t.prob[i], t.T);
    if (alias) alias[i] = t.alias[i];
    if (mass_lo) mass_lo[i] = (uint64_t)t.a[i];
    if (mass_hi) mass_hi[i] = (uint64_t)(t.a[i] >> 64);
    if (own_lo) own_lo[i] = (uint64_t)t.prob[i];
    if (own_hi) own_hi[i] = (uint64_t)(t.prob[i] >> 64);
  }
  if (t_lohi) {
    t_lohi[0] = (uint64_t)t.T;
    t_lohi[1] = (uint64_t)(t.T >> 64);
  }
  return 0;
}

// Draws [ns][nd] of the stochastic samples from the seed (reading 4 above).
int oracle_alias_draws(const double* c, int64_t n, uint64_t seed, int32_t ns, int32_t nd, uint32_t* draws) {
  if (ns < 1 || nd < 1) {
    snprintf(a_err, sizeof a_err, "need n_samples >= 1 and n_draws >= 1");
    return -1;
  }
  Table t;
  const int st = build(c, n, t);
  if (st) return st;
  std::vector<uint64_t> P(n);
  for (int64_t i = 0; i < n; ++i) P[i] = threshold(t.prob[i], t.T);
  for (int64_t s = 0; s < ns; ++s)
    for (int64_t k = 0; k < nd; ++k) {
      const uint64_t u = (uint64_t)(s * nd + k);
      const uint64_t r1 = splitmix_output(seed, 2 * u + 1);
      const uint64_t r2 = splitmix_output(seed, 2 * u + 2);
      const uint64_t b = (uint64_t)(((u128)r1 * (u128)(uint64_t)n) >> 64);
      draws[s * nd + k] = r2 < P[b] ? (uint32_t)b : t.alias[b];
    }
  return 0;
}

}  // extern "C"
