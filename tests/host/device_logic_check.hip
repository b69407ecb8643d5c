// Host-side check of device helper logic (compiled for the host with hipcc):
//  * closed-form key packing / unpacking against a bit-by-bit reference,
//  * H_aa: the reference-relative list formula, the single-word loop form and
//    the plain sum against a direct double loop over occupied pairs.
// Exit status 0 on success.
#define SHCI_DEV __host__ __device__ inline
#include "../../paper_1809_04600_amd/csrc/diag.hpp"
#include "../../paper_1809_04600_amd/csrc/hc.hpp"

#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

using namespace shci;

template <int KW>
static void ref_pack(uint64_t (&k)[KW], uint64_t a0, uint64_t a1, uint64_t b0, uint64_t b1, int n) {
  for (int j = 0; j < KW; ++j) k[j] = 0;
  for (int p = 0; p < n; ++p) {
    if ((p < 64 ? a0 >> p : a1 >> (p - 64)) & 1) k[p >> 6] |= 1ull << (p & 63);
    if ((p < 64 ? b0 >> p : b1 >> (p - 64)) & 1) {
      const int q = n + p;
      k[q >> 6] |= 1ull << (q & 63);
    }
  }
}

static int check_pack() {
  std::mt19937_64 g(1);
  int bad = 0;
  for (int n = 1; n <= 127; ++n)
    for (int it = 0; it < 500; ++it) {
      const uint64_t m0 = n >= 64 ? ~0ull : ((1ull << n) - 1);
      const uint64_t m1 = n <= 64 ? 0 : ((1ull << (n - 64)) - 1);
      const uint64_t a0 = g() & m0, a1 = g() & m1, b0 = g() & m0, b1 = g() & m1;
      uint64_t k[4], r[4];
      pack_det<4>(k, a0, a1, b0, b1, n);
      ref_pack<4>(r, a0, a1, b0, b1, n);
      for (int j = 0; j < 4; ++j) bad += k[j] != r[j];
      uint64_t x0, x1, y0, y1;
      unpack_det<4>(k, n, x0, x1, y0, y1);
      bad += (x0 != a0) + (x1 != a1) + (y0 != b0) + (y1 != b1);
    }
  printf("pack/unpack mismatches: %d\n", bad);
  return bad;
}

static int check_diag(int n, int na, int nb, unsigned seed) {
  std::mt19937_64 g(seed);
  std::normal_distribution<double> N(0, 1);
  std::vector<double> h(n), J(n * n), K(n * n);
  for (int p = 0; p < n; ++p) h[p] = -2 + 0.1 * p + 0.01 * N(g);
  for (int p = 0; p < n; ++p)
    for (int q = p; q < n; ++q) {
      const double v = 0.1 + 0.02 * N(g), k = 0.02 * std::fabs(N(g));
      J[p * n + q] = J[q * n + p] = v;
      K[p * n + q] = K[q * n + p] = (p == q ? v : k);
    }
  const DiagLayout L = DiagLayout::make(n);
  std::vector<double> tab(L.total);
  for (int p = 0; p < n; ++p) tab[p] = h[p];
  for (int q = 0; q < n; ++q)
    for (int p = 0; p <= q; ++p) {
      tab[L.oj + q * (q + 1) / 2 + p] = J[p * n + q];
      if (p < q) tab[L.os + q * (q - 1) / 2 + p] = J[p * n + q] - K[p * n + q];
    }
  auto bit = [](const uint64_t* s, int p) { return (s[p >> 6] >> (p & 63)) & 1ull; };
  auto direct = [&](const uint64_t* a, const uint64_t* b) {
    double e = 0;
    for (int p = 0; p < n; ++p) e += (bit(a, p) ? h[p] : 0) + (bit(b, p) ? h[p] : 0);
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        if (bit(a, p) && bit(a, q)) e += J[p * n + q] - K[p * n + q];
        if (bit(b, p) && bit(b, q)) e += J[p * n + q] - K[p * n + q];
      }
    for (int p = 0; p < n; ++p)
      for (int q = 0; q < n; ++q)
        if (bit(a, p) && bit(b, q)) e += J[p * n + q];
    return e;
  };
  auto rand_string = [&](int ne, uint64_t* s) {
    s[0] = s[1] = 0;
    int c = 0;
    while (c < ne) {
      const int p = (int)(g() % n);
      if (!bit(s, p)) {
        s[p >> 6] |= 1ull << (p & 63);
        ++c;
      }
    }
  };
  // random source i: F of both spins and H_ii as in the generator, then the
  // H_aa of random singles and doubles (all three spin cases) by the update
  auto occ_list = [&](const uint64_t* s, uint8_t* out) {
    int c = 0;
    for (int p = 0; p < n; ++p)
      if (bit(s, p)) out[c++] = (uint8_t)p;
    return c;
  };
  auto pick = [&](const uint64_t* s, bool occupied) {
    for (;;) {
      const int p = (int)(g() % n);
      if ((bit(s, p) != 0) == occupied) return p;
    }
  };
  double maxerr = 0.0;
  int nchk = 0;
  for (int it = 0; it < 400; ++it) {
    uint64_t a[2], b[2];
    rand_string(na, a);
    rand_string(nb, b);
    uint8_t oa[128], ob[128];
    const int ca = occ_list(a, oa), cb = occ_list(b, ob);
    std::vector<double> F(256, 0.0);
    double part = 0.0;
    for (int x = 0; x < n; ++x) {
      fock_diag2(tab.data(), L, x, oa, ca, ob, cb, F[x], F[128 + x]);
      if (bit(a, x)) part += h[x] + F[x];
      if (bit(b, x)) part += h[x] + F[128 + x];
    }
    const double hii = 0.5 * part;
    maxerr = std::fmax(maxerr, std::fabs(hii - direct(a, b)));
    for (int rep = 0; rep < 8; ++rep) {
      uint64_t xa[2] = {a[0], a[1]}, xb[2] = {b[0], b[1]};
      auto flip2 = [](uint64_t* s, int p) { s[p >> 6] ^= 1ull << (p & 63); };
      double d = 0.0;
      const int kind = (int)(g() % 5);  // singles alpha/beta, doubles aa/bb/ab
      if (kind < 2) {
        const uint64_t* s = kind ? b : a;
        if ((kind ? nb : na) == 0 || (kind ? nb : na) == n) continue;
        const int p = pick(s, true), r = pick(s, false);
        d = en_single(F.data() + (kind ? 128 : 0), tab.data(), L, p, r);
        flip2(kind ? xb : xa, p);
        flip2(kind ? xb : xa, r);
      } else if (kind < 4) {
        const bool beta = kind == 3;
        const int ne_s = beta ? nb : na;
        if (ne_s < 2 || n - ne_s < 2) continue;
        const uint64_t* s = beta ? b : a;
        const int p = pick(s, true);
        int q = pick(s, true);
        while (q == p) q = pick(s, true);
        const int r = pick(s, false);
        int t = pick(s, false);
        while (t == r) t = pick(s, false);
        const double* Fs = F.data() + (beta ? 128 : 0);
        d = en_double(Fs, Fs, tab.data(), L, p, q, r, t, true);
        uint64_t* xs = beta ? xb : xa;
        flip2(xs, p);
        flip2(xs, q);
        flip2(xs, r);
        flip2(xs, t);
      } else {
        if (na == 0 || nb == 0 || na == n || nb == n) continue;
        const int p = pick(a, true), r = pick(a, false);
        const int q = pick(b, true), t = pick(b, false);
        d = en_double(F.data(), F.data() + 128, tab.data(), L, p, q, r, t, false);
        flip2(xa, p);
        flip2(xa, r);
        flip2(xb, q);
        flip2(xb, t);
      }
      maxerr = std::fmax(maxerr, std::fabs((hii + d) - direct(xa, xb)));
      ++nchk;
    }
  }
  printf("H_aa update n=%d na=%d nb=%d (%d excitations): max |error| %.3g\n", n, na, nb, nchk, maxerr);
  return maxerr > 1e-11;
}

// triangle split, the folded integral table of the H c kernels, and the fold
// prefilter's bound
static int check_hc_helpers() {
  int bad = 0;
  for (int64_t k = 0; k < 40000000; k += (k < 100000 ? 1 : 7)) {
    int64_t hi, lo;
    tri_split(k, hi, lo);
    bad += !(lo >= 0 && lo <= hi && hi * (hi + 1) / 2 + lo == k);
  }
  const int n = 9;
  std::mt19937_64 g(5);
  std::normal_distribution<double> N(0, 1);
  std::vector<double> eri((size_t)n * n * n * n);
  for (int p = 0; p < n; ++p)
    for (int q = 0; q <= p; ++q)
      for (int r = 0; r < n; ++r)
        for (int s = 0; s <= r; ++s) {
          if (p * (p + 1) / 2 + q < r * (r + 1) / 2 + s) continue;
          const double v = N(g);
          const int idx[8][4] = {{p, q, r, s}, {q, p, r, s}, {p, q, s, r}, {q, p, s, r},
                                 {r, s, p, q}, {s, r, p, q}, {r, s, q, p}, {s, r, q, p}};
          for (auto& t : idx) eri[((size_t)(t[0] * n + t[1]) * n + t[2]) * n + t[3]] = v;
        }
  const int64_t npair = n * (n + 1) / 2, tot = npair * (npair + 1) / 2;
  std::vector<double> g8(tot);
  for (int64_t k = 0; k < tot; ++k) {
    int64_t P, Q, p, q, r, s;
    tri_split(k, P, Q);
    tri_split(P, p, q);
    tri_split(Q, r, s);
    g8[k] = eri[((size_t)(p * n + q) * n + r) * n + s];
  }
  for (int p = 0; p < n; ++p)
    for (int q = 0; q < n; ++q)
      for (int r = 0; r < n; ++r)
        for (int s = 0; s < n; ++s)
          bad += eri_g8(g8.data(), p, q, r, s) != eri[((size_t)(p * n + q) * n + r) * n + s];
  for (int it = 0; it < 100000; ++it) {
    const uint64_t a0 = g(), a1 = g() & 0xfff, b0 = a0 ^ (1ull << (g() % 64)) ^ (1ull << (g() % 64)),
                   b1 = a1 ^ ((g() & 1) ? (1ull << (g() % 12)) : 0);
    const int full = __builtin_popcountll(a0 ^ b0) + __builtin_popcountll(a1 ^ b1);
    bad += __builtin_popcount(fold32(a0, a1) ^ fold32(b0, b1)) > full;
  }
  printf("H c helpers: %d mismatches\n", bad);
  return bad;
}

int main() {
  int bad = check_pack();
  bad += check_hc_helpers();
  bad += check_diag(10, 3, 3, 1);
  bad += check_diag(40, 8, 8, 2);
  bad += check_diag(76, 14, 14, 3);
  bad += check_diag(100, 5, 4, 4);
  return bad ? 1 : 0;
}
