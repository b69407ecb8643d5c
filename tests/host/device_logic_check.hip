// Host-side check of device helper logic (compiled for the host with hipcc):
//  * closed-form key packing / unpacking against a bit-by-bit reference,
//  * H_aa: the reference-relative list formula, the single-word loop form and
//    the plain sum against a direct double loop over occupied pairs.
// Exit status 0 on success.
#define SHCI_DEV __host__ __device__ inline
#include "../../paper_1809_04600_amd/csrc/diag.hpp"

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
  // reference det R: lowest orbitals, then F_p(sigma) and E(R) as on the device
  uint64_t ra[2] = {0, 0}, rb[2] = {0, 0};
  for (int p = 0; p < na; ++p) ra[p >> 6] |= 1ull << (p & 63);
  for (int p = 0; p < nb; ++p) rb[p >> 6] |= 1ull << (p & 63);
  for (int t = 0; t < 2 * n; ++t) {
    const int p = t % n, sp = t / n;
    const uint64_t* same = sp ? rb : ra;
    const uint64_t* oth = sp ? ra : rb;
    double v = h[p];
    for (int q = 0; q < n; ++q) {
      if (bit(same, q) && q != p) v += J[p * n + q] - K[p * n + q];
      if (bit(oth, q)) v += J[p * n + q];
    }
    tab[L.of + t] = v;
  }
  tab[L.oe] = diag_plain(ra[0], ra[1], rb[0], rb[1], tab.data(), L);
  double maxerr = std::fabs(tab[L.oe] - direct(ra, rb));
  DiagTab<false> T;
  T.g = tab.data();
  T.L = L;
  const uint64_t r[4] = {ra[0], ra[1], rb[0], rb[1]};
  for (int it = 0; it < 5000; ++it) {
    uint64_t a[2], b[2];
    rand_string(na, a);
    rand_string(nb, b);
    const double e0 = direct(a, b);
    maxerr = std::fmax(maxerr, std::fabs(diag_energy<false>(a[0], a[1], b[0], b[1], r, T, na + nb) - e0));
    if (n <= 64) maxerr = std::fmax(maxerr, std::fabs(diag_energy1<false>(a[0], b[0], r[0], r[2], T, 0) - e0));
  }
  printf("H_aa n=%d na=%d nb=%d: max |error| %.3g\n", n, na, nb, maxerr);
  return maxerr > 1e-11;
}

int main() {
  int bad = check_pack();
  bad += check_diag(10, 3, 3, 1);
  bad += check_diag(40, 8, 8, 2);
  bad += check_diag(76, 14, 14, 3);
  bad += check_diag(100, 5, 4, 4);
  return bad ? 1 : 0;
}
