// Epstein-Nesbet diagonal H_aa (partition equation) on the device.
//
// Packed table layout (doubles), built once per integral set, with the
// reference part rewritten per call:
//   [0, n)                     h_pp
//   [n, n + n(n+1)/2)          (pp|qq), p <= q, at q(q+1)/2 + p
//   [.., + n(n-1)/2)           (pp|qq) - (pq|qp), p < q, at q(q-1)/2 + p
//   [.., + 2n)                 F_p(sigma) of the reference determinant R:
//                              h_pp + sum_{q in R_sigma, q != p} [(pp|qq)-(pq|qp)]
//                                   + sum_{q in R_other} (pp|qq)
//   [.., + 1)                  E(R)
// With particles P = a \ R and holes Q = R \ a (spin orbitals) and W the pair
// energy (J - K for equal spins, J otherwise), an exact rearrangement of the
// sum over occupied pairs gives
//   E(a) = E(R) + sum_{x in P} F_x - sum_{y in Q} F_y - sum_{x in P, y in Q} W_xy
//          + sum_{x<x' in P} W_xx' + sum_{y<y' in Q} W_yy'.
// For a far from R the empty reference is used instead (F = h, E = 0,
// P = a, Q = empty), which is the plain sum over occupied pairs.
#pragma once
#include "common.hpp"

namespace shci {

extern __shared__ double g_lds_tab[];  // dynamic LDS of the reduce kernels

struct DiagLayout {
  int n;
  int oj, os, of, oe, total;
  SHCI_DEV static DiagLayout make(int n) {
    DiagLayout L;
    L.n = n;
    L.oj = n;
    L.os = L.oj + n * (n + 1) / 2;
    L.of = L.os + n * (n - 1) / 2;
    L.oe = L.of + 2 * n;
    L.total = L.oe + 1;
    return L;
  }
};

inline int diag_table_doubles(int n) { return n * n + 3 * n + 1; }

template <bool LDS>
struct DiagTab {
  const double* g;  // global copy (used when LDS == false)
  DiagLayout L;
  SHCI_DEV double at(int i) const {
    if constexpr (LDS)
      return g_lds_tab[i];
    else
      return g[i];
  }
};

SHCI_DEV uint64_t sel4(int m, uint64_t v0, uint64_t v1, uint64_t v2, uint64_t v3) {
  return m == 0 ? v0 : (m == 1 ? v1 : (m == 2 ? v2 : v3));
}

// lowest set bit of the 128-bit value (x0 | x1 << 64), cleared; branch-free
// on values so the pair stays in registers
SHCI_DEV int pop_bit(uint64_t& x0, uint64_t& x1) {
  const bool lo = x0 != 0ull;
  const uint64_t w = lo ? x0 : x1;
  const int p = __builtin_ffsll((long long)w) - 1 + (lo ? 0 : 64);
  const uint64_t wn = w & (w - 1ull);
  x0 = lo ? wn : x0;
  x1 = lo ? x1 : wn;
  return p;
}

// single-word version of pop_bit (all orbitals below 64)
SHCI_DEV int pop_bit1(uint64_t& x) {
  const int p = __builtin_ffsll((long long)x) - 1;
  x &= x - 1ull;
  return p;
}

// H_aa for n <= 64 (one word per spin string); same formula as below.
template <bool LDS>
SHCI_DEV double diag_energy1(uint64_t a, uint64_t b, uint64_t ra, uint64_t rb, const DiagTab<LDS>& T,
                             int ne) {
  const int n = T.L.n;
  const int l = __builtin_popcountll(a & ~ra) + __builtin_popcountll(b & ~rb);
  const bool use_ref = 3 * l * l + 2 * l < ne * (ne + 1) / 2;
  double e = 0.0;
  int fo = T.L.of;
  if (use_ref) {
    e = T.at(T.L.oe);
  } else {
    ra = rb = 0ull;
    fo = 0;
  }
  const uint64_t m0 = a & ~ra, m1 = b & ~rb, m2 = ra & ~a, m3 = rb & ~b;
#pragma unroll 1
  for (int c = 0; c < 4; ++c) {
    uint64_t x = sel4(c, m0, m1, m2, m3);
    const int off = fo + ((use_ref && (c & 1)) ? n : 0);
    double s = 0.0;
    while (x) s += T.at(off + pop_bit1(x));
    e = (c < 2) ? e + s : e - s;
  }
#pragma unroll 1
  for (int c = 0; c < 10; ++c) {
    int xm, ym, kind;
    double sign = 1.0;
    switch (c) {
      case 0: xm = 0; ym = 0; kind = 0; break;
      case 1: xm = 1; ym = 1; kind = 0; break;
      case 2: xm = 0; ym = 1; kind = 2; break;
      case 3: xm = 2; ym = 2; kind = 0; break;
      case 4: xm = 3; ym = 3; kind = 0; break;
      case 5: xm = 2; ym = 3; kind = 2; break;
      case 6: xm = 0; ym = 2; kind = 1; sign = -1.0; break;
      case 7: xm = 1; ym = 3; kind = 1; sign = -1.0; break;
      case 8: xm = 0; ym = 3; kind = 2; sign = -1.0; break;
      default: xm = 1; ym = 2; kind = 2; sign = -1.0; break;
    }
    uint64_t x = sel4(xm, m0, m1, m2, m3);
    const uint64_t yi = sel4(ym, m0, m1, m2, m3);
    if (!(x && yi)) continue;
    double s = 0.0;
    while (x) {
      const int p = pop_bit1(x);
      uint64_t y = (kind == 0) ? (yi & ~((2ull << p) - 1ull)) : yi;
      while (y) {
        const int q = pop_bit1(y);
        const int lo = p < q ? p : q, hi = p < q ? q : p;
        s += (kind == 2) ? T.at(T.L.oj + ((hi * (hi + 1)) >> 1) + lo)
                         : T.at(T.L.os + ((hi * (hi - 1)) >> 1) + lo);
      }
    }
    e += sign * s;
  }
  return e;
}

// With signs s = +1 for particles and -1 for holes, the formula above reads
//   E(a) = E(R) + sum_x s_x F_x + sum_{x<y} s_x s_y W_xy
// over the combined list of at most DL_MAX changed spin orbitals; the loops
// below are fully unrolled and predicated (no divergent bit loops).
constexpr int DL_MAX = 12;

template <bool LDS>
SHCI_DEV double diag_list(uint64_t pa0, uint64_t pa1, uint64_t pb0, uint64_t pb1, uint64_t ha0,
                          uint64_t ha1, uint64_t hb0, uint64_t hb1, const DiagTab<LDS>& T) {
  const int n = T.L.n;
  int orb[DL_MAX];
  int spn[DL_MAX];
  double sg[DL_MAX];
  bool ok[DL_MAX];
#pragma unroll
  for (int k = 0; k < DL_MAX; ++k) {
    // next changed spin orbital, in the order P_alpha, P_beta, Q_alpha, Q_beta
    const bool u0 = (pa0 | pa1) != 0ull, u1 = (pb0 | pb1) != 0ull, u2 = (ha0 | ha1) != 0ull,
               u3 = (hb0 | hb1) != 0ull;
    const int c = u0 ? 0 : (u1 ? 1 : (u2 ? 2 : (u3 ? 3 : 4)));
    uint64_t x0 = c == 0 ? pa0 : (c == 1 ? pb0 : (c == 2 ? ha0 : hb0));
    uint64_t x1 = c == 0 ? pa1 : (c == 1 ? pb1 : (c == 2 ? ha1 : hb1));
    ok[k] = c < 4;
    const int p = ok[k] ? pop_bit(x0, x1) : 0;
    orb[k] = p;
    spn[k] = c & 1;
    sg[k] = c < 2 ? 1.0 : -1.0;
    if (c == 0) { pa0 = x0; pa1 = x1; }
    if (c == 1) { pb0 = x0; pb1 = x1; }
    if (c == 2) { ha0 = x0; ha1 = x1; }
    if (c == 3) { hb0 = x0; hb1 = x1; }
  }
  double e = T.at(T.L.oe);
#pragma unroll
  for (int k = 0; k < DL_MAX; ++k)
    if (ok[k]) e += sg[k] * T.at(T.L.of + spn[k] * n + orb[k]);
#pragma unroll
  for (int k2 = 1; k2 < DL_MAX; ++k2) {
    if (!ok[k2]) continue;
#pragma unroll
    for (int k1 = 0; k1 < k2; ++k1) {
      const int p = orb[k1], q = orb[k2];
      const int lo = p < q ? p : q, hi = p < q ? q : p;
      const bool same = spn[k1] == spn[k2];
      const double w = same ? T.at(T.L.os + ((hi * (hi - 1)) >> 1) + lo)
                            : T.at(T.L.oj + ((hi * (hi + 1)) >> 1) + lo);
      e += (sg[k1] * sg[k2]) * w;
    }
  }
  return e;
}

// H_aa for determinant a = (alpha a0:a1, beta b0:b1); r = reference det.
template <bool LDS>
SHCI_DEV double diag_energy(uint64_t a0, uint64_t a1, uint64_t b0, uint64_t b1, const uint64_t (&r)[4],
                            const DiagTab<LDS>& T, int ne) {
  {
    const uint64_t pa0 = a0 & ~r[0], pa1 = a1 & ~r[1], pb0 = b0 & ~r[2], pb1 = b1 & ~r[3];
    const int l = __builtin_popcountll(pa0) + __builtin_popcountll(pa1) + __builtin_popcountll(pb0) + __builtin_popcountll(pb1);
    if (2 * l <= DL_MAX)
      return diag_list<LDS>(pa0, pa1, pb0, pb1, r[0] & ~a0, r[1] & ~a1, r[2] & ~b0, r[3] & ~b1, T);
  }
  if (T.L.n <= 64) return diag_energy1<LDS>(a0, b0, r[0], r[2], T, ne);
  const int n = T.L.n;
  uint64_t r0 = r[0], r1 = r[1], r2 = r[2], r3 = r[3];
  int l = __builtin_popcountll(a0 & ~r0) + __builtin_popcountll(a1 & ~r1) + __builtin_popcountll(b0 & ~r2) + __builtin_popcountll(b1 & ~r3);
  const bool use_ref = 3 * l * l + 2 * l < ne * (ne + 1) / 2;
  double e = 0.0;
  if (use_ref) {
    e = T.at(T.L.oe);
  } else {
    r0 = r1 = r2 = r3 = 0ull;
  }
  // masks: 0 particles alpha, 1 particles beta, 2 holes alpha, 3 holes beta
  const uint64_t m0a = a0 & ~r0, m0b = a1 & ~r1;
  const uint64_t m1a = b0 & ~r2, m1b = b1 & ~r3;
  const uint64_t m2a = r0 & ~a0, m2b = r1 & ~a1;
  const uint64_t m3a = r2 & ~b0, m3b = r3 & ~b1;
  // one-orbital terms
#pragma unroll 1
  for (int c = 0; c < 4; ++c) {
    uint64_t x0 = sel4(c, m0a, m1a, m2a, m3a), x1 = sel4(c, m0b, m1b, m2b, m3b);
    const int sp = c & 1;
    double s = 0.0;
    while (x0 | x1) {
      const int p = pop_bit(x0, x1);
      s += use_ref ? T.at(T.L.of + sp * n + p) : T.at(p);
    }
    e = (c < 2) ? e + s : e - s;
  }
  // pair terms: (X, Y, kind, sign); kind 0: X = Y, p < q, J-K; 1: J-K; 2: J
#pragma unroll 1
  for (int c = 0; c < 10; ++c) {
    int xm, ym, kind;
    double sign = 1.0;
    switch (c) {
      case 0: xm = 0; ym = 0; kind = 0; break;
      case 1: xm = 1; ym = 1; kind = 0; break;
      case 2: xm = 0; ym = 1; kind = 2; break;
      case 3: xm = 2; ym = 2; kind = 0; break;
      case 4: xm = 3; ym = 3; kind = 0; break;
      case 5: xm = 2; ym = 3; kind = 2; break;
      case 6: xm = 0; ym = 2; kind = 1; sign = -1.0; break;
      case 7: xm = 1; ym = 3; kind = 1; sign = -1.0; break;
      case 8: xm = 0; ym = 3; kind = 2; sign = -1.0; break;
      default: xm = 1; ym = 2; kind = 2; sign = -1.0; break;
    }
    uint64_t x0 = sel4(xm, m0a, m1a, m2a, m3a), x1 = sel4(xm, m0b, m1b, m2b, m3b);
    const uint64_t y0i = sel4(ym, m0a, m1a, m2a, m3a), y1i = sel4(ym, m0b, m1b, m2b, m3b);
    double s = 0.0;
    while (x0 | x1) {
      const int p = pop_bit(x0, x1);
      uint64_t y0 = y0i, y1 = y1i;
      if (kind == 0) {  // only q > p
        uint64_t lm0, lm1;
        low_mask(p + 1, lm0, lm1);
        y0 &= ~lm0;
        y1 &= ~lm1;
      }
      while (y0 | y1) {
        const int q = pop_bit(y0, y1);
        const int lo = p < q ? p : q, hi = p < q ? q : p;
        s += (kind == 2) ? T.at(T.L.oj + hi * (hi + 1) / 2 + lo) : T.at(T.L.os + hi * (hi - 1) / 2 + lo);
      }
    }
    e += sign * s;
  }
  return e;
}

// plain sum over occupied pairs (reads only h, (pp|qq) and (pp|qq)-(pq|qp))
SHCI_DEV double diag_plain(uint64_t a0, uint64_t a1, uint64_t b0, uint64_t b1, const double* tab,
                           const DiagLayout& L) {
  double e = 0.0;
  for (int sp = 0; sp < 2; ++sp) {
    uint64_t x0 = sp ? b0 : a0, x1 = sp ? b1 : a1;
    while (x0 | x1) {
      const int p = pop_bit(x0, x1);
      e += tab[p];
      uint64_t y0 = x0, y1 = x1;  // orbitals above p, same spin
      while (y0 | y1) {
        const int q = pop_bit(y0, y1);
        e += tab[L.os + ((q * (q - 1)) >> 1) + p];
      }
    }
  }
  uint64_t x0 = a0, x1 = a1;
  while (x0 | x1) {
    const int p = pop_bit(x0, x1);
    uint64_t y0 = b0, y1 = b1;
    while (y0 | y1) {
      const int q = pop_bit(y0, y1);
      const int lo = p < q ? p : q, hi = p < q ? q : p;
      e += tab[L.oj + ((hi * (hi + 1)) >> 1) + lo];
    }
  }
  return e;
}

// Per call: F_p(sigma) of the reference det and E(R) into the packed global
// table (one block).
__global__ void k_diag_ref(const uint64_t* ref, int n, int ne, double* tab) {
  const DiagLayout L = DiagLayout::make(n);
  const uint64_t r0 = ref[0], r1 = ref[1], r2 = ref[2], r3 = ref[3];
  for (int t = threadIdx.x; t < 2 * n; t += blockDim.x) {
    const int p = t % n, sp = t / n;
    double v = tab[p];
    for (int q = 0; q < n; ++q) {
      const bool inA = occ(r0, r1, q), inB = occ(r2, r3, q);
      const int lo = p < q ? p : q, hi = p < q ? q : p;
      const double j = tab[L.oj + hi * (hi + 1) / 2 + lo];
      const double s = (p == q) ? 0.0 : tab[L.os + hi * (hi - 1) / 2 + lo];
      if (sp == 0) {
        if (inA && q != p) v += s;
        if (inB) v += j;
      } else {
        if (inB && q != p) v += s;
        if (inA) v += j;
      }
    }
    tab[L.of + t] = v;
  }
  if (threadIdx.x == 0) tab[L.oe] = diag_plain(r0, r1, r2, r3, tab, L);
}

}  // namespace shci
