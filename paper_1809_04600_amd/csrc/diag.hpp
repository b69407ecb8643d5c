// Epstein-Nesbet diagonal H_aa (the partition that gives the PT2 denominators
// E0 - H_aa, Sec. II) as an update from the source determinant.
//
// Packed table layout (doubles), built once per integral set:
//   [0, n)                     h_pp
//   [n, n + n(n+1)/2)          (pp|qq), p <= q, at q(q+1)/2 + p
//   [.., + n(n-1)/2)           (pp|qq) - (pq|qp), p < q, at q(q-1)/2 + p
// W_xy is the pair energy of two occupied spin orbitals: J - K for equal
// spins, J otherwise.  For a determinant i with occupied set O,
//   F_x = h_xx + sum_{y in O, y != x} W_xy      (Fock-like diagonal of i)
//   H_ii = 1/2 sum_{x in O} (h_xx + F_x),
// and for a = i with holes Q and particles P (spin orbitals) the sum over
// occupied pairs rearranges exactly to
//   H_aa = H_ii + sum_{x in P} F_x - sum_{y in Q} F_y - sum_{x in P, y in Q} W_xy
//          + sum_{x<x' in P} W_xx' + sum_{y<y' in Q} W_yy'.
// A single or double excitation therefore costs a fixed handful of lookups,
// independent of the number of electrons.
#pragma once
#include "common.hpp"

namespace shci {

struct DiagLayout {
  int n;
  int oj, os, total;
  SHCI_HD static DiagLayout make(int n) {
    DiagLayout L;
    L.n = n;
    L.oj = n;
    L.os = L.oj + n * (n + 1) / 2;
    L.total = L.os + n * (n - 1) / 2;
    return L;
  }
};

inline int diag_table_doubles(int n) { return n * n + n; }

// W of spin orbitals x != y (same: equal spins)
SHCI_HD double pair_w(const double* tab, const DiagLayout& L, int x, int y, bool same) {
  const int lo = x < y ? x : y, hi = x < y ? y : x;
  return same ? tab[L.os + ((hi * (hi - 1)) >> 1) + lo] : tab[L.oj + ((hi * (hi + 1)) >> 1) + lo];
}

// F_x for x alpha (fa) and x beta (fb) of a determinant with occupied
// orbitals occA[0..na) and occB[0..nb); table loads are issued eight
// occupied orbitals at a time and added in list order
SHCI_HD void fock_diag2(const double* tab, const DiagLayout& L, int x, const uint8_t* occA, int na,
                        const uint8_t* occB, int nb, double& fa, double& fb) {
  fa = tab[x];
  fb = fa;
  for (int side = 0; side < 2; ++side) {
    const uint8_t* oc = side ? occB : occA;
    const int no = side ? nb : na;
    for (int k0 = 0; k0 < no; k0 += 8) {
      double sv[8], jv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const bool in = k0 + u < no;
        const int k = in ? (int)oc[k0 + u] : x;
        sv[u] = (in && k != x) ? pair_w(tab, L, x, k, true) : 0.0;
        jv[u] = in ? pair_w(tab, L, x, k, false) : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        // orbitals of spin alpha add W to F_x(alpha) as equal spins and to
        // F_x(beta) as opposite spins; beta orbitals the other way round
        fa += side ? jv[u] : sv[u];
        fb += side ? sv[u] : jv[u];
      }
    }
  }
}

// H_aa - H_ii for the single p -> r (F: the Fock-like diagonal of that spin)
SHCI_HD double en_single(const double* F, const double* tab, const DiagLayout& L, int p, int r) {
  return (F[r] - F[p]) - pair_w(tab, L, r, p, true);
}

// H_aa - H_ii for the double p -> r, q -> s; r takes p's spin (diagonal Fp),
// s takes q's (Fq); same: p and q have equal spins
SHCI_HD double en_double(const double* Fp, const double* Fq, const double* tab, const DiagLayout& L,
                         int p, int q, int r, int s, bool same) {
  double d = (Fp[r] + Fq[s]) - (Fp[p] + Fq[q]);
  d -= (pair_w(tab, L, r, p, true) + pair_w(tab, L, s, q, true)) +
       (pair_w(tab, L, r, q, same) + pair_w(tab, L, s, p, same));
  d += pair_w(tab, L, r, s, same) + pair_w(tab, L, p, q, same);
  return d;
}

}  // namespace shci
