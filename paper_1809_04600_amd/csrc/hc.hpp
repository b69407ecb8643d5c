// H c on the variational space through alpha and beta string lists
// (section III, Table I and Algorithms 1-2).
//
// Determinants are grouped by their alpha string and by their beta string
// (open-addressing string tables; a group is named by its smallest
// determinant index, so the grouping is deterministic).  Each group's members
// are listed in index order (stable radix sort of (group, index) pairs), and
// every alpha group carries the list of alpha groups one single excitation
// away.  Row i of y = H c then visits
//   * the members of its beta group (same beta string: alpha singles and
//     doubles),
//   * the members of its alpha group (same alpha string: beta singles and
//     doubles),
//   * for each alpha group one alpha single away, its members whose beta
//     string is one beta single away (opposite-spin doubles): a small group
//     is scanned, a large one is probed with the beta groups one single away
//     from the row's beta string through a table of (alpha group, beta
//     group) pairs, whichever visits fewer entries,
// and adds H_ii c_i.  The other-spin strings of each group's members are
// packed in member order, so scans stream them, together with a 32-bit fold
// of each (the XOR of its 32-bit quarters): two strings k excitations apart
// differ in 2k bits, and folding can only cancel differing bits, so a fold
// difference of more than 2k bits rules the pair out before the full strings
// are read.  Elements are evaluated from the row's determinant as
// the source, with the phases and the canonical single-element sum of the
// excitation generator.  One wavefront per row; lanes take the members, and
// the row sum is a fixed butterfly, so y is deterministic.
#pragma once
#include "diag.hpp"
#include "kernels.hpp"

namespace shci {

constexpr uint32_t STR_EMPTY = 0xffffffffu;

struct StrTab {
  uint32_t* slot;  // smallest determinant index holding the string, or STR_EMPTY
  uint64_t mask;   // capacity - 1 (capacity a power of two >= 2 N)
};

SHCI_DEV uint64_t str_hash(uint64_t w0, uint64_t w1) {
  return fmix64(fmix64(0x9e3779b97f4a7c15ull ^ w0) ^ w1);
}

// the string of spin `spin` of determinant i
SHCI_DEV void str_of(const uint64_t* dets, int64_t i, int spin, uint64_t& w0, uint64_t& w1) {
  w0 = dets[4 * i + 2 * spin];
  w1 = dets[4 * i + 2 * spin + 1];
}

// insert every determinant's string: the slot of a string ends with the
// smallest index that holds it (the capacity is at least twice the number of
// determinants, so every probe sequence meets an empty slot)
__global__ void k_str_insert(const uint64_t* dets, int64_t nd, int spin, StrTab t) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= nd) return;
  uint64_t w0, w1;
  str_of(dets, i, spin, w0, w1);
  uint64_t s = str_hash(w0, w1) & t.mask;
  for (;;) {
    const uint32_t cur = atomicCAS(&t.slot[s], STR_EMPTY, (uint32_t)i);
    if (cur == STR_EMPTY) return;
    uint64_t v0, v1;
    str_of(dets, cur, spin, v0, v1);  // every index ever held by a slot has the slot's string
    if (v0 == w0 && v1 == w1) {
      atomicMin(&t.slot[s], (uint32_t)i);
      return;
    }
    s = (s + 1) & t.mask;
  }
}

// group of a string (smallest determinant index holding it), STR_EMPTY if absent
SHCI_DEV uint32_t str_find(const uint64_t* dets, int spin, const StrTab& t, uint64_t w0, uint64_t w1) {
  uint64_t s = str_hash(w0, w1) & t.mask;
  for (;;) {
    const uint32_t cur = t.slot[s];
    if (cur == STR_EMPTY) return STR_EMPTY;
    uint64_t v0, v1;
    str_of(dets, cur, spin, v0, v1);
    if (v0 == w0 && v1 == w1) return cur;
    s = (s + 1) & t.mask;
  }
}

__global__ void k_str_group(const uint64_t* dets, int64_t nd, int spin, StrTab t, uint32_t* grp) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= nd) return;
  uint64_t w0, w1;
  str_of(dets, i, spin, w0, w1);
  grp[i] = str_find(dets, spin, t, w0, w1);
}

// ---------------------------------------------------------------------------
// Stable LSD radix sort of (key, value) uint32 pairs, 8-bit digits, one
// wavefront per tile of 256 pairs.
// ---------------------------------------------------------------------------
constexpr int PAIR_TILE = 256;

SHCI_DEV void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// hist[d * ntiles + tile] = pairs of the tile with digit d
__global__ void __launch_bounds__(256) k_pair_count(const uint32_t* key, int64_t n, int shift, int64_t ntiles,
                                                    uint32_t* hist) {
  __shared__ uint32_t cnt[4][256];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t tile = (int64_t)blockIdx.x * 4 + wv;
  if (tile >= ntiles) return;
  for (int d = lane; d < 256; d += 64) cnt[wv][d] = 0;
  wave_sync();
  for (int r = 0; r < PAIR_TILE / 64; ++r) {
    const int64_t i = tile * PAIR_TILE + r * 64 + lane;
    if (i < n) atomicAdd(&cnt[wv][(key[i] >> shift) & 255u], 1u);
  }
  wave_sync();
  for (int d = lane; d < 256; d += 64) hist[(int64_t)d * ntiles + tile] = cnt[wv][d];
}

// stable placement: offs is the exclusive scan of hist (digit-major)
__global__ void __launch_bounds__(256) k_pair_place(const uint32_t* kin, const uint32_t* vin, int64_t n, int shift,
                                                    int64_t ntiles, const uint32_t* offs, uint32_t* kout,
                                                    uint32_t* vout) {
  __shared__ uint32_t base[4][256];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t tile = (int64_t)blockIdx.x * 4 + wv;
  if (tile >= ntiles) return;
  for (int d = lane; d < 256; d += 64) base[wv][d] = offs[(int64_t)d * ntiles + tile];
  wave_sync();
  for (int r = 0; r < PAIR_TILE / 64; ++r) {
    const int64_t i = tile * PAIR_TILE + r * 64 + lane;
    const bool valid = i < n;
    const uint32_t k = valid ? kin[i] : 0u;
    const uint32_t d = (k >> shift) & 255u;
    uint64_t peers = ballot(valid);
#pragma unroll
    for (int bb = 0; bb < 8; ++bb) {
      const bool on = (d >> bb) & 1u;
      const uint64_t m = ballot(on);
      peers &= on ? m : ~m;
    }
    const int rk = rank_below(peers);
    const uint32_t prior = valid ? base[wv][d] : 0u;
    wave_sync();
    if (valid && rk == 0) base[wv][d] = prior + (uint32_t)__popcll(peers);
    wave_sync();
    if (valid) {
      kout[prior + rk] = k;
      vout[prior + rk] = vin[i];
    }
  }
}

// ---------------------------------------------------------------------------
// Groups one single excitation away (Table I: the alpha- and beta-singles
// lists)
// ---------------------------------------------------------------------------
struct SinglesArgs {
  const uint64_t* dets;
  int64_t nd;
  int n, ne;  // orbitals, electrons of the spin
  int spin;
  StrTab t;
  const uint32_t* grp;  // group of each determinant for that spin
  uint32_t* cnt;        // per representative: number of neighbours
  const uint64_t* off;  // per representative: first list position (WRITE)
  uint32_t* list;       // neighbour groups (WRITE)
};

// One wavefront per representative determinant (the smallest index of its
// group); candidates r -> s (r occupied, s empty, both ascending) in order,
// found strings appended in that order.
template <bool WRITE>
__global__ void __launch_bounds__(256) k_str_singles(SinglesArgs a) {
  __shared__ uint8_t s_occ[4][128], s_vir[4][128];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t nwaves = (int64_t)gridDim.x * 4;
  const int n = a.n, no = a.ne, nv = n - a.ne;
  uint8_t* occl = s_occ[wv];
  uint8_t* virl = s_vir[wv];
  for (int64_t i = (int64_t)blockIdx.x * 4 + wv; i < a.nd; i += nwaves) {
    if (a.grp[i] != (uint32_t)i) continue;  // uniform
    const uint64_t w0 = a.dets[4 * i + 2 * a.spin], w1 = a.dets[4 * i + 2 * a.spin + 1];
    {
      int co = 0, cv = 0;
      for (int h = 0; h < 2; ++h) {
        const int p = lane + 64 * h;
        const bool in = p < n;
        const bool o = in && (((h ? w1 : w0) >> lane) & 1ull);
        uint64_t m = ballot(o);
        if (o) occl[co + rank_below(m)] = (uint8_t)p;
        co += __popcll(m);
        m = ballot(in && !o);
        if (in && !o) virl[cv + rank_below(m)] = (uint8_t)p;
        cv += __popcll(m);
      }
    }
    wave_sync();
    const int ncand = no * nv;
    uint32_t found = 0;  // uniform
    for (int j0 = 0; j0 < ncand; j0 += 64) {
      const int j = j0 + lane;
      uint32_t g = STR_EMPTY;
      if (j < ncand) {
        const int r = occl[j / nv], s = virl[j % nv];
        uint64_t x0 = w0, x1 = w1;
        flip(x0, x1, r);
        flip(x0, x1, s);
        g = str_find(a.dets, a.spin, a.t, x0, x1);
      }
      const bool hit = g != STR_EMPTY;
      const uint64_t hb = ballot(hit);
      if constexpr (WRITE) {
        if (hit) a.list[a.off[i] + found + rank_below(hb)] = g;
      }
      found += (uint32_t)__popcll(hb);
    }
    if constexpr (!WRITE) {
      if (lane == 0) a.cnt[i] = found;
    }
    wave_sync();
  }
}

// ---------------------------------------------------------------------------
// Table of (alpha group, beta group) -> determinant, open addressing on the
// 64-bit key gA << 32 | gB (capacity a power of two >= 2 N)
// ---------------------------------------------------------------------------
constexpr uint64_t PAIR_EMPTY = ~0ull;

struct PairTab {
  uint64_t* key;
  uint32_t* val;
  uint64_t mask;
};

__global__ void k_pairtab_insert(const uint32_t* grpA, const uint32_t* grpB, int64_t nd, PairTab t) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= nd) return;
  const uint64_t k = ((uint64_t)grpA[i] << 32) | grpB[i];
  uint64_t s = fmix64(k) & t.mask;
  for (;;) {
    const unsigned long long cur = atomicCAS((unsigned long long*)&t.key[s], (unsigned long long)PAIR_EMPTY,
                                             (unsigned long long)k);
    if (cur == PAIR_EMPTY || cur == k) {
      // equal keys only for a repeated determinant (reported by the rows)
      atomicMin(&t.val[s], (uint32_t)i);
      return;
    }
    s = (s + 1) & t.mask;
  }
}

SHCI_DEV uint32_t pairtab_find(const PairTab& t, uint32_t ga, uint32_t gb) {
  const uint64_t k = ((uint64_t)ga << 32) | gb;
  uint64_t s = fmix64(k) & t.mask;
  for (;;) {
    const uint64_t cur = t.key[s];
    if (cur == PAIR_EMPTY) return STR_EMPTY;
    if (cur == k) return t.val[s];
    s = (s + 1) & t.mask;
  }
}

SHCI_HD uint32_t fold32(uint64_t w0, uint64_t w1) {
  return (uint32_t)w0 ^ (uint32_t)(w0 >> 32) ^ (uint32_t)w1 ^ (uint32_t)(w1 >> 32);
}

// the other-spin string of each member, in member order, and its fold
__global__ void k_pack_other(const uint32_t* mem, const uint64_t* dets, int64_t nd, int other, uint64_t* o0,
                             uint64_t* o1, uint32_t* of) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= nd) return;
  const int64_t j = mem[e];
  const uint64_t w0 = dets[4 * j + 2 * other], w1 = dets[4 * j + 2 * other + 1];
  o0[e] = w0;
  o1[e] = w1;
  of[e] = fold32(w0, w1);
}

// ---------------------------------------------------------------------------
// Rows of y = H c
// ---------------------------------------------------------------------------
struct HcArgs {
  Tables T;
  const uint64_t* dets;
  const double* c;
  int64_t nd;
  const uint32_t* grpA;   // alpha group of each determinant
  const uint32_t* grpB;   // beta group
  const uint32_t* memA;   // members of the alpha groups, group by group, index order
  const uint32_t* memB;
  const uint64_t* startA; // [nd + 1] first member position of group g (groups named by index)
  const uint64_t* startB;
  const uint64_t* soff;   // [nd + 1] alpha-singles list of group g: [soff[g], soff[g + 1])
  const uint32_t* slist;
  const uint64_t* soffB;  // beta-singles lists
  const uint32_t* slistB;
  const uint64_t* bOfA0;  // beta string of alpha-group member e (words 0, 1)
  const uint64_t* bOfA1;
  const uint64_t* aOfB0;  // alpha string of beta-group member e
  const uint64_t* aOfB1;
  const uint32_t* bOfAf;  // folds of the packed strings
  const uint32_t* aOfBf;
  PairTab pt;
  double* y;
  uint32_t* nconn;        // optional
  uint32_t* flag;         // |= 4: a determinant occurs twice
};

SHCI_HD int64_t pair_index(int p, int q) { return p > q ? (int64_t)p * (p + 1) / 2 + q : (int64_t)q * (q + 1) / 2 + p; }

// (pq|rs) from the folded table
SHCI_DEV double eri_g8(const double* g8, int p, int q, int r, int s) {
  const int64_t a = pair_index(p, q), b = pair_index(r, s);
  return g8[a > b ? a * (a + 1) / 2 + b : b * (b + 1) / 2 + a];
}

// single p -> r of spin `alpha` from the source with occupied lists occA/occB,
// in the generator's canonical order (h_pr, alpha occupied ascending, beta
// occupied ascending; equal-spin k != p add (pr|kk) - (pk|kr), the other spin
// adds (pr|kk)), without the phase
SHCI_DEV double single_elem(const Tables& T, const uint8_t* occA, int na, const uint8_t* occB, int nb,
                            bool alpha, int p, int r) {
  const int n = T.n;
  const size_t nn = (size_t)n * n, pr = (size_t)p * n + r;
  const double* tabA = alpha ? T.sD : T.sJ;
  const double* tabB = alpha ? T.sJ : T.sD;
  double acc = T.h1[pr];
  for (int k = 0; k < na; ++k)
    if (!(alpha && occA[k] == p)) acc = acc + tabA[occA[k] * nn + pr];
  for (int k = 0; k < nb; ++k)
    if (!(!alpha && occB[k] == p)) acc = acc + tabB[occB[k] * nn + pr];
  return acc;
}

SHCI_DEV int lowest(uint64_t x0, uint64_t x1) {
  return x0 ? __builtin_ctzll(x0) : 64 + __builtin_ctzll(x1);
}

__global__ void __launch_bounds__(256) k_hc_rows(HcArgs a) {
  __shared__ uint8_t s_occ[4][2][128];
  __shared__ uint32_t s_q[4][128];  // queue of same-string members that pass the fold
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t nwaves = (int64_t)gridDim.x * 4;
  const Tables& T = a.T;
  const int n = T.n, na = T.na, nb = T.nb;
  uint8_t* occA = s_occ[wv][0];
  uint8_t* occB = s_occ[wv][1];
  const DiagLayout DL = DiagLayout::make(n);
  for (int64_t i = (int64_t)blockIdx.x * 4 + wv; i < a.nd; i += nwaves) {
    const uint64_t A0 = a.dets[4 * i], A1 = a.dets[4 * i + 1], B0 = a.dets[4 * i + 2], B1 = a.dets[4 * i + 3];
    {
      int ca = 0, cb = 0;
      for (int h = 0; h < 2; ++h) {
        const int p = lane + 64 * h;
        const bool in = p < n;
        const bool oa = in && (((h ? A1 : A0) >> lane) & 1ull);
        const bool ob = in && (((h ? B1 : B0) >> lane) & 1ull);
        uint64_t m = ballot(oa);
        if (oa) occA[ca + rank_below(m)] = (uint8_t)p;
        ca += __popcll(m);
        m = ballot(ob);
        if (ob) occB[cb + rank_below(m)] = (uint8_t)p;
        cb += __popcll(m);
      }
    }
    wave_sync();
    // H_ii = 1/2 sum over occupied spin orbitals of (h_xx + F_x)
    double part = 0.0;
    for (int x = lane; x < n; x += 64) {
      double fa, fb;
      fock_diag2(T.diag, DL, x, occA, na, occB, nb, fa, fb);
      const double hx = T.diag[x];
      if (occ(A0, A1, x)) part += hx + fa;
      if (occ(B0, B1, x)) part += hx + fb;
    }
    double acc = 0.0;
    uint32_t cnt = 0;
    bool dup = false;
    // Same-string groups: members whose fold passes are queued (member
    // position in the low 31 bits, bit 31 set for the alpha group) and
    // evaluated 64 at a time on full wavefronts.
    uint32_t* qu = s_q[wv];
    int qn = 0;  // uniform
    auto process = [&](int m) {
      const bool valid = lane < m;
      const uint32_t code = valid ? qu[lane] : 0u;
      const bool inA = (code >> 31) != 0;  // member of the row's alpha group: beta excitation
      const uint64_t e = code & 0x7fffffffu;
      double H = 0.0;
      int d = 0;
      uint32_t j = 0;
      if (valid) {
        j = inA ? a.memA[e] : a.memB[e];
        const uint64_t S0 = inA ? B0 : A0, S1 = inA ? B1 : A1;
        const uint64_t x0 = inA ? a.bOfA0[e] : a.aOfB0[e], x1 = inA ? a.bOfA1[e] : a.aOfB1[e];
        const uint64_t h0 = S0 & ~x0, h1 = S1 & ~x1, q0 = x0 & ~S0, q1 = x1 & ~S1;
        d = __popcll(h0) + __popcll(h1);
        if (d == 1) {
          const int p = lowest(h0, h1), r = lowest(q0, q1);
          H = single_elem(T, occA, na, occB, nb, !inA, p, r);
          if (between(S0, S1, p, r) & 1) H = -H;
        } else if (d == 2) {
          const int p = lowest(h0, h1), r = lowest(q0, q1);
          const int qq = lowest(h0 & (h0 - 1), h0 ? h1 : (h1 & (h1 - 1)));
          const int ss = lowest(q0 & (q0 - 1), q0 ? q1 : (q1 & (q1 - 1)));
          uint64_t y0 = S0, y1 = S1;
          int par = between(y0, y1, p, r);
          flip(y0, y1, p);
          flip(y0, y1, r);
          par += between(y0, y1, qq, ss);
          H = eri_g8(T.g8, p, r, qq, ss) - eri_g8(T.g8, p, ss, qq, r);
          if (par & 1) H = -H;
        }
        dup = dup || d == 0;
        cnt += (d == 1 || d == 2);
        acc += H * a.c[j];
      }
    };
    auto scan = [&](uint64_t lo, uint64_t hi, const uint32_t* fo, const uint32_t* mem, uint32_t fi, uint32_t tag) {
      for (uint64_t e0 = lo; e0 < hi; e0 += 64) {  // uniform
        const uint64_t e = e0 + lane;
        const bool pass = e < hi && __popc(fo[e] ^ fi) <= 4 && mem[e] != (uint32_t)i;
        const uint64_t pb = ballot(pass);
        if (pass) qu[qn + rank_below(pb)] = (uint32_t)e | tag;
        qn += __popcll(pb);
        wave_sync();
        if (qn >= 64) {
          process(64);
          const uint32_t rest = (lane + 64 < qn) ? qu[lane + 64] : 0u;
          wave_sync();
          if (lane + 64 < qn) qu[lane] = rest;
          qn -= 64;
          wave_sync();
        }
      }
    };
    {
      const uint32_t gB = a.grpB[i], gA = a.grpA[i];
      scan(a.startB[gB], a.startB[gB + 1], a.aOfBf, a.memB, fold32(A0, A1), 0u);
      scan(a.startA[gA], a.startA[gA + 1], a.bOfAf, a.memA, fold32(B0, B1), 0x80000000u);
      if (qn > 0) process(qn);
      wave_sync();
    }
    // alpha single and beta single: alpha groups one alpha single away, their
    // members one beta single away
    {
      const uint32_t ga = a.grpA[i], gb = a.grpB[i];
      const uint32_t fb = fold32(B0, B1);
      const uint64_t sb0 = a.soffB[gb], nsb = a.soffB[gb + 1] - sb0;
      for (uint64_t sidx = a.soff[ga]; sidx < a.soff[ga + 1]; ++sidx) {  // uniform
        const uint32_t g2 = a.slist[sidx];
        const uint64_t z0 = a.dets[4 * (int64_t)g2], z1 = a.dets[4 * (int64_t)g2 + 1];
        const int p = lowest(A0 & ~z0, A1 & ~z1), r = lowest(z0 & ~A0, z1 & ~A1);
        const int para = between(A0, A1, p, r);
        const uint64_t m0 = a.startA[g2], m1 = a.startA[g2 + 1];
        if (m1 - m0 <= nsb) {
          // scan the members of the alpha group
          for (uint64_t e = m0 + lane; e < m1; e += 64) {
            if (__popc(a.bOfAf[e] ^ fb) > 2) continue;
            const uint64_t x0 = a.bOfA0[e], x1 = a.bOfA1[e];
            const uint64_t h0 = B0 & ~x0, h1 = B1 & ~x1;
            if (__popcll(h0) + __popcll(h1) != 1) continue;
            const int q = lowest(h0, h1), s = lowest(x0 & ~B0, x1 & ~B1);
            double H = eri_g8(T.g8, p, r, q, s);
            if ((para + between(B0, B1, q, s)) & 1) H = -H;
            cnt += 1;
            acc += H * a.c[a.memA[e]];
          }
        } else {
          // probe (alpha group, beta group one single away) pairs
          for (uint64_t k = lane; k < nsb; k += 64) {
            const uint32_t gb2 = a.slistB[sb0 + k];
            const uint32_t j = pairtab_find(a.pt, g2, gb2);
            if (j == STR_EMPTY) continue;
            const uint64_t x0 = a.dets[4 * (int64_t)gb2 + 2], x1 = a.dets[4 * (int64_t)gb2 + 3];
            const int q = lowest(B0 & ~x0, B1 & ~x1), s = lowest(x0 & ~B0, x1 & ~B1);
            double H = eri_g8(T.g8, p, r, q, s);
            if ((para + between(B0, B1, q, s)) & 1) H = -H;
            cnt += 1;
            acc += H * a.c[j];
          }
        }
      }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      part += __shfl_xor(part, o);
      acc += __shfl_xor(acc, o);
      cnt += __shfl_xor(cnt, o);
    }
    if (ballot(dup) && lane == 0) atomicOr(a.flag, 4u);
    if (lane == 0) {
      a.y[i] = acc + (0.5 * part) * a.c[i];
      if (a.nconn) a.nconn[i] = cnt;
    }
    wave_sync();
  }
}

// keys = group of each determinant, values = its index
__global__ void k_pair_init(const uint32_t* grp, int64_t n, uint32_t* k, uint32_t* v) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  k[i] = grp[i];
  v[i] = (uint32_t)i;
}

// deterministic sum of n uint32 values (fixed chunks, fixed tree)
__global__ void __launch_bounds__(1024) k_sum_u32(const uint32_t* x, int64_t n, uint64_t* out) {
  __shared__ uint64_t r[1024];
  const int t = threadIdx.x;
  const int64_t chunk = (n + 1023) / 1024;
  uint64_t s = 0;
  for (int64_t i = t * chunk; i < min(n, (int64_t)(t + 1) * chunk); ++i) s += x[i];
  r[t] = s;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if (t < o) r[t] += r[t + o];
    __syncthreads();
  }
  if (t == 0) *out = r[0];
}

// deterministic <c|y> and <c|c> (fixed chunks, fixed tree): out[0], out[1]
__global__ void __launch_bounds__(1024) k_dot2(const double* c, const double* y, int64_t nd, double* out) {
  __shared__ double r1[1024], r2[1024];
  const int t = threadIdx.x;
  const int64_t chunk = (nd + 1023) / 1024;
  double s1 = 0.0, s2 = 0.0;
  for (int64_t i = t * chunk; i < min(nd, (int64_t)(t + 1) * chunk); ++i) {
    s1 += c[i] * y[i];
    s2 += c[i] * c[i];
  }
  r1[t] = s1;
  r2[t] = s2;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if (t < o) {
      r1[t] += r1[t + o];
      r2[t] += r2[t + o];
    }
    __syncthreads();
  }
  if (t == 0) {
    out[0] = r1[0];
    out[1] = r2[0];
  }
}

}  // namespace shci
