// Excitation generator: one wavefront per work item (a source determinant, or
// a distinct sampled determinant, restricted to a range of its occupied
// pairs), work items assigned round-robin to persistent wavefronts.
//
// For each source det i it emits every single and double excitation a with
// |H_ai| |c_i| > eps2 (screened PT2 equation, section II.B):
//  * singles p->r: a per-(p,r) upper bound of |H_ai| skips hopeless pairs;
//    survivors get the exact element h_pr + sum_k [...] accumulated in a
//    fixed order (occupied alpha ascending, then occupied beta ascending);
//  * doubles: for every occupied pair the heat-bath list of that pair is
//    walked in decreasing |value| (the first eight entries of eight pairs at
//    once, longer lists 64 entries at a time), and the walk stops at the
//    first entry that fails the screen (section II.A, heat-bath traversal
//    with early exit).  Entries whose target orbitals are occupied are skipped.
//  * fermion signs come from popcounts of the occupied bits between the
//    orbitals involved; a same-spin double is p->r then q->s.
// Lane-parallel emission uses ballot + mbcnt compaction, so the record order
// is fixed by (source index, generation order) and the run is deterministic.
// The same walk runs in three modes: the count walk counts the kept terms of
// each work item (and, for the singleton split, lists each one's grouping
// hash); the write walk writes records at the counted offsets (in split mode
// only the terms whose hash passes the filter of repeated hashes, the others
// summed in place); the adjoint walk adds dE2/dc_i from the kept per-a
// factors.
#pragma once
#include "diag.hpp"
#include "kernels.hpp"

namespace shci {

enum GenMode { GEN_COUNT = 0, GEN_WRITE = 1, GEN_GRAD = 2 };

struct VSet {
  uint64_t* tab = nullptr;  // slots: fingerprint << 32 | index; ~0 = empty
  uint64_t mask = 0;
  const uint64_t* dets = nullptr;
  // presence filter (blocked, two bits per member in one 64-bit word):
  // word h >> (64 - fbits), bits (h >> 20) & 63 and (h >> 26) & 63 are set
  // for every member.  ~32 bits per member (false positives ~0.5%); the
  // lookups of one bucket (equal top hash bits) fall into the same few words.
  uint64_t* filt = nullptr;
  int fbits = 0;
};

// two bits of a hash in one 64-bit word of a blocked presence filter:
// word h >> (64 - fbits), bits (h >> 20) & 63 and (h >> 26) & 63
SHCI_DEV uint64_t filt_bits(uint64_t h) { return (1ull << ((h >> 20) & 63)) | (1ull << ((h >> 26) & 63)); }

// false: certainly never inserted; true: maybe
SHCI_DEV bool filt_maybe(const uint64_t* words, int fbits, uint64_t h) {
  const uint64_t m = filt_bits(h);
  return (words[h >> (64 - fbits)] & m) == m;
}

SHCI_DEV void filt_insert(uint64_t* words, int fbits, uint64_t h) {
  atomicOr((unsigned long long*)&words[h >> (64 - fbits)], (unsigned long long)filt_bits(h));
}

SHCI_DEV uint64_t vfilt_bits(uint64_t h) { return filt_bits(h); }
SHCI_DEV bool vfilt_maybe(const VSet& V, uint64_t h) { return filt_maybe(V.filt, V.fbits, h); }

// membership in the hash set of V of a determinant that passed the filter
template <int KW>
SHCI_DEV bool vset_probe(const VSet& V, const uint64_t (&k)[KW], uint64_t h, int n) {
  uint64_t slot = h & V.mask;
  const uint32_t fp = (uint32_t)(h >> 32);
  for (uint64_t probe = 0; probe <= V.mask; ++probe) {
    const uint64_t e = V.tab[slot];
    if (e == ~0ull) return false;
    if ((uint32_t)(e >> 32) == fp) {
      const uint64_t i = e & 0xffffffffull;
      uint64_t dk[KW];
      pack_det<KW>(dk, V.dets[4 * i], V.dets[4 * i + 1], V.dets[4 * i + 2], V.dets[4 * i + 3], n);
      bool eq = true;
#pragma unroll
      for (int w = 0; w < KW; ++w) eq = eq && (dk[w] == k[w]);
      if (eq) return true;
    }
    slot = (slot + 1) & V.mask;
  }
  return false;
}

// membership of a packed determinant key (det bits only) in the hash set of V;
// h is det_hash(k)
template <int KW>
SHCI_DEV bool vset_contains_h(const VSet& V, const uint64_t (&k)[KW], uint64_t h, int n) {
  return vfilt_maybe(V, h) && vset_probe<KW>(V, k, h, n);
}

template <int KW>
SHCI_DEV bool vset_contains(const VSet& V, const uint64_t (&k)[KW], int n) {
  return vset_contains_h<KW>(V, k, det_hash<KW>(k, n), n);
}

// Grouping hash of a term: the determinant hash with the sample id mixed in,
// so the terms of one a in one sample share it; even and never 0 (odd values
// mark the fillers of the hash list).
SHCI_DEV uint64_t group_hash(uint64_t h, uint32_t sid) {
  const uint64_t g = (h ^ ((uint64_t)sid * 0x9e3779b97f4a7c15ull)) & ~1ull;
  return g ? g : 2ull;
}
// filler of an unused slot p of the hash list: odd, spread like the hashes;
// its work item is HASH_HOLE
constexpr uint32_t HASH_HOLE = 0xffffffffu;
SHCI_DEV uint64_t hole_hash(uint64_t p) { return fmix64(p ^ 0x5851f42d4c957f2dull) | 1ull; }

struct LookupArgs {
  Uniq U;
  const int32_t* nseg = nullptr;
  GroupPlan G;
};

constexpr int DL_CAP = 32;  // differences from the reference kept for the singles filter

struct GenArgs {
  int n, na, nb;
  const uint64_t* dets;
  const double* c;
  int64_t n_items;         // work items
  const uint32_t* w_src;   // work item -> source (det, or distinct sampled det)
  const uint32_t* w_rng;   // work item -> occupied-pair range [lo, hi) as lo | hi << 16
  // sample mode: distinct sampled determinants
  const uint32_t* it_det;
  const uint32_t* it_w;
  const uint32_t* it_s;
  double sum_abs;
  double nd;
  double eps2, eps2_d;
  Tables T;
  uint32_t* flag;  // |= 32: a write walk kept a different number of terms than its count walk
  uint32_t* counts;
  const uint64_t* offs;
  Recs out;
  uint32_t* counter;
  int sbits, auxbit;
  uint32_t bmask, bsel;    // hash batch: keep a only if (hash(a) & bmask) == bsel
  const int32_t* sbatch;   // sample mode, nullable: batch of each sample (replaces bsel)
  int bits_hash;           // bucket id = top bits_hash bits of the key hash | sample id above
  // singles prefilter: Fock-like elements of a reference determinant R,
  // Fref[s][p][r] = h_pr + sum_{k in R_s, k != p} sD[k][p][r] + sum_{k in R_s'} sJ[k][p][r]
  const uint64_t* ref;
  const double* Fref;
  double smarg;            // rounding margin, in units of the bound U_pr
  LookupArgs L;
  double* grad;
  int pay_pos;             // payload: the record's own position (keep-mode adjoint) instead of the source
  // singleton split.  Count walk: the grouping hash and work item of every
  // kept term go to hkey / hitem, in runs of hrun >= 64 slots that each
  // wavefront claims from *hclaim (slots past hcap are not written; unused
  // slots of a claimed run are filled with hole_hash / HASH_HOLE).
  uint64_t* hkey;
  uint32_t* hitem;
  uint64_t hcap;
  unsigned long long* hclaim;
  int hrun;
  // Write walk: a term whose grouping hash passes the filter mfilt of hashes
  // seen more than once becomes a record (at offs of its work item, which
  // count such terms); every other term is the only one of its a, and its
  // contribution is summed in place into the work item's partials PI.
  const uint64_t* mfilt;
  int mfbits;
  VSet V;
  double e0;
  double inv_ndd;  // 1 / (N_d (N_d - 1))
  Partials PI;
};

SHCI_DEV int tri_inv(int u) {
  // largest y with y(y-1)/2 <= u
  int y = (int)floorf((1.0f + sqrtf(1.0f + 8.0f * (float)u)) * 0.5f);
  while (y * (y - 1) / 2 > u) --y;
  while ((y + 1) * y / 2 <= u) ++y;
  return y;
}

// Position of a unique key (flag bit clear; sample id in the key in sample
// mode) in the unique store, or -1.  Buckets and the in-bucket order use the
// determinant hash; sid selects the sample's range of buckets.
template <int KW>
SHCI_DEV int64_t lookup_u(const uint64_t (&key)[KW], int n, uint32_t sid, const LookupArgs& L) {
  const uint64_t h = det_hash<KW>(key, n);
  const int bh = L.G.bits_hash;
  const uint64_t b = (bh ? (h >> (64 - bh)) : 0ull) | ((uint64_t)sid << bh);
  const uint32_t h2 = (uint32_t)((h << bh) >> 32);
  const uint64_t lo = L.U.start[b];
  const int cnt = L.nseg[b];
  int a = 0, z = cnt;
  while (a < z) {
    const int m = (a + z) >> 1;
    if (L.U.h2[lo + m] < h2)
      a = m + 1;
    else
      z = m;
  }
  for (int j = a; j < cnt && L.U.h2[lo + j] == h2; ++j) {
    bool eq = true;
#pragma unroll
    for (int w = 0; w < KW; ++w) eq = eq && (L.U.k[w][lo + j] == key[w]);
    if (eq) return (int64_t)(lo + j);
  }
  return -1;
}

template <int KW, int MODE, bool SAMPLE, typename VT>
SHCI_DEV void gen_body(const GenArgs& a) {
  __shared__ uint8_t s_lists[4][4][128];
  __shared__ uint16_t s_dl[4][DL_CAP];   // differences of the source from R
  __shared__ uint16_t s_sq[4][128];      // queue of singles candidates
  __shared__ uint8_t s_plist[4][64];
  __shared__ uint8_t s_llist[4][64];
  __shared__ double s_F[4][256];         // Fock-like diagonal of the source, alpha | beta << 7
  __shared__ uint32_t s_dq[4][128];      // queue of kept doubles: excitation code
  __shared__ double s_dv[4][128];        //   and table value
  const int wv = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  uint8_t* occA = s_lists[wv][0];
  uint8_t* virA = s_lists[wv][1];
  uint8_t* occB = s_lists[wv][2];
  uint8_t* virB = s_lists[wv][3];
  const int n = a.n, na = a.na, nb = a.nb, va = n - a.na, vb = n - a.nb;
  const double eps2 = a.eps2;
  const Tables& T = a.T;

  // work items round-robin over wavefronts (heavy sources are already split
  // into several items, so a static assignment is balanced)
  const int64_t nwaves_total = (int64_t)gridDim.x * (blockDim.x >> 6);
  const int64_t wave_gid = (int64_t)blockIdx.x * (blockDim.x >> 6) + wv;
  const bool hmode = MODE == GEN_COUNT && a.hkey != nullptr;   // count walk lists grouping hashes
  const bool fmode = MODE == GEN_WRITE && a.mfilt != nullptr;  // write walk splits off singletons
  uint64_t hpos = 0, hend = 0;  // this wavefront's claimed run of the hash list (uniform)
  for (int64_t item = wave_gid; item < a.n_items; item += nwaves_total) {

    const int64_t src = a.w_src[item];
    const uint32_t rng = a.w_rng[item];
    const int pair_lo = (int)(rng & 0xffffu), pair_hi = (int)(rng >> 16);
    int64_t i = src;
    double w = 1.0;
    uint32_t sid = 0;
    if constexpr (SAMPLE) {
      i = a.it_det[src];
      w = (double)a.it_w[src];
      sid = a.it_s[src];
    }
    const uint64_t A0 = a.dets[4 * i + 0], A1 = a.dets[4 * i + 1];
    const uint64_t B0 = a.dets[4 * i + 2], B1 = a.dets[4 * i + 3];
    const double ci = a.c[i];
    const double absc = fabs(ci);
    double pr = 1.0;
    if constexpr (SAMPLE) pr = absc / a.sum_abs;
    // per-source factors of the stochastic estimator: x = (w / p) c H and
    // z = (w (N_d - 1) / p) (c H)^2 (the divisions once per source)
    const double wp = SAMPLE ? w / pr : 1.0;
    const double wq = SAMPLE ? w * (a.nd - 1.0) / pr : 1.0;

    // occupied / virtual lists of both spins in LDS (wave-private)
    {
      const bool inlo = lane < n, inhi = lane + 64 < n;
      const bool oa0 = inlo && ((A0 >> lane) & 1ull), oa1 = inhi && ((A1 >> lane) & 1ull);
      const bool ob0 = inlo && ((B0 >> lane) & 1ull), ob1 = inhi && ((B1 >> lane) & 1ull);
      uint64_t m;
      m = ballot(oa0);
      if (oa0) occA[rank_below(m)] = (uint8_t)lane;
      int c0 = __popcll(m);
      m = ballot(oa1);
      if (oa1) occA[c0 + rank_below(m)] = (uint8_t)(lane + 64);
      m = ballot(inlo && !oa0);
      if (inlo && !oa0) virA[rank_below(m)] = (uint8_t)lane;
      c0 = __popcll(m);
      m = ballot(inhi && !oa1);
      if (inhi && !oa1) virA[c0 + rank_below(m)] = (uint8_t)(lane + 64);
      m = ballot(ob0);
      if (ob0) occB[rank_below(m)] = (uint8_t)lane;
      c0 = __popcll(m);
      m = ballot(ob1);
      if (ob1) occB[c0 + rank_below(m)] = (uint8_t)(lane + 64);
      m = ballot(inlo && !ob0);
      if (inlo && !ob0) virB[rank_below(m)] = (uint8_t)lane;
      c0 = __popcll(m);
      m = ballot(inhi && !ob1);
      if (inhi && !ob1) virB[c0 + rank_below(m)] = (uint8_t)(lane + 64);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    // H_aa of every written term is an update of the source's H_ii by the
    // Fock-like diagonal F of the source (both spins, one orbital per lane)
    double hii = 0.0;
    double* Fw = s_F[wv];
    const DiagLayout DL = DiagLayout::make(n);
    if constexpr (MODE == GEN_WRITE) {
      double part = 0.0;
      for (int x = lane; x < n; x += 64) {
        double fa, fb;
        fock_diag2(T.diag, DL, x, occA, na, occB, nb, fa, fb);
        Fw[x] = fa;
        Fw[128 + x] = fb;
        const double hx = T.diag[x];
        if (occ(A0, A1, x)) part += hx + fa;
        if (occ(B0, B1, x)) part += hx + fb;
      }
      // butterfly: every lane ends with the same (commutative) sum
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) part += __shfl_xor(part, o);
      hii = 0.5 * part;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }

    uint64_t obase = 0, oend = 0;
    if constexpr (MODE == GEN_WRITE) {
      obase = a.offs[item];
      oend = a.offs[item + 1];
    }
    uint64_t cursor = 0;  // uniform
    double gacc = 0.0;
    // in-place sums of the singletons of this work item (per lane)
    double fe2 = 0.0, fde0 = 0.0, fe2sq = 0.0, fdmn = INFINITY;
    int64_t fnt = 0, fng = 0;
    int32_t fnu = 0, fni = 0, fnz = 0;

    auto emit = [&](bool keep, uint64_t x0, uint64_t x1, uint64_t y0, uint64_t y1, double H, double haa) {
      if (a.bmask) {  // uniform
        if (keep) {
          uint64_t hk[KW];
          pack_det<KW>(hk, x0, x1, y0, y1, n);
          const uint32_t want = (SAMPLE && a.sbatch) ? (uint32_t)a.sbatch[sid] : a.bsel;
          keep = ((uint32_t)det_hash<KW>(hk, n) & a.bmask) == want;
        }
      }
      const uint64_t bal = ballot(keep);
      if constexpr (MODE == GEN_COUNT) {
        if (hmode) {
          // grouping hash of every kept term into this wavefront's run of
          // the hash list (a new run is claimed when the current one is full)
          uint64_t g = 0;
          if (keep) {
            uint64_t key[KW];
            pack_det<KW>(key, x0, x1, y0, y1, n);
            g = group_hash(det_hash<KW>(key, n), sid);
          }
          const uint64_t cnt = (uint64_t)__popcll(bal);
          const uint64_t r = (uint64_t)rank_below(bal);
          const uint64_t room = hend - hpos;
          uint64_t pos = hpos + r;
          if (cnt > room) {
            unsigned long long nb = 0;
            if (lane == 0) nb = atomicAdd(a.hclaim, (unsigned long long)a.hrun);
            nb = __shfl(nb, 0);
            if (r >= room) pos = (uint64_t)nb + (r - room);
            hpos = (uint64_t)nb + (cnt - room);
            hend = (uint64_t)nb + (uint64_t)a.hrun;
          } else {
            hpos += cnt;
          }
          if (keep && pos < a.hcap) {
            a.hkey[pos] = g;
            a.hitem[pos] = (uint32_t)item;
          }
        }
        cursor += (uint64_t)__popcll(bal);
      } else if constexpr (MODE == GEN_WRITE) {
        uint64_t key[KW];
        uint64_t h = 0;
        if (keep) {
          pack_det<KW>(key, x0, x1, y0, y1, n);
          h = det_hash<KW>(key, n);
        }
        bool wr = keep, single = false;
        if (fmode) {
          // a grouping hash outside the filter of repeated hashes: this
          // term is the only one of its a (in its sample)
          single = keep && !filt_maybe(a.mfilt, a.mfbits, group_hash(h, sid));
          wr = keep && !single;
        }
        const uint64_t bw = fmode ? ballot(wr) : bal;
        const uint64_t pos = obase + cursor + (uint64_t)rank_below(bw);
        if (wr && pos < oend) {  // the count walk sized [obase, oend)
          {
            // bucket id: top hash bits of the determinant, sample id above
            uint32_t b = a.bits_hash ? (uint32_t)(h >> (64 - a.bits_hash)) : 0u;
            if constexpr (SAMPLE) b |= sid << a.bits_hash;
            a.out.bid[pos] = b;
          }
          if constexpr (SAMPLE) put_bits<KW>(key, (uint64_t)sid, 0ull, 2 * n);
          if constexpr (SAMPLE) {
            if (fabs(H) * absc > a.eps2_d) put_bits<KW>(key, 1ull, 0ull, a.auxbit);
            const double ch = ci * H;
            // x and z = x^2 + y of the stochastic estimator (see SegSum)
            const double xv = wp * ch;
            const double zv = wq * ch * ch;
            static_cast<VT*>(a.out.v)[pos] = (VT)xv;
            static_cast<VT*>(a.out.v2)[pos] = (VT)zv;
          } else {
            // flag: the term also passes the upper threshold of a
            // two-threshold evaluation (eps2_d is infinite otherwise)
            if (fabs(H) * absc > a.eps2_d) put_bits<KW>(key, 1ull, 0ull, a.auxbit);
            VT t;
            if constexpr (sizeof(VT) == 4)
              t = (float)H * (float)ci;
            else
              t = H * ci;
            static_cast<VT*>(a.out.v)[pos] = t;
          }
#pragma unroll
          for (int q = 0; q < KW; ++q) a.out.k[q][pos] = key[q];
          a.out.haa[pos] = haa;
          if (a.out.pay) a.out.pay[pos] = a.pay_pos ? (uint32_t)pos : (uint32_t)i;
        }
        cursor += (uint64_t)__popcll(bw);
        if (single) {
          // the bucket reduce of a segment of one term, in place: a in V
          // is dropped; otherwise A_a = t (deterministic) or the sample
          // bracket reduces to z (X^2 - Q = 0 exactly for one term), and a
          // term above the upper threshold cancels its own contribution
          fng += 1;
          if (!vset_contains_h<KW>(a.V, key, h, n)) {
            const bool up = fabs(H) * absc > a.eps2_d;
            const double Dd = a.e0 - haa;
            const double rd = 1.0 / Dd;
            double contrib;
            if constexpr (SAMPLE) {
              const double ch = ci * H;
              const double z = (double)(VT)(wq * ch * ch);
              const double G = rd * a.inv_ndd;
              contrib = (up ? 0.0 : z) * G;
              fde0 += -contrib * rd;
            } else {
              double X;
              if constexpr (sizeof(VT) == 4)
                X = (double)((float)H * (float)ci);
              else
                X = H * ci;
              const double a2 = up ? 0.0 : X * X;
              contrib = a2 * rd;
              fde0 += -a2 * rd * rd;
            }
            fe2 += contrib;
            fe2sq += contrib * contrib;
            fnt += 1;
            fnu += 1;
            fni += Dd > 0.0;
            fnz += Dd == 0.0;
            fdmn = fmin(fdmn, fabs(Dd));
          }
        }
      } else {  // GEN_GRAD
        if (keep) {
          uint64_t key[KW];
          pack_det<KW>(key, x0, x1, y0, y1, n);
          if constexpr (SAMPLE) put_bits<KW>(key, (uint64_t)sid, 0ull, 2 * n);
          const int64_t o = lookup_u<KW>(key, n, sid, a.L);
          if (o >= 0) {
            if constexpr (SAMPLE) {
              // d/dc_i of the sample bracket (X^2 - Q + Z) - (X_d^2 - Q_d + Z_d)
              // at frozen w, p and masks, in the same cancellation-free form
              // as the forward: 2 (X - x_i) w H / p + 2 w (N_d - 1) / p c H^2,
              // minus the same with X_d for terms above eps2_d (stored
              // factors 2 X G, 2 X_d G and G; x_i rounded as stored)
              const double wh = wp * H;
              const double G = a.L.U.D[o];
              const bool dflag = fabs(H) * absc > a.eps2_d;
              if (dflag) {
                gacc += (a.L.U.g[o] - a.L.U.A[o]) * wh;
              } else {
                const double xi = (double)(VT)(wp * (ci * H));
                gacc += (a.L.U.g[o] - 2.0 * xi * G) * wh + 2.0 * wq * ci * H * H * G;
              }
            } else {
              gacc += H * a.L.U.g[o];
            }
          }
        }
      }
    };

    // ---------------- singles ----------------
    // The screened element is the exact one, summed in the canonical order
    // (h_pr, occupied alpha ascending, occupied beta ascending; same-spin k
    // add (pr|kk)-(pk|kr) for k != p, other-spin k add (pr|kk)).  Two cheap
    // filters run first: the bound U_pr |c_i| <= eps2, then the same element
    // evaluated relative to R (Fref plus the orbitals where the source and R
    // differ) with a margin that covers the rounding of both sums.  Survivors
    // are queued and evaluated exactly 64 at a time, in candidate order.
    const int nsa = na * va, nsing = (pair_lo == 0) ? nsa + nb * vb : 0;  // singles with the first range
    if (nsing > 0) {
      const size_t nn = (size_t)n * n;
      // difference list: alpha particles, alpha holes, beta particles, beta
      // holes (entry k | spin << 7 | hole << 8)
      int ndl = 0;
      {
        const uint64_t R0 = a.ref[0], R1 = a.ref[1], R2 = a.ref[2], R3 = a.ref[3];
        const uint64_t dm[8] = {A0 & ~R0, A1 & ~R1, R0 & ~A0, R1 & ~A1,
                                B0 & ~R2, B1 & ~R3, R2 & ~B0, R3 & ~B1};
        int tot = 0;
#pragma unroll
        for (int w = 0; w < 8; ++w) tot += __popcll(dm[w]);
        if (tot <= DL_CAP) {
#pragma unroll
          for (int w = 0; w < 8; ++w) {
            const bool in = (w & 1) ? (lane + 64 < n && ((dm[w] >> lane) & 1ull)) : (lane < n && ((dm[w] >> lane) & 1ull));
            const uint64_t m = ballot(in);
            if (in)
              s_dl[wv][ndl + rank_below(m)] =
                  (uint16_t)((lane + ((w & 1) ? 64 : 0)) | ((w >> 2) << 7) | (((w >> 1) & 1) << 8));
            ndl += __popcll(m);
          }
        } else {
          ndl = -1;  // too far from R: no relative filter
        }
      }
      uint16_t* sq = s_sq[wv];
      int qn = 0;  // uniform
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      // candidate j -> (spin, p, r); the division by the number of virtual
      // orbitals goes through a float reciprocal with one integer correction
      // (exact for j < 2^24)
      const float inv_va = va ? 1.0f / (float)va : 0.0f, inv_vb = vb ? 1.0f / (float)vb : 0.0f;
      auto cand_of = [&](int j, bool& alpha, int& p, int& r) {
        alpha = j < nsa;
        const int jj = alpha ? j : j - nsa;
        const int d = alpha ? va : vb;
        int q = (int)((float)jj * (alpha ? inv_va : inv_vb));
        int rm = jj - q * d;
        if (rm < 0) {
          --q;
          rm += d;
        } else if (rm >= d) {
          ++q;
          rm -= d;
        }
        p = alpha ? occA[q] : occB[q];
        r = alpha ? virA[rm] : virB[rm];
      };
      // exact evaluation and emission of queue entries [0, cnt)
      auto process = [&](int cnt) {
        const bool valid = lane < cnt;
        bool alpha = true;
        int p = 0, r = 0;
        if (valid) cand_of((int)sq[lane], alpha, p, r);
        double H = 0.0;
        if (valid) {
          const size_t pr_off = (size_t)p * n + r;
          const double* tabA = alpha ? T.sD : T.sJ;
          const double* tabB = alpha ? T.sJ : T.sD;
          double acc = T.h1[pr_off];
          for (int kk0 = 0; kk0 < na; kk0 += 8) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
              v[u] = 0.0;
              if (kk0 + u < na) v[u] = tabA[occA[kk0 + u] * nn + pr_off];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u)
              if (kk0 + u < na && !(alpha && occA[kk0 + u] == p)) acc = acc + v[u];
          }
          for (int kk0 = 0; kk0 < nb; kk0 += 8) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
              v[u] = 0.0;
              if (kk0 + u < nb) v[u] = tabB[occB[kk0 + u] * nn + pr_off];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u)
              if (kk0 + u < nb && !(!alpha && occB[kk0 + u] == p)) acc = acc + v[u];
          }
          const int par = alpha ? between(A0, A1, p, r) : between(B0, B1, p, r);
          H = (par & 1) ? -acc : acc;
        }
        const bool keep = valid && (fabs(H) * absc > eps2);
        uint64_t x0 = A0, x1 = A1, y0 = B0, y1 = B1;
        if (alpha) {
          flip(x0, x1, p);
          flip(x0, x1, r);
        } else {
          flip(y0, y1, p);
          flip(y0, y1, r);
        }
        double haa = 0.0;
        if constexpr (MODE == GEN_WRITE) {
          if (keep) haa = hii + en_single(Fw + (alpha ? 0 : 128), T.diag, DL, p, r);
        }
        emit(keep, x0, x1, y0, y1, H, haa);
      };
      for (int j0 = 0; j0 < nsing; j0 += 64) {
        const int j = j0 + lane;
        const bool valid = j < nsing;
        bool alpha = true;
        int p = 0, r = 0;
        if (valid) cand_of(j, alpha, p, r);
        const size_t pr_off = (size_t)p * n + r;
        const double ub = valid ? T.ubound[pr_off] : 0.0;
        bool maybe = valid && (ub * absc > eps2);
        bool sure = false;  // kept for certain (count walk without batch filter)
        if (ndl >= 0 && maybe) {
          const int sp = alpha ? 0 : 1;
          double h = a.Fref[sp * nn + pr_off];
          // corrections loaded eight at a time
          for (int t0 = 0; t0 < ndl; t0 += 8) {
            double v[8];
            uint32_t e[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
              e[u] = (t0 + u < ndl) ? (uint32_t)s_dl[wv][t0 + u] : 0xffffu;
              const int k = (int)(e[u] & 127u);
              const bool same = (int)((e[u] >> 7) & 1u) == sp;
              v[u] = 0.0;
              if (e[u] != 0xffffu && !(same && k == p)) v[u] = (same ? T.sD : T.sJ)[k * nn + pr_off];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) h = ((e[u] >> 8) & 1u) ? h - v[u] : h + v[u];
          }
          maybe = (fabs(h) + a.smarg * ub) * absc * (1.0 + 0x1p-50) > eps2;
          // the margin bounds |H - h| several times over, so this implies the
          // exact element passes; only counting needs no value
          if constexpr (MODE == GEN_COUNT) sure = (fabs(h) - a.smarg * ub) * absc * (1.0 - 0x1p-50) > eps2;
        }
        if constexpr (MODE == GEN_COUNT) {
          if (a.bmask == 0u) {  // uniform
            if (hmode) {
              // listed without the exact element: only the key is needed
              uint64_t x0 = A0, x1 = A1, y0 = B0, y1 = B1;
              if (alpha) {
                flip(x0, x1, p);
                flip(x0, x1, r);
              } else {
                flip(y0, y1, p);
                flip(y0, y1, r);
              }
              emit(sure, x0, x1, y0, y1, 0.0, 0.0);
            } else {
              cursor += (uint64_t)__popcll(ballot(sure));
            }
            maybe = maybe && !sure;
          }
        }
        const uint64_t mb = ballot(maybe);
        if (maybe) sq[qn + rank_below(mb)] = (uint16_t)j;
        qn += __popcll(mb);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (qn >= 64) {
          process(64);
          const uint16_t rest = (lane + 64 < qn) ? sq[lane + 64] : (uint16_t)0;
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
          if (lane + 64 < qn) sq[lane] = rest;
          qn -= 64;
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
      }
      if (qn > 0) process(qn);
    }

    // ---------------- doubles ----------------
    // Occupied pairs in windows of 64.  Pairs whose largest element can pass
    // are probed eight at a time (8 lanes each, first 8 entries); pairs whose
    // first 8 entries all pass are walked afterwards 64 entries at a time.
    const int caa = na * (na - 1) / 2, cbb = nb * (nb - 1) / 2;
    const float inv_nb = nb ? 1.0f / (float)nb : 0.0f;
    auto decode = [&](int u, int& p, int& q, int& type, int64_t& off, int64_t& len) {
      if (u < caa) {
        const int y = tri_inv(u), x = u - y * (y - 1) / 2;
        p = occA[x];
        q = occA[y];
        type = 0;
      } else if (u < caa + cbb) {
        const int v = u - caa;
        const int y = tri_inv(v), x = v - y * (y - 1) / 2;
        p = occB[x];
        q = occB[y];
        type = 1;
      } else {
        const int v = u - caa - cbb;
        int qa = (int)((float)v * inv_nb);
        int rb = v - qa * nb;
        if (rb < 0) {
          --qa;
          rb += nb;
        } else if (rb >= nb) {
          ++qa;
          rb -= nb;
        }
        p = occA[qa];
        q = occB[rb];
        type = 2;
      }
      if (type < 2) {
        off = (int64_t)(q * (q - 1) / 2 + p) * T.lss;
        len = T.lss;
      } else {
        off = (int64_t)T.nss * T.lss + (int64_t)(p * n + q) * T.los;
        len = T.los;
      }
    };
    // Kept doubles are queued (type << 28 | p << 21 | q << 14 | r << 7 | s,
    // and the table value) and written 64 at a time, so the key, hash, H_aa
    // and stores of a write run on full wavefronts.  Plain counting needs
    // no queue.
    const bool dqueue = MODE != GEN_COUNT || a.bmask != 0u || hmode;  // uniform
    uint32_t* dq = s_dq[wv];
    double* dv = s_dv[wv];
    int dqn = 0;  // uniform
    auto dflush = [&](int cnt) {
      const bool valid = lane < cnt;
      const uint32_t cd = valid ? dq[lane] : 0u;
      const double v = valid ? dv[lane] : 0.0;
      const int type = (int)(cd >> 28), p = (int)((cd >> 21) & 127u), q = (int)((cd >> 14) & 127u),
                r = (int)((cd >> 7) & 127u), s2 = (int)(cd & 127u);
      uint64_t x0 = A0, x1 = A1, y0 = B0, y1 = B1;
      int par = 0;
      if (type == 0) {
        par = between(x0, x1, p, r);
        flip(x0, x1, p);
        flip(x0, x1, r);
        par += between(x0, x1, q, s2);
        flip(x0, x1, q);
        flip(x0, x1, s2);
      } else if (type == 1) {
        par = between(y0, y1, p, r);
        flip(y0, y1, p);
        flip(y0, y1, r);
        par += between(y0, y1, q, s2);
        flip(y0, y1, q);
        flip(y0, y1, s2);
      } else {
        par = between(A0, A1, p, r) + between(B0, B1, q, s2);
        flip(x0, x1, p);
        flip(x0, x1, r);
        flip(y0, y1, q);
        flip(y0, y1, s2);
      }
      double haa = 0.0;
      if constexpr (MODE == GEN_WRITE) {
        if (valid)
          haa = hii + en_double(Fw + (type == 1 ? 128 : 0), Fw + (type == 0 ? 0 : 128), T.diag, DL, p, q,
                                r, s2, type < 2);
      }
      emit(valid, x0, x1, y0, y1, (par & 1) ? -v : v, haa);
    };
    // one heat-bath entry (value v, target rs) of pair (p, q, type)
    auto dbl = [&](bool pass, int type, int p, int q, double v, uint16_t rs) {
      const int r = rs & 0xff, s2 = rs >> 8;
      bool keep = pass;
      if (type == 0)
        keep = keep && !occ(A0, A1, r) && !occ(A0, A1, s2);
      else if (type == 1)
        keep = keep && !occ(B0, B1, r) && !occ(B0, B1, s2);
      else
        keep = keep && !occ(A0, A1, r) && !occ(B0, B1, s2);
      const uint64_t bal = ballot(keep);
      if (!dqueue) {
        cursor += (uint64_t)__popcll(bal);
        return;
      }
      if (keep) {
        const int o = dqn + rank_below(bal);
        dq[o] = ((uint32_t)type << 28) | ((uint32_t)p << 21) | ((uint32_t)q << 14) | ((uint32_t)r << 7) |
                (uint32_t)s2;
        dv[o] = v;
      }
      dqn += __popcll(bal);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      if (dqn >= 64) {
        dflush(64);
        const bool mv = lane + 64 < dqn;
        const uint32_t rc = mv ? dq[lane + 64] : 0u;
        const double rv = mv ? dv[lane + 64] : 0.0;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (mv) {
          dq[lane] = rc;
          dv[lane] = rv;
        }
        dqn -= 64;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
    };
    uint8_t* plist = s_plist[wv];
    uint8_t* llist = s_llist[wv];
    for (int u0 = pair_lo; u0 < pair_hi; u0 += 64) {
      const int u = u0 + lane;
      bool need = false;
      if (u < pair_hi) {
        int p, q, type;
        int64_t off, len;
        decode(u, p, q, type, off, len);
        const int key = (type < 2) ? q * (q - 1) / 2 + p : T.nss + p * n + q;
        need = T.hb_max[key] * absc > eps2;
      }
      const uint64_t nb_ = ballot(need);
      const int nneed = __popcll(nb_);
      if (need) plist[rank_below(nb_)] = (uint8_t)lane;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      int nlong = 0;
      const int g = lane >> 3, sl = lane & 7;
      for (int r0 = 0; r0 < nneed; r0 += 8) {
        const int pi = r0 + g;
        const bool active = pi < nneed;
        int p = 0, q = 0, type = 0;
        int64_t off = 0, len = 0;
        if (active) decode(u0 + plist[pi], p, q, type, off, len);
        const bool valid = active && sl < len;
        double v = 0.0;
        uint16_t rs = 0;
        if (valid) {
          v = T.hb_val[off + sl];
          rs = T.hb_rs[off + sl];
        }
        const bool pass = valid && (fabs(v) * absc > eps2);
        const uint64_t pb = ballot(pass);
        dbl(pass, type, p, q, v, rs);
        const bool is_long = active && sl == 0 && ((pb >> (g * 8)) & 0xffull) == 0xffull && len > 8;
        const uint64_t lb = ballot(is_long);
        if (is_long) llist[nlong + rank_below(lb)] = plist[pi];
        nlong += __popcll(lb);
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      for (int li = 0; li < nlong; ++li) {
        int p, q, type;
        int64_t off, len;
        decode(u0 + llist[li], p, q, type, off, len);  // uniform
        for (int64_t e0 = 8; e0 < len; e0 += 64) {
          const int64_t e = e0 + lane;
          double v = 0.0;
          uint16_t rs = 0;
          if (e < len) {
            v = T.hb_val[off + e];
            rs = T.hb_rs[off + e];
          }
          const bool pass = (e < len) && (fabs(v) * absc > eps2);
          const uint64_t pb = ballot(pass);
          if (pb == 0ull) break;
          dbl(pass, type, p, q, v, rs);
          if (pb != ~0ull) break;
        }
      }
    }

    if (dqn > 0) dflush(dqn);
    if constexpr (MODE == GEN_COUNT) {
      if (lane == 0) a.counts[item] = (uint32_t)cursor;
    }
    if constexpr (MODE == GEN_WRITE) {
      if (lane == 0 && obase + cursor != oend) atomicOr(a.flag, 32u);
      if (fmode) {
        // the work item's singleton partials (fixed butterfly)
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
          fe2 += __shfl_xor(fe2, o);
          fde0 += __shfl_xor(fde0, o);
          fe2sq += __shfl_xor(fe2sq, o);
          fdmn = fmin(fdmn, __shfl_xor(fdmn, o));
          fnt += __shfl_xor(fnt, o);
          fng += __shfl_xor(fng, o);
          fnu += __shfl_xor(fnu, o);
          fni += __shfl_xor(fni, o);
          fnz += __shfl_xor(fnz, o);
        }
        if (lane == 0) {
          a.PI.e2[item] = fe2;
          a.PI.de0[item] = fde0;
          a.PI.e2sq[item] = fe2sq;
          a.PI.mind[item] = fdmn;
          a.PI.nterm[item] = fnt;
          a.PI.ngen[item] = fng;
          a.PI.nuniq[item] = fnu;
          a.PI.nintr[item] = fni;
          a.PI.nzero[item] = fnz;
        }
      }
    }
    if constexpr (MODE == GEN_GRAD) {
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) gacc += __shfl_xor(gacc, o);
      if (lane == 0) a.grad[item] = gacc;  // per work item; summed per source afterwards
    }
    __builtin_amdgcn_wave_barrier();
  }
  if (hmode) {
    // the rest of the last claimed run: distinct fillers without a work item
    for (uint64_t p = hpos + (uint64_t)lane; p < hend; p += 64)
      if (p < a.hcap) {
        a.hkey[p] = hole_hash(p);
        a.hitem[p] = HASH_HOLE;
      }
  }
}

// The walks of the generator.  The count walk carries the least state and
// gains from six wavefronts per SIMD, the deterministic write walk from five,
// the sample write walk (in-place sums of the singleton split) from four; the
// adjoint walk keeps the compiler's choice (all measured).
template <int KW, bool SAMPLE, typename VT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6, 8))) k_gen_count(GenArgs a) {
  gen_body<KW, GEN_COUNT, SAMPLE, VT>(a);
}
template <int KW, typename VT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5, 8))) k_gen_write(GenArgs a) {
  gen_body<KW, GEN_WRITE, false, VT>(a);
}
template <int KW, typename VT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8))) k_gen_write_sample(GenArgs a) {
  gen_body<KW, GEN_WRITE, true, VT>(a);
}
template <int KW, bool SAMPLE, typename VT>
__global__ void __launch_bounds__(256) k_gen_grad(GenArgs a) {
  gen_body<KW, GEN_GRAD, SAMPLE, VT>(a);
}

// dE2/dc_i = sum of the partial adjoints of the work items of source i, in
// item order
// sample mode: add each item's adjoint to its determinant; the items of one
// sample are distinct determinants, so one launch per sample has no conflicts
// and the sample order fixes the summation order
__global__ void k_grad_scatter(const double* gitem, const uint32_t* it_det, int64_t count, double scale,
                               double* grad) {
  const int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (u < count) grad[it_det[u]] += scale * gitem[u];
}

// grad[s] (+)= sum of the parts of source s's work items (divided by c_s
// when c is given: the keep-mode parts hold t * 2 A_a / D_a with t = H_ai c_i)
__global__ void k_grad_sum(const uint32_t* nsplit, const uint64_t* off, const double* part, int64_t n_src,
                           double* grad, int accumulate, const double* c = nullptr) {
  const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= n_src) return;
  double g = 0.0;
  for (uint32_t j = 0; j < nsplit[s]; ++j) g += part[off[s] + j];
  if (c) g = g == 0.0 ? 0.0 : g / c[s];
  grad[s] = accumulate ? grad[s] + g : g;  // hash batches add in batch order
}

// keep-mode adjoint: part[item] = sum of the per-record terms of the item's
// records (generation order; one wavefront per item, fixed butterfly)
__global__ void k_keep_item_sum(const uint64_t* offs, int64_t n_items, const double* contrib, double* part) {
  const int64_t item = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (item >= n_items) return;
  const uint64_t lo = offs[item], hi = offs[item + 1];
  double s = 0.0;
  for (uint64_t r = lo + lane; r < hi; r += 64) s += contrib[r];
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o);
  if (lane == 0) part[item] = s;
}

// Work split: a source whose heat-bath walks are long (small eps2 / |c_i|) is
// cut into several work items over its occupied pairs, so that no wavefront
// walks far more entries than the others.  The estimate uses, per table kind,
// the number of entries with |value| >= 2^e (mag_cum), at e = floor(log2 t).
constexpr double SPLIT_TARGET = 4096.0;  // estimated passing entries per work item

struct SplitArgs {
  int n, na, nb;
  int nss;
  int64_t lss, los;
  const double* c;
  const uint32_t* it_det;  // sample mode (nullable)
  int64_t n_src;
  double eps2;
  const double* mag_cum;   // [2][72]: same-spin, opposite-spin
  uint32_t* nsplit;        // [n_src]
};

SHCI_DEV int npairs_of(int na, int nb) { return na * (na - 1) / 2 + nb * (nb - 1) / 2 + na * nb; }

__global__ void k_split_count(SplitArgs a) {
  const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= a.n_src) return;
  const int64_t i = a.it_det ? (int64_t)a.it_det[s] : s;
  const double absc = fabs(a.c[i]);
  const int npairs = npairs_of(a.na, a.nb);
  double ess = 0.0, eos = 0.0;
  if (absc > 0.0) {
    const double t = a.eps2 / absc;
    if (t <= 0.0) {
      ess = (double)a.lss;
      eos = (double)a.los;
    } else {
      int e = ilogb(t);
      e = e < -64 ? -64 : (e > 7 ? 7 : e);
      ess = a.mag_cum[e + 64] / (a.nss > 0 ? a.nss : 1);
      eos = a.mag_cum[72 + e + 64] / ((double)a.n * a.n);
    }
  }
  const int pss = a.na * (a.na - 1) / 2 + a.nb * (a.nb - 1) / 2, pos = a.na * a.nb;
  const double work = pss * ess + pos * eos;
  int k = (int)ceil(work / SPLIT_TARGET);
  k = k < 1 ? 1 : (k > npairs ? npairs : k);
  a.nsplit[s] = (uint32_t)k;
}

__global__ void k_split_fill(const uint32_t* nsplit, const uint64_t* off, int64_t n_src, int npairs,
                             uint32_t* w_src, uint32_t* w_rng) {
  const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= n_src) return;
  const int k = (int)nsplit[s];
  const uint64_t o = off[s];
  for (int j = 0; j < k; ++j) {
    const int lo = (int)((int64_t)j * npairs / k), hi = (int)((int64_t)(j + 1) * npairs / k);
    w_src[o + j] = (uint32_t)s;
    w_rng[o + j] = (uint32_t)lo | ((uint32_t)hi << 16);
  }
}

}  // namespace shci
