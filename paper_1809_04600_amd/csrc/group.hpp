// Grouping of screened terms by perturbative determinant a, and the reduction
// of each group to its contribution A_a^2 / (E0 - H_aa).
//
// The paper accumulates the partial sums A_a = sum_i H_ai c_i in a concurrent
// hash table (section V.C).  Here the terms that need grouping are
// materialised as records (packed key of a, value(s), H_aa from the
// generator) and grouped by a hash partition instead (with the singleton
// split, hashsplit.hpp, only the terms whose a may have several terms):
//  1. a least-significant-digit radix partition of the records on the bucket
//     id (the top bits of a 64-bit hash of the key; in sample mode the sample
//     id sits above them), 8 bits per pass, stable: per 8192-record tile,
//     each wavefront ranks its slice by ballot matching, one scan places the
//     digits, and every array goes out through LDS as contiguous digit runs;
//  2. per bucket, one wavefront (reduce_wave.hpp): the bucket's records are
//     read once into registers, 32-bit sort keys (hash bits below the bucket
//     id, record position) are sorted by a bitonic network across lanes, so
//     equal keys become adjacent in record order; segment heads add their
//     members' values (deterministic order); buckets too large, or with two
//     keys sharing the sorted bits, go to a block kernel that sorts by the
//     full key;
//  3. members of V are dropped by a lookup in a hash set of V behind a
//     presence filter; H_aa is the one the generator computed (an update of
//     the source's diagonal, diag.hpp), taken from the segment's first
//     record; the contribution and dE2/dE0 term are summed per wavefront in a
//     fixed order;
//  4. the partials are summed by fixed-shape trees.
#pragma once
#include "gen.hpp"
#include "diag.hpp"

namespace shci {

constexpr int PTILE_ITEMS = 32;               // records per thread per partition tile
                                              // (8192-record tiles: longer digit runs per
                                              // tile; faster than 4096 on passes of ~1e9
                                              // records, ~9% slower on 1e7)
constexpr int PTILE = 256 * PTILE_ITEMS;      // records per partition tile

// Per-a accumulation of the terms of one segment (records of equal a).
// Deterministic mode: A = sum of t = H c.  Sample mode: each record holds
// x = w c H / p and z = x^2 + y = w (N_d - 1) / p (c H)^2, where y is the
// second term of the stochastic estimator; then X^2 + Y = (X^2 - Q) + Z with
// X = sum x, Q = sum x^2, Z = sum z.  For an a reached by one term X^2 - Q
// is exactly 0, so the estimator does not subtract two nearly equal numbers.
// FP32 values are summed with TwoSum (hi, lo); x^2 of an FP32 x is exact in
// FP64.  Terms flagged with the deterministic-threshold bit also enter the
// *d sums.
template <typename VT>
struct SegSum {
  double X = 0.0, Q = 0.0, Z = 0.0, Xd = 0.0, Qd = 0.0, Zd = 0.0;
  float xs = 0.f, xc = 0.f, zs = 0.f, zc = 0.f, xds = 0.f, xdc = 0.f, zds = 0.f, zdc = 0.f;
  // deterministic term; d: the term also passes the upper threshold of a
  // two-threshold evaluation (its sum is X_d)
  SHCI_DEV void add(VT x, bool d) {
    if constexpr (sizeof(VT) == 4) {
      two_sum_f32(xs, xc, (float)x);
      if (d) two_sum_f32(xds, xdc, (float)x);
    } else {
      X = X + (double)x;
      if (d) Xd = Xd + (double)x;
    }
  }
  SHCI_DEV void add_sample(VT x, VT z, bool d) {
    const double xq = (double)x * (double)x;
    Q = Q + xq;
    if constexpr (sizeof(VT) == 4) {
      two_sum_f32(xs, xc, (float)x);
      two_sum_f32(zs, zc, (float)z);
      if (d) {
        two_sum_f32(xds, xdc, (float)x);
        two_sum_f32(zds, zdc, (float)z);
        Qd = Qd + xq;
      }
    } else {
      X = X + (double)x;
      Z = Z + (double)z;
      if (d) {
        Xd = Xd + (double)x;
        Zd = Zd + (double)z;
        Qd = Qd + xq;
      }
    }
  }
  SHCI_DEV void finish() {
    if constexpr (sizeof(VT) == 4) {
      X = (double)xs + (double)xc;
      Z = (double)zs + (double)zc;
      Xd = (double)xds + (double)xdc;
      Zd = (double)zds + (double)zdc;
    }
  }
  // (X^2 + Y) - (X_d^2 + Y_d)
  SHCI_DEV double sample_bracket() const { return ((X * X - Q) + Z) - ((Xd * Xd - Qd) + Zd); }
};

template <int KW>
SHCI_DEV void load_key(const Recs& r, int64_t idx, uint64_t (&k)[KW]) {
#pragma unroll
  for (int w = 0; w < KW; ++w) k[w] = r.k[w][idx];
}

// bucket id of a key (aux bit cleared) and its 64-bit hash
template <int KW>
SHCI_DEV uint64_t bucket_id(const uint64_t (&k)[KW], const GroupPlan& G, int n, uint64_t& h) {
  h = det_hash<KW>(k, n);
  uint64_t b = G.bits_hash ? (h >> (64 - G.bits_hash)) : 0ull;
  if (G.sbits) {
    uint64_t s0, s1;
    get_bits<KW>(k, 2 * n, G.sbits, s0, s1);
    b |= s0 << G.bits_hash;
  }
  return b;
}

SHCI_DEV uint32_t sort_hash(uint64_t h, const GroupPlan& G) {
  return (uint32_t)((h << G.bits_hash) >> 32);
}

// ---------------------------------------------------------------------------
// Block-level stable multisplit of up to 256 items per round (8-bit digits).
// run[d] holds the next free slot of digit d; wcnt is per-wave scratch that
// must be zero on entry and is left zero.
// ---------------------------------------------------------------------------
struct SplitScratch {
  uint32_t run[256];
  uint16_t wcnt[4][256];
};

SHCI_DEV uint32_t split_round(SplitScratch& S, bool valid, uint32_t d, int dbits) {
  const int wv = threadIdx.x >> 6;
  uint64_t peers = ballot(valid);
  for (int b = 0; b < dbits; ++b) {
    const bool on = (d >> b) & 1u;
    const uint64_t bb = ballot(on);
    peers &= on ? bb : ~bb;
  }
  const int r = rank_below(peers);
  if (valid && r == 0) S.wcnt[wv][d] = (uint16_t)__popcll(peers);
  __syncthreads();
  uint32_t pos = 0;
  if (valid) {
    pos = S.run[d] + (uint32_t)r;
    for (int w = 0; w < wv; ++w) pos += S.wcnt[w][d];
  }
  __syncthreads();
  {
    const int t = threadIdx.x;
    S.run[t] += (uint32_t)S.wcnt[0][t] + S.wcnt[1][t] + S.wcnt[2][t] + S.wcnt[3][t];
    S.wcnt[0][t] = S.wcnt[1][t] = S.wcnt[2][t] = S.wcnt[3][t] = 0;
  }
  __syncthreads();
  return pos;
}

SHCI_DEV uint32_t block_scan256(uint32_t v, uint32_t* sh, uint32_t* tot) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int o = 1; o < 256; o <<= 1) {
    uint32_t x = (t >= o) ? sh[t - o] : 0u;
    __syncthreads();
    sh[t] += x;
    __syncthreads();
  }
  const uint32_t incl = sh[t];
  *tot = sh[255];
  __syncthreads();
  return incl - v;
}

// ---------------------------------------------------------------------------
// Partition pass kernels
// ---------------------------------------------------------------------------
struct PassArgs {
  Recs in, out;
  int64_t n;
  GroupPlan G;
  int nbits_n;  // orbitals (for the sample-id position)
  int auxbit;
  int shift, dbits;
  uint32_t* hist;        // [2^dbits][ntiles]
  const uint32_t* offs;  // exclusive scan of hist
  int ntiles;
};

// Tiles are dealt to blocks so that each of the 8 XCDs (blocks are
// dispatched round-robin over them) takes a contiguous range of tiles: the
// output runs of neighbouring tiles then meet in one XCD's L2.  The grid has
// 8 * ceil(ntiles / 8) blocks; blocks past the last tile return at once.
SHCI_DEV int xcd_tile(int b, int ntiles) {
  const int per = (ntiles + 7) / 8;
  return (b & 7) * per + (b >> 3);
}

template <int KW>
__global__ void __launch_bounds__(256) k_part_hist(PassArgs a) {
  __shared__ uint32_t cnt[256];
  const int tile = xcd_tile(blockIdx.x, a.ntiles);
  if (tile >= a.ntiles) return;
  cnt[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)tile * PTILE;
  const uint32_t dmask = (1u << a.dbits) - 1u;
#pragma unroll 4
  for (int j = 0; j < PTILE_ITEMS; ++j) {
    const int64_t idx = base + (int64_t)j * 256 + threadIdx.x;
    if (idx < a.n) atomicAdd(&cnt[(a.in.bid[idx] >> a.shift) & dmask], 1u);
  }
  __syncthreads();
  if (threadIdx.x < (1 << a.dbits)) a.hist[(int64_t)threadIdx.x * a.ntiles + tile] = cnt[threadIdx.x];
}

// One stable LSD pass over the bucket id, one tile of PTILE records per
// block.  Each wavefront ranks its own contiguous slice of the tile (ballot
// match per round, running per-digit counts in its LDS slice, no block
// barrier), which keeps the order stable; one scan then gives every digit its
// place in the tile.  Every array is staged through LDS in digit order and
// written out so that consecutive threads write consecutive records of one
// digit run (coalesced stores).
constexpr int PWAVES = 16;                      // wavefronts per partition block
constexpr int PTHREADS = 64 * PWAVES;
constexpr int PW_ITEMS = PTILE / PWAVES / 64;   // rounds per wavefront

// exclusive scan of 256 per-digit values held by threads [0, 256) of a block
// of PTHREADS threads (the others take part in the barriers only)
SHCI_DEV uint32_t digit_scan(uint32_t v, uint32_t* sh) {
  const int t = threadIdx.x;
  if (t < 256) sh[t] = v;
  __syncthreads();
  for (int o = 1; o < 256; o <<= 1) {
    uint32_t x = 0;
    if (t < 256 && t >= o) x = sh[t - o];
    __syncthreads();
    if (t < 256) sh[t] += x;
    __syncthreads();
  }
  const uint32_t incl = (t < 256) ? sh[t] : 0u;
  __syncthreads();
  return incl - v;
}

struct ScatterShared {
  uint16_t wc[PWAVES][256];  // per-wavefront count of each digit
  uint16_t wb[PWAVES][256];  // first local position of each (wavefront, digit)
  uint32_t lstart[256];      // first local position of each digit
  uint32_t gbase[256];       // first output position of each digit for this tile
  uint32_t scan[256];
  uint8_t sdig[PTILE];       // digit of each local position
  uint64_t stage[PTILE];
};

// record handled by (wavefront wv, lane, round j) within a tile
SHCI_DEV int tile_slot(int wv, int lane, int j) { return wv * (PTILE / PWAVES) + j * 64 + lane; }

// bit pattern of a 4- or 8-byte value in a 64-bit register, and back
template <typename T>
SHCI_DEV uint64_t to_bits(T v) {
  if constexpr (sizeof(T) == 8) {
    uint64_t u;
    __builtin_memcpy(&u, &v, 8);
    return u;
  } else {
    uint32_t u;
    __builtin_memcpy(&u, &v, 4);
    return u;
  }
}
template <typename T>
SHCI_DEV T from_bits(uint64_t u) {
  T v;
  if constexpr (sizeof(T) == 8) {
    __builtin_memcpy(&v, &u, 8);
  } else {
    const uint32_t w = (uint32_t)u;
    __builtin_memcpy(&v, &w, 4);
  }
  return v;
}

// One record array of a tile: values of this thread's records (held in
// 64-bit registers, 4-byte arrays zero-extended) are placed at their local
// positions in LDS, then written out as contiguous digit runs.
template <typename T>
SHCI_DEV void tile_load(const T* in, int64_t base, int tile_n, uint64_t (&r)[PW_ITEMS]) {
  const int t = threadIdx.x, wv = t >> 6, lane = t & 63;
  // every load is issued (slots past the tile re-read its first record), so
  // the loads of a thread are in flight together
#pragma unroll
  for (int j = 0; j < PW_ITEMS; ++j) {
    const int q = tile_slot(wv, lane, j);
    r[j] = to_bits<T>(in[base + (q < tile_n ? q : 0)]);
  }
}

// (S: any shared layout with stage, sdig, lstart and gbase as ScatterShared)
template <typename T, typename S>
SHCI_DEV void tile_scatter(S& L, const uint64_t (&r)[PW_ITEMS], T* out, int tile_n,
                           const uint16_t (&lpos)[PW_ITEMS]) {
  const int t = threadIdx.x, wv = t >> 6, lane = t & 63;
  T* st = reinterpret_cast<T*>(L.stage);
#pragma unroll
  for (int j = 0; j < PW_ITEMS; ++j) {
    const int q = tile_slot(wv, lane, j);
    if (q < tile_n) st[lpos[j]] = from_bits<T>(r[j]);
  }
  __syncthreads();
  // all LDS reads first, then the stores (distinct registers, so the stores
  // issue back to back)
  T val[PW_ITEMS];
  int64_t dst[PW_ITEMS];
#pragma unroll
  for (int j = 0; j < PW_ITEMS; ++j) {
    const int q = j * PTHREADS + t;
    const int qq = q < tile_n ? q : 0;
    const uint32_t d = L.sdig[qq];
    dst[j] = (int64_t)L.gbase[d] + (qq - (int)L.lstart[d]);
    val[j] = st[qq];
  }
#pragma unroll
  for (int j = 0; j < PW_ITEMS; ++j)
    if (j * PTHREADS + t < tile_n) out[dst[j]] = val[j];
  __syncthreads();
}

// Local positions of this thread's records of a tile (digits d, stable
// order): each wavefront ranks its slice by ballot match with running
// per-digit counts in its LDS slice, one scan places the digits.  Fills
// L.sdig and L.lstart; L.wc must be zero on entry.  (S: any shared layout
// with wc, wb, lstart, scan and sdig as ScatterShared)
template <typename S>
SHCI_DEV void tile_rank(S& L, const uint32_t (&dg)[PW_ITEMS], int tile_n, int dbits, uint16_t (&lpos)[PW_ITEMS]) {
  const int t = threadIdx.x, wv = t >> 6, lane = t & 63;
  uint8_t dig[PW_ITEMS];
  uint16_t* wc = L.wc[wv];
#pragma unroll
  for (int j = 0; j < PW_ITEMS; ++j) {
    const int q = tile_slot(wv, lane, j);
    const bool valid = q < tile_n;
    const uint32_t d = valid ? dg[j] : 0u;
    uint64_t peers = ballot(valid);
    for (int bb = 0; bb < dbits; ++bb) {
      const bool on = (d >> bb) & 1u;
      const uint64_t m = ballot(on);
      peers &= on ? m : ~m;
    }
    const int r = rank_below(peers);
    const uint32_t prior = valid ? wc[d] : 0u;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (valid && r == 0) wc[d] = (uint16_t)(prior + __popcll(peers));
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    lpos[j] = (uint16_t)(prior + r);  // rank within digit d among this wavefront's records
    dig[j] = (uint8_t)d;
  }
  __syncthreads();
  uint32_t cnt_t = 0;
  if (t < 256) {
#pragma unroll
    for (int w = 0; w < PWAVES; ++w) cnt_t += L.wc[w][t];
  }
  const uint32_t ls = digit_scan(cnt_t, L.scan);
  if (t < 256) {
    L.lstart[t] = ls;
    uint32_t acc = ls;
#pragma unroll
    for (int w = 0; w < PWAVES; ++w) {
      L.wb[w][t] = (uint16_t)acc;
      acc += L.wc[w][t];
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < PW_ITEMS; ++j) {
    const int q = tile_slot(wv, lane, j);
    lpos[j] = (uint16_t)(lpos[j] + L.wb[wv][dig[j]]);
    if (q < tile_n) L.sdig[lpos[j]] = dig[j];
  }
  __syncthreads();
}

template <int KW, typename VT, bool V2, bool PAY>
__global__ void __launch_bounds__(PTHREADS) k_part_scatter(PassArgs a) {
  __shared__ ScatterShared L;
  const int tile = xcd_tile(blockIdx.x, a.ntiles);
  if (tile >= a.ntiles) return;
  const int t = threadIdx.x;
  if (t < 256) {
#pragma unroll
    for (int w = 0; w < PWAVES; ++w) L.wc[w][t] = 0;
    L.gbase[t] = (t < (1 << a.dbits)) ? a.offs[(int64_t)t * a.ntiles + tile] : 0u;
  }
  __syncthreads();
  const int64_t base = (int64_t)tile * PTILE;
  const int tile_n = (int)((a.n - base < (int64_t)PTILE) ? (a.n - base) : (int64_t)PTILE);
  const uint32_t dmask = (1u << a.dbits) - 1u;
  uint16_t lpos[PW_ITEMS];
  // bucket ids of this thread's records, then (in flight during the ranking)
  // the first key word
  uint64_t ids[PW_ITEMS], cur[PW_ITEMS], nxt[PW_ITEMS];
  tile_load<uint32_t>(a.in.bid, base, tile_n, ids);
  tile_load<uint64_t>(a.in.k[0], base, tile_n, cur);
  {
    uint32_t dg[PW_ITEMS];
#pragma unroll
    for (int j = 0; j < PW_ITEMS; ++j) dg[j] = ((uint32_t)ids[j] >> a.shift) & dmask;
    tile_rank(L, dg, tile_n, a.dbits, lpos);
  }
  // arrays in order: key words, v, [v2], H_aa, [payload], bucket id; the
  // next array's loads are issued before the current one is written
  constexpr int NA = KW + 3 + (V2 ? 1 : 0) + (PAY ? 1 : 0);
  auto load_arr = [&](int x, uint64_t (&r)[PW_ITEMS]) {
    if (x < KW) {
#pragma unroll
      for (int w = 0; w < KW; ++w)
        if (w == x) tile_load<uint64_t>(a.in.k[w], base, tile_n, r);
      return;
    }
    x -= KW;
    if (x == 0) return tile_load<VT>(static_cast<const VT*>(a.in.v), base, tile_n, r);
    if constexpr (V2) {
      if (x == 1) return tile_load<VT>(static_cast<const VT*>(a.in.v2), base, tile_n, r);
      x -= 1;
    }
    if (x == 1) return tile_load<double>(a.in.haa, base, tile_n, r);
    if constexpr (PAY) {
      if (x == 2) return tile_load<uint32_t>(a.in.pay, base, tile_n, r);
      x -= 1;
    }
    tile_load<uint32_t>(a.in.bid, base, tile_n, r);
  };
  auto store_arr = [&](int x, const uint64_t (&r)[PW_ITEMS]) {
    if (x < KW) {
#pragma unroll
      for (int w = 0; w < KW; ++w)
        if (w == x) tile_scatter<uint64_t>(L, r, a.out.k[w], tile_n, lpos);
      return;
    }
    x -= KW;
    if (x == 0) return tile_scatter<VT>(L, r, static_cast<VT*>(a.out.v), tile_n, lpos);
    if constexpr (V2) {
      if (x == 1) return tile_scatter<VT>(L, r, static_cast<VT*>(a.out.v2), tile_n, lpos);
      x -= 1;
    }
    if (x == 1) return tile_scatter<double>(L, r, a.out.haa, tile_n, lpos);
    if constexpr (PAY) {
      if (x == 2) return tile_scatter<uint32_t>(L, r, a.out.pay, tile_n, lpos);
      x -= 1;
    }
    tile_scatter<uint32_t>(L, r, a.out.bid, tile_n, lpos);
  };
#pragma unroll
  for (int x = 0; x < NA; ++x) {
    if (x + 1 < NA) load_arr(x + 1, nxt);
    store_arr(x, cur);
#pragma unroll
    for (int j = 0; j < PW_ITEMS; ++j) cur[j] = nxt[j];
  }
}

// ---------------------------------------------------------------------------
// Bucket reduce
// ---------------------------------------------------------------------------
struct RedArgs {
  Recs in;
  int64_t nrec;
  GroupPlan G;
  int n, auxbit;
  double e0, nd;
  VSet V;
  Partials P;
  Uniq U;
  uint32_t* overflow;
  int want_u;
  const uint64_t* bstart;   // [nbucket + 1] bucket start offsets (nullable: binary search)
  const uint32_t* blist;    // buckets to process (nullable: all)
  const uint32_t* nlist;    // device count of blist
  double* contrib;          // keep-mode adjoint (nullable): contrib[pay] = t * 2 A_a / D_a (0 for a in V)
};

template <int KW>
__global__ void k_vset_insert(VSet V, int64_t nd, int n, uint32_t* flag) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= nd) return;
  uint64_t k[KW];
  pack_det<KW>(k, V.dets[4 * i], V.dets[4 * i + 1], V.dets[4 * i + 2], V.dets[4 * i + 3], n);
  const uint64_t h = det_hash<KW>(k, n);
  const uint32_t fp = (uint32_t)(h >> 32);
  const uint64_t entry = ((uint64_t)fp << 32) | (uint64_t)i;
  atomicOr((unsigned long long*)&V.filt[h >> (64 - V.fbits)], (unsigned long long)vfilt_bits(h));
  uint64_t slot = h & V.mask;
  for (uint64_t probe = 0; probe <= V.mask; ++probe) {
    const unsigned long long old =
        atomicCAS((unsigned long long*)&V.tab[slot], ~0ull, (unsigned long long)entry);
    if (old == ~0ull) return;
    if ((uint32_t)(old >> 32) == fp) {
      const uint64_t j = old & 0xffffffffull;
      bool eq = true;
      for (int w = 0; w < 4; ++w) eq = eq && (V.dets[4 * j + w] == V.dets[4 * i + w]);
      if (eq) {
        atomicOr(flag, 4u);
        return;
      }
    }
    slot = (slot + 1) & V.mask;
  }
  atomicOr(flag, 8u);  // table full (cannot happen at load <= 1/2)
}

// exclusive scan of 256 values held one per thread; returns the prefix,
// total in *tot (all threads)

template <int C>
struct SortBufs {
  uint32_t h2a[C], h2b[C];
  uint16_t ia[C], ib[C];
};

// one stable 8-bit LSD pass over M items: (sh, si) -> (dh, di)
template <int C, class DigitF>
SHCI_DEV void lds_pass(int M, const uint32_t* sh, const uint16_t* si, uint32_t* dh, uint16_t* di,
                       SplitScratch& S, uint32_t* scan_sh, DigitF digit) {
  const int t = threadIdx.x;
  S.run[t] = 0;
  __syncthreads();
  for (int j = t; j < M; j += 256) atomicAdd(&S.run[digit(j)], 1u);
  __syncthreads();
  uint32_t tot;
  const uint32_t start = block_scan256(S.run[t], scan_sh, &tot);
  __syncthreads();
  S.run[t] = start;
  __syncthreads();
  for (int j0 = 0; j0 < M; j0 += 256) {
    const int j = j0 + t;
    const bool valid = j < M;
    const uint32_t d = valid ? digit(j) : 0u;
    const uint32_t pos = split_round(S, valid, d, 8);
    if (valid) {
      dh[pos] = sh[j];
      di[pos] = si[j];
    }
  }
  __syncthreads();
}

template <int KW, int C, bool SAMPLE, typename VT>
struct RedShared {
  uint64_t key[KW][C];
  VT v[C];
  VT v2[SAMPLE ? C : 1];
  SortBufs<C> sb;
  uint16_t seg[C + 1];
  SplitScratch S;
  uint32_t scan[256];
  double red[256];
  double red2[256];
  double red3[256];
  int64_t ired[256];
  int64_t ired2[256];
  int32_t ired3[256];
  int32_t ired4[256];
  int32_t ired5[256];
  double dmin[256];
  uint64_t lohi[2];
  uint32_t flag;
  uint32_t nseg;
};

template <int KW, int C, bool SAMPLE, typename VT>
__global__ void __launch_bounds__(256) k_reduce(RedArgs a) {
  __shared__ RedShared<KW, C, SAMPLE, VT> R;
  if (a.blist && (int64_t)*a.nlist <= (int64_t)blockIdx.x) return;
  const int t = threadIdx.x;
  const int n = a.n;
  R.S.wcnt[0][t] = R.S.wcnt[1][t] = R.S.wcnt[2][t] = R.S.wcnt[3][t] = 0;
  __syncthreads();

  const int64_t nb = a.blist ? (int64_t)*a.nlist : a.G.nbucket;
  for (int64_t bi = blockIdx.x; bi < nb; bi += gridDim.x) {
    const int64_t b = a.blist ? (int64_t)a.blist[bi] : bi;
    if (a.bstart) {
      if (t < 2) {
        int64_t v = (int64_t)a.bstart[b + t];
        R.lohi[t] = (uint64_t)(v < 0 ? 0 : (v > a.nrec ? a.nrec : v));
      }
    } else if (t < 2) {
      // bucket bounds by binary search on the (sorted) bucket ids
      const uint64_t target = (uint64_t)b + (uint64_t)t;
      int64_t lo = 0, hi = a.nrec;
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        uint64_t k[KW];
        load_key<KW>(a.in, mid, k);
        clear_aux<KW>(k, a.auxbit);
        uint64_t h;
        if (bucket_id<KW>(k, a.G, n, h) < target)
          lo = mid + 1;
        else
          hi = mid;
      }
      R.lohi[t] = (uint64_t)lo;
    }
    if (t == 0) R.flag = 0;
    __syncthreads();
    const int64_t lo = (int64_t)R.lohi[0];
    const int64_t hi_ = (int64_t)R.lohi[1];
    const int M = (int)(hi_ > lo ? hi_ - lo : 0);
    if (M > C) {
      if (t == 0) {
        atomicOr(a.overflow, 1u);
        a.P.e2[b] = 0.0;
        a.P.de0[b] = 0.0;
        a.P.e2sq[b] = 0.0;
        a.P.nterm[b] = 0;
        a.P.ngen[b] = 0;
        a.P.nuniq[b] = 0;
        a.P.nintr[b] = 0;
        a.P.nzero[b] = 0;
        a.P.mind[b] = INFINITY;
        a.P.nseg[b] = 0;
        if (a.want_u) a.U.start[b] = (uint64_t)lo;
      }
      __syncthreads();
      continue;
    }
    // load records
    for (int j = t; j < M; j += 256) {
      uint64_t k[KW];
      load_key<KW>(a.in, lo + j, k);
#pragma unroll
      for (int w = 0; w < KW; ++w) R.key[w][j] = k[w];
      R.v[j] = static_cast<const VT*>(a.in.v)[lo + j];
      if constexpr (SAMPLE) R.v2[j] = static_cast<const VT*>(a.in.v2)[lo + j];
      clear_aux<KW>(k, a.auxbit);
      R.sb.h2a[j] = sort_hash(det_hash<KW>(k, a.n), a.G);
      R.sb.ia[j] = (uint16_t)j;
    }
    __syncthreads();
    // LSD sort on the 32-bit in-bucket hash
    for (int pass = 0; pass < 4; ++pass) {
      const int sh = pass * 8;
      if ((pass & 1) == 0)
        lds_pass<C>(M, R.sb.h2a, R.sb.ia, R.sb.h2b, R.sb.ib, R.S, R.scan,
                    [&](int j) { return (R.sb.h2a[j] >> sh) & 0xffu; });
      else
        lds_pass<C>(M, R.sb.h2b, R.sb.ib, R.sb.h2a, R.sb.ia, R.S, R.scan,
                    [&](int j) { return (R.sb.h2b[j] >> sh) & 0xffu; });
    }
    auto key_eq = [&](int x, int y) {
      bool eq = true;
#pragma unroll
      for (int w = 0; w < KW; ++w) {
        uint64_t kx = R.key[w][x], ky = R.key[w][y];
        if (w == (a.auxbit >> 6)) {
          kx &= ~(1ull << (a.auxbit & 63));
          ky &= ~(1ull << (a.auxbit & 63));
        }
        eq = eq && (kx == ky);
      }
      return eq;
    };
    // different keys sharing the 32 hash bits: sort by the full key first
    for (int j = t + 1; j < M; j += 256)
      if (R.sb.h2a[j] == R.sb.h2a[j - 1] && !key_eq(R.sb.ia[j], R.sb.ia[j - 1])) R.flag = 1;
    __syncthreads();
    if (R.flag) {
      // restart from load order: h2a/ia were permuted; rebuild identity order
      for (int j = t; j < M; j += 256) {
        uint64_t k[KW];
#pragma unroll
        for (int w = 0; w < KW; ++w) k[w] = R.key[w][j];
        clear_aux<KW>(k, a.auxbit);
        R.sb.h2a[j] = sort_hash(det_hash<KW>(k, a.n), a.G);
        R.sb.ia[j] = (uint16_t)j;
      }
      __syncthreads();
      const int keybits = a.auxbit;  // all grouping bits lie below the aux bit
      const int kpasses = (keybits + 7) / 8;
      bool in_a = true;
      for (int pass = 0; pass < kpasses + 4; ++pass) {
        auto digit_key = [&](int j) -> uint32_t {
          const int idx = in_a ? R.sb.ia[j] : R.sb.ib[j];
          const int bit = pass * 8;
          const int w = bit >> 6, o = bit & 63;
          uint64_t x = 0;
#pragma unroll
          for (int q = 0; q < KW; ++q)
            if (q == w) x = R.key[q][idx];
          uint32_t dgt = (uint32_t)(x >> o) & 0xffu;
          // stay below the aux bit
          const int hi = keybits - bit;
          if (hi < 8) dgt &= (1u << hi) - 1u;
          return dgt;
        };
        auto digit_h2 = [&](int j) -> uint32_t {
          const uint32_t hv = in_a ? R.sb.h2a[j] : R.sb.h2b[j];
          return (hv >> ((pass - kpasses) * 8)) & 0xffu;
        };
        if (pass < kpasses) {
          if (in_a)
            lds_pass<C>(M, R.sb.h2a, R.sb.ia, R.sb.h2b, R.sb.ib, R.S, R.scan, digit_key);
          else
            lds_pass<C>(M, R.sb.h2b, R.sb.ib, R.sb.h2a, R.sb.ia, R.S, R.scan, digit_key);
        } else {
          if (in_a)
            lds_pass<C>(M, R.sb.h2a, R.sb.ia, R.sb.h2b, R.sb.ib, R.S, R.scan, digit_h2);
          else
            lds_pass<C>(M, R.sb.h2b, R.sb.ib, R.sb.h2a, R.sb.ia, R.S, R.scan, digit_h2);
        }
        in_a = !in_a;
      }
      if (!in_a) {
        for (int j = t; j < M; j += 256) {
          R.sb.h2a[j] = R.sb.h2b[j];
          R.sb.ia[j] = R.sb.ib[j];
        }
        __syncthreads();
      }
    }
    // segment heads in sorted order -> segment starts
    const int per = (M + 255) / 256;
    const int j_lo = t * per, j_hi = min(M, j_lo + per);
    uint32_t cnt = 0;
    for (int j = j_lo; j < j_hi; ++j) cnt += (j == 0) || !key_eq(R.sb.ia[j], R.sb.ia[j - 1]);
    uint32_t nsg;
    uint32_t sidx = block_scan256(cnt, R.scan, &nsg);
    for (int j = j_lo; j < j_hi; ++j)
      if ((j == 0) || !key_eq(R.sb.ia[j], R.sb.ia[j - 1])) R.seg[sidx++] = (uint16_t)j;
    if (t == 0) R.seg[nsg] = (uint16_t)M;
    __syncthreads();

    double e2p = 0.0, de0p = 0.0, e2sq = 0.0, dmn = INFINITY;
    int64_t nterm = 0, ngen = 0;
    int32_t nuniq = 0, nintr = 0, nzero = 0;
    for (uint32_t s = t; s < nsg; s += 256) {
      const int j0 = R.seg[s], j1 = R.seg[s + 1];
      const int first = R.sb.ia[j0];
      SegSum<VT> sum;
      for (int j = j0; j < j1; ++j) {
        const int id = R.sb.ia[j];
        const bool dflag = (R.key[a.auxbit >> 6][id] >> (a.auxbit & 63)) & 1ull;
        if constexpr (SAMPLE)
          sum.add_sample(R.v[id], R.v2[id], dflag);
        else
          sum.add(R.v[id], dflag);
      }
      sum.finish();
      const double X = sum.X;
      uint64_t k[KW];
#pragma unroll
      for (int w = 0; w < KW; ++w) k[w] = R.key[w][first];
      clear_aux<KW>(k, a.auxbit);
      uint64_t a0, a1, b0, b1;
      unpack_det<KW>(k, n, a0, a1, b0, b1);
      uint64_t dk[KW];
      pack_det<KW>(dk, a0, a1, b0, b1, n);  // det bits only (no sample id)
      const bool inv = vset_contains<KW>(a.V, dk, n);
      const int cntk = j1 - j0;
      ngen += cntk;
      double Dd = 0.0, g = 0.0, gd = 0.0, gG = 0.0;
      if (!inv) {
        const double haa = a.in.haa[lo + first];
        Dd = a.e0 - haa;
        double contrib;
        if constexpr (SAMPLE) {
          const double G = 1.0 / (Dd * a.nd * (a.nd - 1.0));
          contrib = sum.sample_bracket() * G;
          de0p += -contrib / Dd;
          g = 2.0 * X * G;
          gd = 2.0 * sum.Xd * G;
          gG = G;
        } else {
          const double a2 = X * X - sum.Xd * sum.Xd;  // see k_reduce_wave
          contrib = a2 / Dd;
          de0p += -a2 / (Dd * Dd);
          g = 2.0 * X / Dd;
        }
        e2p += contrib;
        e2sq += contrib * contrib;
        nterm += cntk;
        nuniq += 1;
        nintr += Dd > 0.0;
        nzero += Dd == 0.0;
        dmn = fmin(dmn, fabs(Dd));
      }
      if constexpr (!SAMPLE) {
        if (a.contrib) {
          for (int j = j0; j < j1; ++j) {
            const int id = R.sb.ia[j];
            a.contrib[a.in.pay[lo + id]] = inv ? 0.0 : (double)R.v[id] * g;
          }
        }
      }
      if (a.want_u) {
        const int64_t o = lo + s;
#pragma unroll
        for (int w = 0; w < KW; ++w) a.U.k[w][o] = k[w];
        a.U.h2[o] = R.sb.h2a[j0];
        // deterministic: A_a, D_a, 2 A_a / D_a; sample: 2 X^d G, G, 2 X G with
        // G = 1 / (D_a Nd (Nd - 1)) (the adjoint's per-a factors)
        a.U.A[o] = SAMPLE ? gd : X;
        a.U.D[o] = SAMPLE ? gG : Dd;
        a.U.g[o] = g;
        a.U.cnt[o] = inv ? -cntk : cntk;
      }
    }
    // fixed-shape block reductions
    R.red[t] = e2p;
    R.red2[t] = de0p;
    R.red3[t] = e2sq;
    R.ired[t] = nterm;
    R.ired2[t] = ngen;
    R.ired3[t] = nuniq;
    R.ired4[t] = nintr;
    R.ired5[t] = nzero;
    R.dmin[t] = dmn;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (t < o) {
        R.red[t] += R.red[t + o];
        R.red2[t] += R.red2[t + o];
        R.red3[t] += R.red3[t + o];
        R.ired[t] += R.ired[t + o];
        R.ired2[t] += R.ired2[t + o];
        R.ired3[t] += R.ired3[t + o];
        R.ired4[t] += R.ired4[t + o];
        R.ired5[t] += R.ired5[t + o];
        R.dmin[t] = fmin(R.dmin[t], R.dmin[t + o]);
      }
      __syncthreads();
    }
    if (t == 0) {
      a.P.e2[b] = R.red[0];
      a.P.de0[b] = R.red2[0];
      a.P.e2sq[b] = R.red3[0];
      a.P.nterm[b] = R.ired[0];
      a.P.ngen[b] = R.ired2[0];
      a.P.nuniq[b] = R.ired3[0];
      a.P.nintr[b] = R.ired4[0];
      a.P.nzero[b] = R.ired5[0];
      a.P.mind[b] = R.dmin[0];
      a.P.nseg[b] = (int32_t)nsg;
      if (a.want_u) a.U.start[b] = (uint64_t)lo;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Final reductions (one block; fixed order)
// ---------------------------------------------------------------------------
// first level of the final reduction: block b sums buckets [b*chunk, ...)
// into slot b of Q (same layout as Partials); fixed order
__global__ void __launch_bounds__(256) k_final_partial(Partials P, int64_t nb, int64_t chunk, Partials Q) {
  __shared__ double r1[256], r2[256], r3[256], r4[256];
  __shared__ int64_t i1[256], i2[256], i3[256], i4[256], i5[256];
  const int t = threadIdx.x;
  const int64_t lo = (int64_t)blockIdx.x * chunk, hi = min(nb, lo + chunk);
  double e = 0.0, d = 0.0, q = 0.0, mn = INFINITY;
  int64_t nt = 0, ng = 0, nu = 0, ni = 0, nz = 0;
  for (int64_t b = lo + t; b < hi; b += 256) {
    e += P.e2[b];
    d += P.de0[b];
    q += P.e2sq[b];
    mn = fmin(mn, P.mind[b]);
    nt += P.nterm[b];
    ng += P.ngen[b];
    nu += P.nuniq[b];
    ni += P.nintr[b];
    nz += P.nzero[b];
  }
  r1[t] = e; r2[t] = d; r3[t] = mn; r4[t] = q;
  i1[t] = nt; i2[t] = ng; i3[t] = nu; i4[t] = ni; i5[t] = nz;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) {
      r1[t] += r1[t + o];
      r2[t] += r2[t + o];
      r4[t] += r4[t + o];
      r3[t] = fmin(r3[t], r3[t + o]);
      i1[t] += i1[t + o];
      i2[t] += i2[t + o];
      i3[t] += i3[t + o];
      i4[t] += i4[t + o];
      i5[t] += i5[t + o];
    }
    __syncthreads();
  }
  if (t == 0) {
    const int b = blockIdx.x;
    Q.e2[b] = r1[0];
    Q.de0[b] = r2[0];
    Q.e2sq[b] = r4[0];
    Q.mind[b] = r3[0];
    Q.nterm[b] = i1[0];
    Q.ngen[b] = i2[0];
    Q.nuniq[b] = (int32_t)i3[0];
    Q.nintr[b] = (int32_t)i4[0];
    Q.nzero[b] = (int32_t)i5[0];
  }
}

// first level of the final reduction over the block kernel's buckets only:
// block b sums the per-bucket partials of the buckets marked in `bits` among
// [b*chunk, (b+1)*chunk) into slot b of Q; thread t takes the bitmap words
// t, t + 256, ... of the range (fixed order)
__global__ void __launch_bounds__(256) k_final_partial_marked(Partials P, const uint32_t* bits, int64_t nb,
                                                              int64_t chunk, Partials Q) {
  __shared__ double r1[256], r2[256], r3[256], r4[256];
  __shared__ int64_t i1[256], i2[256], i3[256], i4[256], i5[256];
  const int t = threadIdx.x;
  const int64_t lo = (int64_t)blockIdx.x * chunk, hi = min(nb, lo + chunk);
  double e = 0.0, d = 0.0, q = 0.0, mn = INFINITY;
  int64_t nt = 0, ng = 0, nu = 0, ni = 0, nz = 0;
  for (int64_t wd = lo / 32 + t; wd * 32 < hi; wd += 256) {
    uint32_t m = bits[wd];
    while (m) {
      const int64_t b = wd * 32 + __ffs(m) - 1;
      m &= m - 1;
      if (b < lo || b >= hi) continue;
      e += P.e2[b];
      d += P.de0[b];
      q += P.e2sq[b];
      mn = fmin(mn, P.mind[b]);
      nt += P.nterm[b];
      ng += P.ngen[b];
      nu += P.nuniq[b];
      ni += P.nintr[b];
      nz += P.nzero[b];
    }
  }
  r1[t] = e; r2[t] = d; r3[t] = mn; r4[t] = q;
  i1[t] = nt; i2[t] = ng; i3[t] = nu; i4[t] = ni; i5[t] = nz;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) {
      r1[t] += r1[t + o];
      r2[t] += r2[t + o];
      r4[t] += r4[t + o];
      r3[t] = fmin(r3[t], r3[t + o]);
      i1[t] += i1[t + o];
      i2[t] += i2[t + o];
      i3[t] += i3[t + o];
      i4[t] += i4[t + o];
      i5[t] += i5[t + o];
    }
    __syncthreads();
  }
  if (t == 0) {
    const int b = blockIdx.x;
    Q.e2[b] = r1[0];
    Q.de0[b] = r2[0];
    Q.e2sq[b] = r4[0];
    Q.mind[b] = r3[0];
    Q.nterm[b] = i1[0];
    Q.ngen[b] = i2[0];
    Q.nuniq[b] = (int32_t)i3[0];
    Q.nintr[b] = (int32_t)i4[0];
    Q.nzero[b] = (int32_t)i5[0];
  }
}

struct DevResult {
  double e2, de0, mind, e2sq;
  int64_t nterm, ngen, nuniq, nintr, nzero;
  uint32_t overflow, flags;
};

__global__ void __launch_bounds__(1024) k_final(Partials P, int64_t nb, int64_t seg_lo, int64_t seg_n,
                                                const uint32_t* overflow, const uint32_t* flags,
                                                DevResult* res, double* per_sample, int64_t per_seg,
                                                double* per_sample_de0, double sample_scale) {
  // sums buckets [seg_lo + s*per_seg, ...) per segment s when per_sample != NULL,
  // or everything into res
  __shared__ double r1[1024], r2[1024], r3[1024], r4[1024];
  __shared__ int64_t i1[1024], i2[1024], i3[1024], i4[1024], i5[1024];
  const int t = threadIdx.x;
  const int64_t lo = per_sample ? seg_lo + (int64_t)blockIdx.x * per_seg : 0;
  const int64_t cnt = per_sample ? per_seg : nb;
  const int64_t chunk = (cnt + 1023) / 1024;
  const int64_t b0 = lo + t * chunk, b1 = min(lo + cnt, b0 + chunk);
  double e = 0.0, d = 0.0, q = 0.0, mn = INFINITY;
  int64_t nt = 0, ng = 0, nu = 0, ni = 0, nz = 0;
  for (int64_t b = b0; b < b1; ++b) {
    e += P.e2[b];
    d += P.de0[b];
    q += P.e2sq[b];
    mn = fmin(mn, P.mind[b]);
    nt += P.nterm[b];
    ng += P.ngen[b];
    nu += P.nuniq[b];
    ni += P.nintr[b];
    nz += P.nzero[b];
  }
  r1[t] = e; r2[t] = d; r3[t] = mn; r4[t] = q;
  i1[t] = nt; i2[t] = ng; i3[t] = nu; i4[t] = ni; i5[t] = nz;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if (t < o) {
      r1[t] += r1[t + o];
      r2[t] += r2[t + o];
      r4[t] += r4[t + o];
      r3[t] = fmin(r3[t], r3[t + o]);
      i1[t] += i1[t + o];
      i2[t] += i2[t + o];
      i3[t] += i3[t + o];
      i4[t] += i4[t + o];
      i5[t] += i5[t + o];
    }
    __syncthreads();
  }
  if (t == 0) {
    if (per_sample) {
      per_sample[blockIdx.x] = sample_scale * r1[0];
      if (per_sample_de0) per_sample_de0[blockIdx.x] = sample_scale * r2[0];
      // statistics accumulate over the per-sample blocks
      atomicAdd((unsigned long long*)&res->nterm, (unsigned long long)i1[0]);
      atomicAdd((unsigned long long*)&res->ngen, (unsigned long long)i2[0]);
      atomicAdd((unsigned long long*)&res->nuniq, (unsigned long long)i3[0]);
      atomicAdd((unsigned long long*)&res->nintr, (unsigned long long)i4[0]);
      atomicAdd((unsigned long long*)&res->nzero, (unsigned long long)i5[0]);
      // |D| >= 0: the bit patterns of non-negative doubles order like the values
      atomicMin((unsigned long long*)&res->mind, (unsigned long long)__double_as_longlong(r3[0]));
    } else {
      res->e2 = r1[0];
      res->de0 = r2[0];
      res->e2sq = r4[0];
      res->mind = r3[0];
      res->nterm = i1[0];
      res->ngen = i2[0];
      res->nuniq = i3[0];
      res->nintr = i4[0];
      res->nzero = i5[0];
      res->overflow = *overflow;
      res->flags = *flags;
    }
  }
}

// Sample mode, first level: block b = s * G + g sums slice g (of G) of
// sample s's per-wavefront slots Pw[s][0..nwaves), of the block kernel's
// buckets of s (marked in `bits`, buckets [s << bits_hash, (s + 1) <<
// bits_hash)) and, with the singleton split, of the in-place partials PI of
// its work items [ib[s], ib[s + 1]), into slot b of Q; fixed ranges per
// thread, then a fixed tree.
template <class F>
SHCI_DEV void slice_of(int64_t n, int g, int G, F&& f) {
  const int64_t lo = n * g / G, hi = n * (g + 1) / G;
  const int64_t per = (hi - lo + 255) / 256;
  const int64_t b0 = lo + (int64_t)threadIdx.x * per, b1 = min(hi, b0 + per);
  for (int64_t i = b0; i < b1; ++i) f(i);
}

__global__ void __launch_bounds__(256) k_final_sample_part(Partials Pw, int64_t nwaves, Partials P, const uint32_t* bits,
                                                           int bits_hash, Partials PI, const uint64_t* ib, int G,
                                                           Partials Q) {
  __shared__ double r1[256], r2[256], r3[256];
  __shared__ int64_t i1[256], i2[256], i3[256], i4[256], i5[256];
  const int t = threadIdx.x;
  const int64_t s = blockIdx.x / G;
  const int g = (int)(blockIdx.x % G);
  double e = 0.0, d = 0.0, mn = INFINITY;
  int64_t nt = 0, ng = 0, nu = 0, ni = 0, nz = 0;
  auto add = [&](const Partials& X, int64_t i) {
    e += X.e2[i];
    d += X.de0[i];
    mn = fmin(mn, X.mind[i]);
    nt += X.nterm[i];
    ng += X.ngen[i];
    nu += X.nuniq[i];
    ni += X.nintr[i];
    nz += X.nzero[i];
  };
  slice_of(nwaves, g, G, [&](int64_t w) { add(Pw, s * nwaves + w); });
  const int64_t b0 = s << bits_hash, nbk = (int64_t)1 << bits_hash;
  if (nbk >= 32) {
    slice_of(nbk / 32, g, G, [&](int64_t wd) {
      uint32_t m = bits[b0 / 32 + wd];
      while (m) {
        add(P, (b0 / 32 + wd) * 32 + __ffs(m) - 1);
        m &= m - 1;
      }
    });
  } else if (g == 0 && t == 0) {
    for (int64_t b = b0; b < b0 + nbk; ++b)
      if ((bits[b >> 5] >> (b & 31)) & 1u) add(P, b);
  }
  if (ib) {
    const int64_t lo = (int64_t)ib[s];
    slice_of((int64_t)ib[s + 1] - lo, g, G, [&](int64_t i) { add(PI, lo + i); });
  }
  r1[t] = e; r2[t] = d; r3[t] = mn;
  i1[t] = nt; i2[t] = ng; i3[t] = nu; i4[t] = ni; i5[t] = nz;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) {
      r1[t] += r1[t + o];
      r2[t] += r2[t + o];
      r3[t] = fmin(r3[t], r3[t + o]);
      i1[t] += i1[t + o];
      i2[t] += i2[t + o];
      i3[t] += i3[t + o];
      i4[t] += i4[t + o];
      i5[t] += i5[t + o];
    }
    __syncthreads();
  }
  if (t == 0) {
    const int64_t b = blockIdx.x;
    Q.e2[b] = r1[0];
    Q.de0[b] = r2[0];
    Q.mind[b] = r3[0];
    Q.nterm[b] = i1[0];
    Q.ngen[b] = i2[0];
    Q.nuniq[b] = (int32_t)i3[0];
    Q.nintr[b] = (int32_t)i4[0];
    Q.nzero[b] = (int32_t)i5[0];
  }
}

// second level, one thread per sample: its G slots in order
__global__ void k_final_sample_sum(Partials Q, int G, int32_t nsamp, DevResult* res, double* per_sample,
                                   double* per_sample_de0, double sample_scale) {
  const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= nsamp) return;
  double e = 0.0, d = 0.0, mn = INFINITY;
  int64_t nt = 0, ng = 0, nu = 0, ni = 0, nz = 0;
  for (int g = 0; g < G; ++g) {
    const int64_t b = s * G + g;
    e += Q.e2[b];
    d += Q.de0[b];
    mn = fmin(mn, Q.mind[b]);
    nt += Q.nterm[b];
    ng += Q.ngen[b];
    nu += Q.nuniq[b];
    ni += Q.nintr[b];
    nz += Q.nzero[b];
  }
  per_sample[s] = sample_scale * e;
  if (per_sample_de0) per_sample_de0[s] = sample_scale * d;
  atomicAdd((unsigned long long*)&res->nterm, (unsigned long long)nt);
  atomicAdd((unsigned long long*)&res->ngen, (unsigned long long)ng);
  atomicAdd((unsigned long long*)&res->nuniq, (unsigned long long)nu);
  atomicAdd((unsigned long long*)&res->nintr, (unsigned long long)ni);
  atomicAdd((unsigned long long*)&res->nzero, (unsigned long long)nz);
  // |D| >= 0: the bit patterns of non-negative doubles order like the values
  atomicMin((unsigned long long*)&res->mind, (unsigned long long)__double_as_longlong(mn));
}

}  // namespace shci
