// Singleton split of the screened terms.
//
// Almost every perturbative determinant a is reached by one term only (at
// the small thresholds of the stochastic part, all but a fraction of a
// percent), and a group of one term needs no grouping: its contribution is
// the term's own.  So before any record is written:
//  1. the count walk lists the 64-bit grouping hash (determinant hash with the
//     sample id mixed in) and the work item of every kept term, 12 bytes a
//     term instead of a record of 44-60;
//  2. the list is partitioned on the top hash bits (LSD passes: the first
//     needs no stability, the later ones rank as the records' passes do),
//     buckets of ~12k hashes (two passes up to ~8e8);
//  3. per bucket, one workgroup finds the 32-bit tags that occur more than
//     once (an LDS hash table) and sets their hashes in a presence filter;
//  4. every listed term whose hash passes the filter is counted for its work
//     item; the scan of these counts places the records.
// The write walk then writes records only for terms whose hash passes the
// filter (every term of an a with several terms does, and a few others:
// shared tags, filter collisions) and sums the contribution of every other
// term in place.  The decision depends on the hash alone, so all terms of one
// a take the same side and the records of an a are complete; the split
// changes the order of the final sums only.
#pragma once
#include "group.hpp"

namespace shci {

struct HPassArgs {
  const uint64_t* kin;
  const uint32_t* iin;
  uint64_t* kout;
  uint32_t* iout;
  int64_t n;
  int nbits;       // bucket id = top nbits of the hash (nbits >= 1)
  int shift, dbits;
  uint32_t* hist;  // [2^dbits][ntiles]
  const uint32_t* offs;
  int ntiles;
};

SHCI_DEV uint32_t hdigit(uint64_t g, const HPassArgs& a) {
  return ((uint32_t)(g >> (64 - a.nbits)) >> a.shift) & ((1u << a.dbits) - 1u);
}

__global__ void __launch_bounds__(256) k_hpart_hist(HPassArgs a) {
  __shared__ uint32_t cnt[256];
  const int tile = xcd_tile(blockIdx.x, a.ntiles);
  if (tile >= a.ntiles) return;
  cnt[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)tile * PTILE;
#pragma unroll 4
  for (int j = 0; j < PTILE_ITEMS; ++j) {
    const int64_t idx = base + (int64_t)j * 256 + threadIdx.x;
    if (idx < a.n) atomicAdd(&cnt[hdigit(a.kin[idx], a)], 1u);
  }
  __syncthreads();
  if (threadIdx.x < (1 << a.dbits)) a.hist[(int64_t)threadIdx.x * a.ntiles + tile] = cnt[threadIdx.x];
}

// One stable LSD pass over (hash, work item) pairs (every pass after the
// first must keep the order of the one before): the ranking of
// k_part_scatter, with a 4-byte stage through which the hashes go in two
// halves, so that the shared layout (59 KB) lets two blocks share a compute
// unit.
struct HStableShared {
  uint16_t wc[PWAVES][256];
  uint16_t wb[PWAVES][256];
  uint32_t lstart[256];
  uint32_t gbase[256];
  uint32_t scan[256];
  uint8_t sdig[PTILE];
  uint32_t stage[PTILE];
};

// tile_scatter for 8-byte values through a 4-byte stage: low halves, then
// high halves, each placed and read back in digit order
template <typename S>
SHCI_DEV void tile_scatter_halves(S& L, const uint64_t (&r)[PW_ITEMS], uint64_t* out, int tile_n,
                                  const uint16_t (&lpos)[PW_ITEMS]) {
  const int t = threadIdx.x, wv = t >> 6, lane = t & 63;
  uint32_t lo[PW_ITEMS];
  int64_t dst[PW_ITEMS];
#pragma unroll
  for (int j = 0; j < PW_ITEMS; ++j)
    if (tile_slot(wv, lane, j) < tile_n) L.stage[lpos[j]] = (uint32_t)r[j];
  __syncthreads();
#pragma unroll
  for (int j = 0; j < PW_ITEMS; ++j) {
    const int q = j * PTHREADS + t;
    const int qq = q < tile_n ? q : 0;
    const uint32_t d = L.sdig[qq];
    dst[j] = (int64_t)L.gbase[d] + (qq - (int)L.lstart[d]);
    lo[j] = L.stage[qq];
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < PW_ITEMS; ++j)
    if (tile_slot(wv, lane, j) < tile_n) L.stage[lpos[j]] = (uint32_t)(r[j] >> 32);
  __syncthreads();
  uint64_t val[PW_ITEMS];
#pragma unroll
  for (int j = 0; j < PW_ITEMS; ++j) {
    const int q = j * PTHREADS + t;
    const int qq = q < tile_n ? q : 0;
    val[j] = ((uint64_t)L.stage[qq] << 32) | lo[j];
  }
#pragma unroll
  for (int j = 0; j < PW_ITEMS; ++j)
    if (j * PTHREADS + t < tile_n) out[dst[j]] = val[j];
  __syncthreads();
}

__global__ void __launch_bounds__(PTHREADS) __attribute__((amdgpu_waves_per_eu(8, 8)))
k_hpart_scatter(HPassArgs a) {
  __shared__ HStableShared L;
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
  uint16_t lpos[PW_ITEMS];
  uint64_t keys[PW_ITEMS], items[PW_ITEMS];
  tile_load<uint64_t>(a.kin, base, tile_n, keys);
  tile_load<uint32_t>(a.iin, base, tile_n, items);
  {
    uint32_t dg[PW_ITEMS];
#pragma unroll
    for (int j = 0; j < PW_ITEMS; ++j) dg[j] = hdigit(keys[j], a);
    tile_rank(L, dg, tile_n, a.dbits, lpos);
  }
  tile_scatter_halves(L, keys, a.kout, tile_n, lpos);
  tile_scatter<uint32_t>(L, items, a.iout, tile_n, lpos);
}

// The first LSD pass over (hash, work item) pairs need not be stable: the
// list is in no particular order to begin with (only a later pass must keep
// the order of the one before, and a single pass only groups).  So each tile
// ranks its pairs by LDS atomics on 256 per-digit counters instead of ballot
// matching, and the smaller shared layout (76 KB) lets two blocks share a
// compute unit, one loading while the other writes.  The pairs of a digit run
// are still written contiguously (LDS staging), at the tile's offsets from
// the histogram pass.
struct HScatterShared {
  uint32_t cnt[256];     // per-digit counts of the tile, then ranks
  uint32_t lstart[256];  // first local position of each digit
  uint32_t gbase[256];   // first output position of each digit for this tile
  uint32_t scan[256];
  uint8_t sdig[PTILE];   // digit of each local position
  uint64_t stage[PTILE];
};

__global__ void __launch_bounds__(PTHREADS) __attribute__((amdgpu_waves_per_eu(8, 8)))
k_hpart_scatter_first(HPassArgs a) {
  __shared__ HScatterShared L;
  const int tile = xcd_tile(blockIdx.x, a.ntiles);
  if (tile >= a.ntiles) return;
  const int t = threadIdx.x, wv = t >> 6, lane = t & 63;
  if (t < 256) {
    L.cnt[t] = 0u;
    L.gbase[t] = (t < (1 << a.dbits)) ? a.offs[(int64_t)t * a.ntiles + tile] : 0u;
  }
  __syncthreads();
  const int64_t base = (int64_t)tile * PTILE;
  const int tile_n = (int)((a.n - base < (int64_t)PTILE) ? (a.n - base) : (int64_t)PTILE);
  uint64_t keys[PW_ITEMS], items[PW_ITEMS];
  tile_load<uint64_t>(a.kin, base, tile_n, keys);
  tile_load<uint32_t>(a.iin, base, tile_n, items);
  uint32_t dg[PW_ITEMS];
  uint16_t lpos[PW_ITEMS];
#pragma unroll
  for (int j = 0; j < PW_ITEMS; ++j) {
    dg[j] = hdigit(keys[j], a);
    lpos[j] = 0;
    if (tile_slot(wv, lane, j) < tile_n) lpos[j] = (uint16_t)atomicAdd(&L.cnt[dg[j]], 1u);
  }
  __syncthreads();
  const uint32_t ex = digit_scan(t < 256 ? L.cnt[t] : 0u, L.scan);
  if (t < 256) L.lstart[t] = ex;
  __syncthreads();
#pragma unroll
  for (int j = 0; j < PW_ITEMS; ++j) {
    if (tile_slot(wv, lane, j) < tile_n) {
      lpos[j] = (uint16_t)(lpos[j] + L.lstart[dg[j]]);
      L.sdig[lpos[j]] = (uint8_t)dg[j];
    }
  }
  __syncthreads();
  tile_scatter<uint64_t>(L, keys, a.kout, tile_n, lpos);
  tile_scatter<uint32_t>(L, items, a.iout, tile_n, lpos);
}

constexpr int HDUP_THREADS = 1024;
constexpr int HDUP_SLOTS = 36864;     // 32-bit tags in LDS (144 KB of gfx950's 160 KB per workgroup)
constexpr int HDUP_FILL = 18432;      // distinct tags a slice aims at when a bucket overflows (load 1/2)
constexpr int64_t HDUP_MEAN = 12500;  // bucket size the bucket bits aim at (load ~1/3)
constexpr int HDUP_PROBES = 1024;     // longest probe run before the table counts as full
constexpr int HDUP_PER_THREAD = 16;   // hashes a thread loads at once (buckets up to 16k)
static_assert(HDUP_SLOTS % 128 == 0, "the table and its mark bits are cleared 16 bytes at a time");

// 32-bit tag of a hash (bits 8..39, low bit forced so that 0 marks an empty
// slot) and its first probe slot, a function of the tag alone
SHCI_DEV uint32_t hdup_tag(uint64_t g) { return (uint32_t)(g >> 8) | 1u; }
SHCI_DEV int hdup_slot(uint32_t tag) { return (int)(((uint64_t)tag * (uint64_t)HDUP_SLOTS) >> 32); }
SHCI_DEV int hdup_next(int s) { return s + 1 == HDUP_SLOTS ? 0 : s + 1; }

// start[b] = first position of bucket b (top nbits of the hash) in the
// sorted list, start[nbucket] = n: one binary search per thread
__global__ void k_hbounds(const uint64_t* g, int64_t n, int nbits, int64_t nbucket, uint64_t* start) {
  const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (b > nbucket) return;
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if ((g[mid] >> (64 - nbits)) < (uint64_t)b)
      lo = mid + 1;
    else
      hi = mid;
  }
  start[b] = (uint64_t)lo;
}

struct HDupArgs {
  const uint64_t* g;
  const uint64_t* bstart;  // bucket bounds (k_hbounds)
  int64_t n;       // listed hashes, sorted by bucket
  int nbits;       // bucket = top nbits of the hash
  int64_t nbucket;
  uint64_t* filt;
  int fbits;
  unsigned long long* nrep;  // distinct repeated tags (the filter's sizing)
};

// Repeated hashes of each bucket into the filter, one workgroup per bucket
// (buckets dealt round-robin), in two sweeps over the bucket's hashes (odd
// fillers skipped):
//  1. each hash's 32-bit tag goes into an LDS table, linear probing with
//     compare-and-swap from a first slot that depends on the tag alone; a tag
//     that finds itself already there marks its slot.  All copies of a tag
//     walk the same probe sequence and slots are never emptied, so every copy
//     after the first stops at the first one: a slot is marked exactly when
//     its tag occurs more than once, whatever the order;
//  2. each hash finds its tag again (read-only probes) and, if the slot is
//     marked, sets itself in the filter.
// The filter thus holds exactly the hashes whose tag occurs more than once in
// their bucket: every repeated hash, plus the rare pairs of distinct hashes
// that share a bucket and a tag (they only become records).  Low load (~1/3
// at the mean bucket size) keeps the probe runs, which a wavefront waits out
// in lockstep, short.  A bucket whose distinct tags overflow the table is
// taken again in 2^k slices by the hash bits below the bucket bits (all
// copies of a hash share a slice), k sized for HDUP_FILL hashes a slice; past
// k = 16 every hash of the bucket is set.
__global__ void __launch_bounds__(HDUP_THREADS) k_hdup(HDupArgs A) {
  __shared__ __align__(16) uint32_t tab[HDUP_SLOTS];
  __shared__ __align__(16) uint32_t repb[HDUP_SLOTS / 32];
  __shared__ int full_s;
  const int t = threadIdx.x;
  unsigned long long nrep = 0;  // per thread
  // A bucket of typical size has all of this thread's hashes loaded at once
  // (every load issued, clamped into the bucket; fillers in place of the
  // missing ones) and kept for both sweeps.  The next bucket's are loaded as
  // soon as the current one's second sweep is done, so that their latency
  // overlaps the count, the barriers and the next table clear.
  uint64_t gv[HDUP_PER_THREAD];
  int64_t have = -1;  // bucket whose hashes gv holds
  auto typical = [&](int64_t lo, int64_t M) { return M >= 2 && lo + M <= A.n && M <= (int64_t)HDUP_PER_THREAD * HDUP_THREADS; };
  auto load = [&](int64_t lo, int64_t M) {
    const int mlast = (int)M - 1;
    // (the thread index passed through an empty asm, so the compiler cannot
    // hoist the sixteen per-thread offsets out of the bucket loop and keep
    // them in registers)
    int tt = t;
    asm volatile("" : "+v"(tt));
#pragma unroll
    for (int i = 0; i < HDUP_PER_THREAD; ++i) {
      const int j = tt + i * HDUP_THREADS;
      const uint64_t v = A.g[lo + (j < mlast ? j : mlast)];
      gv[i] = j <= mlast ? v : 1ull;
    }
  };
  for (int64_t b = blockIdx.x; b < A.nbucket; b += gridDim.x) {
    const int64_t lo = (int64_t)A.bstart[b], M = (int64_t)A.bstart[b + 1] - lo;
    if (M < 2 || lo + M > A.n) continue;  // uniform
    const uint64_t* gp = A.g + lo;
    const bool regs = M <= (int64_t)HDUP_PER_THREAD * HDUP_THREADS;
    if (regs && have != b) load(lo, M);
    have = -1;
    // one table fill first (a large bucket of few distinct tags fits);
    // slices only when the table overflows
    int k = 0;
    for (;;) {
      const int sshift = 64 - A.nbits - k;
      const uint64_t smask = ((uint64_t)1 << k) - 1;
      bool full = false;  // uniform after the barrier
      unsigned long long cnt = 0;
      for (int64_t sl = 0; sl < ((int64_t)1 << k) && !full; ++sl) {
        // fillers and hashes of other slices take no part
        auto live = [&](uint64_t g) { return !(g & 1ull) && (k == 0 || (int64_t)((g >> sshift) & smask) == sl); };
        // (16-byte stores)
        for (int s = t; s < HDUP_SLOTS / 4; s += HDUP_THREADS) reinterpret_cast<uint4*>(tab)[s] = make_uint4(0u, 0u, 0u, 0u);
        for (int s = t; s < HDUP_SLOTS / 128; s += HDUP_THREADS) reinterpret_cast<uint4*>(repb)[s] = make_uint4(0u, 0u, 0u, 0u);
        if (t == 0) full_s = 0;
        __syncthreads();
        bool miss = false;
        // sweep 1 for one hash; false: table full
        // (at the slot where the tag now is, or -1 for a hash that takes
        // no part)
        auto place = [&](uint64_t g, int& at) -> bool {
          at = -1;
          if (!live(g)) return true;
          const uint32_t tag = hdup_tag(g);
          int s = hdup_slot(tag);
          // a probe run this long means the table is (nearly) full
          for (int probe = 0; probe < HDUP_PROBES; ++probe) {
            const uint32_t old = atomicCAS(&tab[s], 0u, tag);
            if (old == 0u) {
              at = s;
              return true;
            }
            if (old == tag) {
              atomicOr(&repb[s >> 5], 1u << (s & 31));
              at = s;
              return true;
            }
            s = hdup_next(s);
          }
          return false;
        };
        // sweep 2 for one hash at the slot of its tag
        auto mark_at = [&](uint64_t g, int s) {
          if (s >= 0 && ((repb[s >> 5] >> (s & 31)) & 1u)) {
            // (through an empty asm, so the filter word and bits of every
            // hash are not computed ahead and held for this rare branch)
            uint64_t gg = g;
            asm volatile("" : "+v"(gg));
            filt_insert(A.filt, A.fbits, gg);
          }
        };
        // the same for a hash whose slot was not kept: found again
        auto mark = [&](uint64_t g) {
          if (!live(g)) return;
          const uint32_t tag = hdup_tag(g);
          int s = hdup_slot(tag);
          for (int probe = 0; probe < HDUP_PROBES && tab[s] != tag; ++probe) s = hdup_next(s);
          mark_at(g, s);
        };
        uint16_t at[HDUP_PER_THREAD];  // slot of each held hash's tag (0xffff: none)
        if (regs) {
#pragma unroll
          for (int i = 0; i < HDUP_PER_THREAD; ++i) {
            int s = -1;
            miss = miss || !place(gv[i], s);
            at[i] = s < 0 ? (uint16_t)0xffffu : (uint16_t)s;
          }
        } else {
          for (int64_t j = t; j < M && !miss; j += HDUP_THREADS) {
            if (*(volatile int*)&full_s) break;  // another thread found the table full
            int s;
            miss = !place(gp[j], s);
          }
        }
        if (miss) full_s = 1;
        __syncthreads();
        full = full_s != 0;
        if (!full) {
          if (regs) {
#pragma unroll
            for (int i = 0; i < HDUP_PER_THREAD; ++i) mark_at(gv[i], at[i] == 0xffffu ? -1 : (int)at[i]);
            // the last slice of this bucket is done with gv: load the next
            // bucket's hashes now
            const int64_t nb = b + gridDim.x;
            if (sl + 1 == ((int64_t)1 << k) && nb < A.nbucket) {
              const int64_t nlo = (int64_t)A.bstart[nb], nM = (int64_t)A.bstart[nb + 1] - nlo;
              if (typical(nlo, nM)) {
                load(nlo, nM);
                have = nb;
              }
            }
          } else {
            for (int64_t j = t; j < M; j += HDUP_THREADS) mark(gp[j]);
          }
          for (int w = t; w < HDUP_SLOTS / 32; w += HDUP_THREADS) cnt += (unsigned long long)__popc(repb[w]);
        }
        __syncthreads();
      }
      if (!full) {
        nrep += cnt;
        break;
      }
      if (k >= 16) {
        // every hash of the bucket (needs > 2^16 HDUP_SLOTS distinct tags)
        for (int64_t j = t; j < M; j += HDUP_THREADS) {
          const uint64_t g = gp[j];
          if (!(g & 1ull)) {
            filt_insert(A.filt, A.fbits, g);
            nrep += 1;
          }
        }
        break;
      }
      int k2 = k + 1;
      while (((int64_t)HDUP_FILL << k2) < M && k2 < 16) ++k2;
      k = k2;
    }
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) nrep += __shfl_xor(nrep, o);
  if ((t & 63) == 0 && nrep) atomicAdd(A.nrep, nrep);
}

// per work item, the listed terms whose hash passes the filter (the terms the
// write walk turns into records); fillers have no work item
__global__ void k_hmark(const uint64_t* g, const uint32_t* item, int64_t n, const uint64_t* filt, int fbits,
                        uint32_t* mcount) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t gj = g[j];
    if (!(gj & 1ull) && filt_maybe(filt, fbits, gj)) atomicAdd(&mcount[item[j]], 1u);
  }
}

// Sample mode: bounds of each sample's work items (items are in sample order;
// the sample of an item is it_s of its source).  ib[s] = first item of sample
// s, ib[nsamp] = n_items.
__global__ void k_item_bounds(const uint32_t* w_src, const uint32_t* it_s, int64_t n_items, int32_t nsamp,
                              uint64_t* ib) {
  const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s > nsamp) return;
  int64_t lo = 0, hi = n_items;
  while (lo < hi) {
    const int64_t m = (lo + hi) >> 1;
    if ((int64_t)it_s[w_src[m]] < s)
      lo = m + 1;
    else
      hi = m;
  }
  ib[s] = (uint64_t)lo;
}

}  // namespace shci
