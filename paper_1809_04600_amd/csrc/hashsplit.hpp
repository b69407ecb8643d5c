// Singleton split of the screened terms.
//
// Almost every perturbative determinant a is reached by one term only (at
// the small thresholds of the stochastic part, all but a fraction of a
// percent), and a group of one term needs no grouping: its contribution is
// the term's own.  So before any record is written:
//  1. the count walk lists the 64-bit grouping hash (determinant hash with the
//     sample id mixed in) and the work item of every kept term, 12 bytes a
//     term instead of a record of 44-60;
//  2. the list is partitioned on the top hash bits (the same stable LSD passes
//     as the records), buckets of ~100 hashes;
//  3. per bucket, one wavefront finds the hashes that occur more than once
//     (an LDS hash table per wavefront) and sets them in a presence filter;
//  4. every listed term whose hash passes the filter is counted for its work
//     item; the scan of these counts places the records.
// The write walk then writes records only for terms whose hash passes the
// filter (every term of an a with several terms does, and a few false
// positives) and sums the contribution of every other term in place.  The
// decision depends on the hash alone, so all terms of one a take the same
// side and the records of an a are complete; the split changes the order of
// the final sums only.
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

// one stable LSD pass over (hash, work item) pairs, as k_part_scatter
__global__ void __launch_bounds__(PTHREADS) k_hpart_scatter(HPassArgs a) {
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
  tile_scatter<uint64_t>(L, keys, a.kout, tile_n, lpos);
  tile_scatter<uint32_t>(L, items, a.iout, tile_n, lpos);
}

// start[b] = first position of bucket b (top nbits of the hash), start[nb] = n
__global__ void k_hbounds(const uint64_t* g, int64_t n, int nbits, int64_t nbucket, uint64_t* start) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j <= n; j += (int64_t)gridDim.x * blockDim.x) {
    const int64_t cur = (j < n) ? (int64_t)(nbits ? (g[j] >> (64 - nbits)) : 0ull) : nbucket;
    const int64_t prv = (j > 0) ? (int64_t)(nbits ? (g[j - 1] >> (64 - nbits)) : 0ull) : -1;
    for (int64_t x = prv + 1; x <= cur; ++x) start[x] = (uint64_t)j;
  }
}

constexpr int HDUP_WAVES = 4;     // wavefronts per block
constexpr int HDUP_SLOTS = 512;   // LDS hash table per wavefront
constexpr int HDUP_MAX = 256;     // hashes per table fill; larger buckets are taken in slices

struct HDupArgs {
  const uint64_t* g;
  const uint32_t* item;
  const uint64_t* bstart;
  int64_t n;  // listed hashes
  int64_t nbucket;
  int nbits;
  int64_t nwaves;
  uint64_t* filt;
  int fbits;
  unsigned long long* nrep;  // distinct repeated hashes set in the filter
};

// Repeated hashes of each bucket into the filter.  Each wavefront takes a
// contiguous range of buckets.  A bucket's hashes (fillers skipped) go into a
// wave-private LDS table, linear probing from the low hash bits with
// compare-and-swap; a hash that finds itself already there marks its slot,
// and every marked slot is set in the filter once.  A bucket with more
// distinct hashes than the table holds is taken again in 2^k slices by the
// hash bits below the bucket bits (a fresh table per slice), so the set of
// repeated hashes, and with it the filter, depends on the listed terms only.
// (Past 2^16 slices every hash of the bucket is set: more records, same
// result.)
__global__ void __launch_bounds__(64 * HDUP_WAVES) k_hdup(HDupArgs A) {
  __shared__ unsigned long long tab[HDUP_WAVES][HDUP_SLOTS];
  __shared__ uint8_t rep[HDUP_WAVES][HDUP_SLOTS];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t wave = (int64_t)blockIdx.x * HDUP_WAVES + wv;
  if (wave >= A.nwaves) return;
  const int64_t per = (A.nbucket + A.nwaves - 1) / A.nwaves;
  const int64_t b_lo = wave * per, b_hi = min(A.nbucket, b_lo + per);
  unsigned long long nrep = 0;  // per lane
  for (int64_t b = b_lo; b < b_hi; ++b) {
    const int64_t lo = (int64_t)A.bstart[b];
    const int64_t M = (int64_t)A.bstart[b + 1] - lo;
    if (M < 2 || lo < 0 || lo + M > A.n) continue;  // uniform
    int k = 0;            // uniform
    for (;;) {
      const int sshift = 64 - A.nbits - k;
      unsigned long long found = 0;  // per lane, this attempt
      bool full = false;             // uniform
      for (int64_t sl = 0; sl < ((int64_t)1 << k) && !full; ++sl) {
        for (int s = lane; s < HDUP_SLOTS; s += 64) {
          tab[wv][s] = 0ull;
          rep[wv][s] = 0;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        bool miss = false;
        for (int64_t j0 = 0; j0 < M; j0 += 64) {
          const int64_t j = j0 + lane;
          if (j < M && A.item[lo + j] != HASH_HOLE) {
            const uint64_t g = A.g[lo + j];
            if (k == 0 || (int64_t)((g >> sshift) & (((uint64_t)1 << k) - 1)) == sl) {
              int s = (int)(g & (HDUP_SLOTS - 1));
              bool placed = false;
              for (int probe = 0; probe < HDUP_SLOTS; ++probe) {
                const unsigned long long old = atomicCAS(&tab[wv][s], 0ull, (unsigned long long)g);
                if (old == 0ull) {
                  placed = true;
                  break;
                }
                if (old == (unsigned long long)g) {
                  rep[wv][s] = 1;
                  placed = true;
                  break;
                }
                s = (s + 1) & (HDUP_SLOTS - 1);
              }
              miss = miss || !placed;
            }
          }
        }
        full = ballot(miss) != 0ull;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        if (!full) {
          for (int s = lane; s < HDUP_SLOTS; s += 64) {
            if (rep[wv][s]) {
              filt_insert(A.filt, A.fbits, tab[wv][s]);
              found += 1;
            }
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
      }
      if (!full) {
        nrep += found;
        break;
      }
      // too many distinct hashes for one table: slices of ~HDUP_MAX hashes
      int k2 = k + 1;
      while (((int64_t)HDUP_MAX << k2) < M) ++k2;
      if (k2 > 16 || A.nbits + k2 >= 64) {
        for (int64_t j = lane; j < M; j += 64) {
          if (A.item[lo + j] != HASH_HOLE) {
            filt_insert(A.filt, A.fbits, A.g[lo + j]);
            nrep += 1;
          }
        }
        break;
      }
      k = k2;
    }
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) nrep += __shfl_xor(nrep, o);
  if (lane == 0 && nrep) atomicAdd(A.nrep, nrep);
}

// per work item, the listed terms whose hash passes the filter (the terms the
// write walk turns into records); fillers have no work item
__global__ void k_hmark(const uint64_t* g, const uint32_t* item, int64_t n, const uint64_t* filt, int fbits,
                        uint32_t* mcount) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t it = item[j];
    if (it != HASH_HOLE && filt_maybe(filt, fbits, g[j])) atomicAdd(&mcount[it], 1u);
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
