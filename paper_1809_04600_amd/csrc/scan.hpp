// Device-wide exclusive prefix sum: tiles of 4096 elements scanned in LDS,
// tile totals scanned recursively, then added back.  Deterministic (integer).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace shci {

constexpr int SCAN_TILE = 4096;  // 256 threads x 16

template <typename TO>
__device__ TO block_excl_scan(TO v, TO* sh, TO* total) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int o = 1; o < 256; o <<= 1) {
    TO x = (t >= o) ? sh[t - o] : (TO)0;
    __syncthreads();
    sh[t] += x;
    __syncthreads();
  }
  TO incl = sh[t];
  *total = sh[255];
  __syncthreads();
  return incl - v;
}

template <typename TI, typename TO>
__global__ void __launch_bounds__(256) k_scan_tiles(const TI* in, TO* out, int64_t n, TO* tile_sums,
                                                    TO* total) {
  __shared__ TO sh[256];
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * 16;
  TO loc[16];
  TO s = 0;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int64_t i = base + j;
    TO v = (i < n) ? (TO)in[i] : (TO)0;
    loc[j] = s;
    s += v;
  }
  TO tot;
  const TO pre = block_excl_scan<TO>(s, sh, &tot);
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int64_t i = base + j;
    if (i < n) out[i] = pre + loc[j];
  }
  if (threadIdx.x == 0) {
    if (tile_sums) tile_sums[blockIdx.x] = tot;
    if (total) *total = tot;
  }
}

template <typename TO>
__global__ void k_scan_add(TO* out, int64_t n, const TO* tile_offs) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] += tile_offs[i / SCAN_TILE];
}

// scratch for up to 4 recursion levels
struct ScanTmp {
  void* lvl[4] = {nullptr, nullptr, nullptr, nullptr};
  void* off[4] = {nullptr, nullptr, nullptr, nullptr};
  // words: 64-bit words per element (2 for 128-bit sums)
  template <class CV>
  void carve(CV& cv, int64_t n, int words = 1) {
    int64_t m = n;
    for (int l = 0; l < 4; ++l) {
      m = (m + SCAN_TILE - 1) / SCAN_TILE;
      lvl[l] = cv.template take<uint64_t>(words * (m + 1));
      off[l] = cv.template take<uint64_t>(words * (m + 1));
      if (m <= 1) break;
    }
  }
};

template <typename TI, typename TO>
int scan_exclusive_lvl(const TI* in, TO* out, int64_t n, ScanTmp& tmp, TO* total, hipStream_t st,
                       int level) {
  if (n <= 0) return 0;
  const int64_t tiles = (n + SCAN_TILE - 1) / SCAN_TILE;
  if (tiles == 1) {
    k_scan_tiles<TI, TO><<<1, 256, 0, st>>>(in, out, n, nullptr, total);
    return hipGetLastError() == hipSuccess ? 0 : -8;
  }
  if (level >= 4) return -6;
  TO* sums = static_cast<TO*>(tmp.lvl[level]);
  TO* offs = static_cast<TO*>(tmp.off[level]);
  k_scan_tiles<TI, TO><<<(unsigned)tiles, 256, 0, st>>>(in, out, n, sums, nullptr);
  int r = scan_exclusive_lvl<TO, TO>(sums, offs, tiles, tmp, total, st, level + 1);
  if (r) return r;
  k_scan_add<TO><<<(unsigned)((n + 255) / 256), 256, 0, st>>>(out, n, offs);
  return hipGetLastError() == hipSuccess ? 0 : -8;
}

// exclusive scan of in[0..n) into out (may alias in for TI == TO); *total
// (device, nullable) receives the sum
template <typename TI, typename TO>
int scan_exclusive(const TI* in, TO* out, int64_t n, ScanTmp& tmp, TO* total, hipStream_t st) {
  return scan_exclusive_lvl<TI, TO>(in, out, n, tmp, total, st, 0);
}

}  // namespace shci
