// Bucket reduce, one wavefront per bucket.
//
// After the hash partition a bucket holds on average ~100 records (at most
// WCAP are handled here).  A wavefront loads the bucket's keys, forms 32-bit
// sort keys (24 hash bits below the bucket id, with the record's position in
// the low byte) and sorts them by a bitonic network in registers, so equal
// determinants become adjacent in record order.  The sorted keys and the full
// hash of every record are kept in LDS (3 KB per wavefront): keys and values
// are read again from global memory (cache-resident) when a segment head sums
// its segment, looks the determinant up in the hash set of V, takes H_aa from
// the record and accumulates the contribution.  No block-wide barrier is
// involved.  Buckets larger than WCAP, or in which two different determinants
// share all sorted hash bits, are listed for the block kernel (k_reduce),
// which sorts by the full key.
#pragma once
#include "group.hpp"

namespace shci {

constexpr int WCAP = 256;       // records per wavefront bucket
constexpr int WRED_WAVES = 8;   // wavefronts per block

// ascending bitonic sort of R*64 keys held as v[r] at element r*64 + lane
template <int R>
SHCI_DEV void wave_bitonic(uint32_t (&v)[R]) {
  const int lane = lane_id();
#pragma unroll
  for (int k = 2; k <= 64 * R; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int e = r * 64 + lane;
        const bool up = (e & k) == 0;
        if (j >= 64) {
          const int rp = r ^ (j >> 6);
          if (rp > r) {
            const uint32_t x = v[r], y = v[rp];
            const bool sw = up ? (x > y) : (x < y);
            v[r] = sw ? y : x;
            v[rp] = sw ? x : y;
          }
        } else {
          const uint32_t p = (uint32_t)__shfl_xor((int)v[r], j);
          const bool lower = (lane & j) == 0;
          const uint32_t mn = v[r] < p ? v[r] : p;
          const uint32_t mx = v[r] < p ? p : v[r];
          v[r] = (lower == up) ? mn : mx;
        }
      }
    }
  }
}

// per-wavefront LDS: the sorted keys of the current bucket and the
// determinant hash of each record (by position)
struct WaveStage {
  uint32_t sk[WCAP];
  uint64_t h[WCAP];
};

struct WaveRedArgs {
  RedArgs r;
  const uint64_t* bstart;  // [nbucket + 1]
  uint32_t* slow_list;     // buckets for the block kernel
  uint32_t* slow_count;
  Partials Pw;             // per-wavefront partials (deterministic mode)
};

// load the bucket's keys, sort their 32-bit sort keys (R*64 >= M) and leave
// them in W.sk, the hashes in W.h
template <int KW, int R>
SHCI_DEV void wave_stage_sort(const RedArgs& a, WaveStage& W, int64_t lo, int M) {
  const int lane = lane_id();
  const int bh = a.G.bits_hash;
  uint32_t sk[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int j = r * 64 + lane;
    sk[r] = ~0u;
    if (j < M) {
      uint64_t k[KW];
      load_key<KW>(a.in, lo + j, k);
      const uint64_t h = det_hash<KW>(k, a.n);
      W.h[j] = h;
      sk[r] = ((uint32_t)((h << bh) >> 32) & ~0xffu) | (uint32_t)j;
    }
  }
  wave_bitonic<R>(sk);
#pragma unroll
  for (int r = 0; r < R; ++r) W.sk[r * 64 + lane] = sk[r];
}

struct SegAcc {
  double e2p = 0.0, de0p = 0.0, e2sq = 0.0, dmn = INFINITY;
  int64_t nterm = 0, ngen = 0;
  int32_t nuniq = 0, nintr = 0, nzero = 0;
};

SHCI_DEV void wave_write_partials(const Partials& P, int64_t b, SegAcc acc) {
  double e2p = acc.e2p, de0p = acc.de0p, e2sq = acc.e2sq, dmn = acc.dmn;
  int64_t nterm = acc.nterm, ngen = acc.ngen;
  int32_t nuniq = acc.nuniq, nintr = acc.nintr, nzero = acc.nzero;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    e2p += __shfl_xor(e2p, o);
    de0p += __shfl_xor(de0p, o);
    e2sq += __shfl_xor(e2sq, o);
    dmn = fmin(dmn, __shfl_xor(dmn, o));
    nterm += __shfl_xor(nterm, o);
    ngen += __shfl_xor(ngen, o);
    nuniq += __shfl_xor(nuniq, o);
    nintr += __shfl_xor(nintr, o);
    nzero += __shfl_xor(nzero, o);
  }
  if (lane_id() == 0) {
    P.e2[b] = e2p;
    P.de0[b] = de0p;
    P.e2sq[b] = e2sq;
    P.nterm[b] = nterm;
    P.ngen[b] = ngen;
    P.nuniq[b] = nuniq;
    P.nintr[b] = nintr;
    P.nzero[b] = nzero;
    P.mind[b] = dmn;
  }
}

SHCI_DEV void wave_zero_partials(const Partials& P, int64_t b) {
  P.e2[b] = 0.0;
  P.de0[b] = 0.0;
  P.e2sq[b] = 0.0;
  P.nterm[b] = 0;
  P.ngen[b] = 0;
  P.nuniq[b] = 0;
  P.nintr[b] = 0;
  P.nzero[b] = 0;
  P.mind[b] = INFINITY;
}

// Returns false if the bucket was handed to the block kernel.  Contributions
// accumulate in acc (per lane); in sample mode the caller reduces acc per
// bucket, otherwise once per wavefront at the end.
template <int KW, bool SAMPLE, typename VT>
SHCI_DEV bool wave_bucket(const RedArgs& a, WaveStage& W, int64_t b, int64_t lo, int M,
                          uint32_t* slow_list, uint32_t* slow_count, SegAcc& acc) {
  const int lane = lane_id();
  const int n = a.n;
  const int bh = a.G.bits_hash;
  const int aw = a.auxbit >> 6;
  const uint64_t am = 1ull << (a.auxbit & 63);
  const VT* vin = static_cast<const VT*>(a.in.v);
  const VT* v2in = static_cast<const VT*>(a.in.v2);
  const uint64_t* auxw = a.in.k[0];  // key word holding the flag bit
#pragma unroll
  for (int w = 1; w < KW; ++w)
    if (w == aw) auxw = a.in.k[w];
  auto key_of = [&](int id, uint64_t (&k)[KW]) {
    load_key<KW>(a.in, lo + id, k);
    clear_aux<KW>(k, a.auxbit);
  };
  // equal sort bits must mean equal determinants
  bool clash = false;
#pragma unroll 1
  for (int e = lane + 1; e < M; e += 64) {
    const uint32_t cur = W.sk[e], prv = W.sk[e - 1];
    if ((cur >> 8) == (prv >> 8)) {
      uint64_t kx[KW], ky[KW];
      key_of((int)(cur & 0xff), kx);
      key_of((int)(prv & 0xff), ky);
      bool eq = true;
#pragma unroll
      for (int w = 0; w < KW; ++w) eq = eq && (kx[w] == ky[w]);
      clash = clash || !eq;
    }
  }
  if (ballot(clash)) {
    if (lane == 0) slow_list[atomicAdd(slow_count, 1u)] = (uint32_t)b;
    return false;
  }
  int nbefore = 0;
#pragma unroll 1
  for (int base = 0; base < M; base += 64) {
    const int e0 = base + lane;
    const uint32_t s0 = (e0 < M) ? W.sk[e0] : 0u;
    const bool head = e0 < M && (e0 == 0 || (s0 >> 8) != (W.sk[e0 - 1] >> 8));
    const uint64_t hb = ballot(head);
    if (head) {
      int e1 = e0 + 1;
      while (e1 < M && (W.sk[e1] >> 8) == (s0 >> 8)) ++e1;
      const int first = (int)(s0 & 0xff);
      SegSum<VT> sum;
      for (int e = e0; e < e1; ++e) {
        const int id = (e == e0) ? first : (int)(W.sk[e] & 0xff);
        if constexpr (SAMPLE)
          sum.add_sample(vin[lo + id], v2in[lo + id], (auxw[lo + id] & am) != 0ull);
        else
          sum.add(vin[lo + id], (auxw[lo + id] & am) != 0ull);
      }
      sum.finish();
      const double X = sum.X;
      uint64_t k[KW];
      key_of(first, k);
      uint64_t a0, a1, b0, b1;
      unpack_det<KW>(k, n, a0, a1, b0, b1);
      uint64_t dk[KW];
#pragma unroll
      for (int w = 0; w < KW; ++w) dk[w] = k[w];
      mask_det<KW>(dk, n);  // determinant bits only (no sample id)
      const uint64_t h = W.h[first];
      const bool inv = vset_contains_h<KW>(a.V, dk, h, n);
      const int cntk = e1 - e0;
      acc.ngen += cntk;
      double Dd = 0.0, g = 0.0, gd = 0.0, gG = 0.0;
      if (!inv) {
        const double haa = a.in.haa[lo + first];
        Dd = a.e0 - haa;
        const double rd = 1.0 / Dd;
        double contrib;
        if constexpr (SAMPLE) {
          const double G = rd / (a.nd * (a.nd - 1.0));
          contrib = sum.sample_bracket() * G;
          acc.de0p += -contrib * rd;
          g = 2.0 * X * G;
          gd = 2.0 * sum.Xd * G;
          gG = G;
        } else {
          // (A^2 - A_hi^2) / D; A_hi (terms above the upper threshold) is 0
          // unless a two-threshold evaluation was asked for
          const double a2 = X * X - sum.Xd * sum.Xd;
          contrib = a2 * rd;
          acc.de0p += -a2 * rd * rd;
          g = 2.0 * X * rd;
        }
        acc.e2p += contrib;
        acc.e2sq += contrib * contrib;
        acc.nterm += cntk;
        acc.nuniq += 1;
        acc.nintr += Dd > 0.0;
        acc.nzero += Dd == 0.0;
        acc.dmn = fmin(acc.dmn, fabs(Dd));
      }
      if (a.want_u) {
        const int64_t o = lo + nbefore + rank_below(hb);
#pragma unroll
        for (int w = 0; w < KW; ++w) a.U.k[w][o] = k[w];
        a.U.h2[o] = (uint32_t)((h << bh) >> 32);
        // deterministic: A_a, D_a, 2 A_a / D_a; sample: 2 X^d G, G, 2 X G with
        // G = 1 / (D_a Nd (Nd - 1)) (the adjoint's per-a factors)
        a.U.A[o] = SAMPLE ? gd : X;
        a.U.D[o] = SAMPLE ? gG : Dd;
        a.U.g[o] = g;
        a.U.cnt[o] = inv ? -cntk : cntk;
      }
    }
    nbefore += __popcll(hb);
  }
  // the contributions stay in acc; the caller writes them once per run of
  // buckets (sample mode) or once per wavefront
  if (lane == 0) wave_zero_partials(a.P, b);
  if (lane == 0) {
    a.P.nseg[b] = nbefore;
    if (a.want_u) a.U.start[b] = (uint64_t)lo;
  }
  return true;
}

template <int KW, bool SAMPLE, typename VT>
__global__ void __launch_bounds__(64 * WRED_WAVES) __attribute__((amdgpu_waves_per_eu(6, 8))) k_reduce_wave(WaveRedArgs A) {
  __shared__ WaveStage WS[WRED_WAVES];
  const RedArgs& a = A.r;
  const int t = threadIdx.x;
  const int wv = t >> 6;
  const int lane = t & 63;
  WaveStage& W = WS[wv];
  const int64_t nwaves = (int64_t)gridDim.x * WRED_WAVES;
  const int bh = a.G.bits_hash;
  SegAcc acc;
  // sample mode: the buckets of one sample that this wavefront reduced add
  // up in acc and are written into the partials of the last of them (the
  // others hold zeros), so the cross-lane reduction runs once per sample
  int64_t last_ok = -1;
  for (int64_t b = (int64_t)blockIdx.x * WRED_WAVES + wv; b < a.G.nbucket; b += nwaves) {
    if constexpr (SAMPLE) {
      if (last_ok >= 0 && (b >> bh) != (last_ok >> bh)) {
        wave_write_partials(a.P, last_ok, acc);
        acc = SegAcc();
        last_ok = -1;
      }
    }
    const int64_t lo = (int64_t)A.bstart[b];
    const int64_t M = (int64_t)A.bstart[b + 1] - lo;
    if (M > WCAP) {
      if (lane == 0) A.slow_list[atomicAdd(A.slow_count, 1u)] = (uint32_t)b;
      continue;
    }
    if (M <= 64)
      wave_stage_sort<KW, 1>(a, W, lo, (int)M);
    else if (M <= 128)
      wave_stage_sort<KW, 2>(a, W, lo, (int)M);
    else
      wave_stage_sort<KW, 4>(a, W, lo, (int)M);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (wave_bucket<KW, SAMPLE, VT>(a, W, b, lo, (int)M, A.slow_list, A.slow_count, acc)) last_ok = b;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  if constexpr (SAMPLE) {
    if (last_ok >= 0) wave_write_partials(a.P, last_ok, acc);
  } else {
    wave_write_partials(A.Pw, (int64_t)blockIdx.x * WRED_WAVES + wv, acc);
  }
}

// bucket start offsets from the bucket id of every record (records are
// sorted by bucket id): start[x] = first record with bucket id >= x
__global__ void k_bucket_bounds(const uint32_t* bid, int64_t nrec, int64_t nbucket, uint64_t* start) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j <= nrec;
       j += (int64_t)gridDim.x * blockDim.x) {
    const int64_t cur = (j < nrec) ? (int64_t)bid[j] : nbucket;
    const int64_t prv = (j > 0) ? (int64_t)bid[j - 1] : -1;
    for (int64_t x = prv + 1; x <= cur; ++x) start[x] = (uint64_t)j;
  }
}

}  // namespace shci
