// Bucket reduce, one wavefront per bucket, in registers.
//
// After the hash partition a bucket holds on average 32-128 records; the
// wavefront path takes buckets of at most WCAP = 128 (one or two records per
// lane).  It reads each record of its bucket from memory exactly once, with
// coalesced loads, and keeps everything in registers (no LDS): lane l holds
// the records at positions l and 64 + l.  While the loads and the presence
// filter words of V are in flight, 32-bit sort keys (24 hash bits below the
// bucket id, the record's position in the low byte) are sorted by a bitonic
// network across lanes, so equal determinants become adjacent in record
// order; each sorted element then takes its key, value(s), flag, H_aa and
// filter bit from the lane that holds them.  Adjacent elements with equal
// sort bits are checked to have equal keys (otherwise the bucket goes to the
// block kernel), and each segment head adds its members' values, read from
// the following lanes in a loop as long as any segment of the wavefront
// continues; a head looks its determinant up in the hash set of V only when
// the filter does not rule it out, and adds the contribution to per-lane
// accumulators.  Buckets larger than WCAP, or with two different
// determinants sharing the sorted hash bits, are listed (and marked in a
// bitmap) for the block kernel (k_reduce), which sorts by the full key.
//
// Partial sums: each wavefront writes its accumulators once (deterministic
// mode) or once per sample it visited, zeros for the samples it skipped
// (sample mode); block-kernel buckets write per-bucket partials, which the
// final reduction reads through the bitmap in bucket order.
#pragma once
#include <type_traits>

#include "group.hpp"

namespace shci {

constexpr int WCAP = 128;       // records per wavefront bucket
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

struct WaveRedArgs {
  RedArgs r;
  const uint64_t* bstart;  // [nbucket + 1]
  uint32_t* slow_list;     // buckets for the block kernel
  uint32_t* slow_count;
  uint32_t* slow_bits;     // [nbucket / 32 + 1] bitmap of the block kernel's buckets (zeroed)
  Partials Pw;             // per-wavefront partials; sample mode: [nsamp][nwaves]
  int64_t nwaves;
  int32_t nsamp;
};

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

// value of register array v at element `pos` (element r*64 + lane of the
// wavefront), read from the lane that holds it
template <int R, typename T>
SHCI_DEV T wave_fetch(const T (&v)[R], int pos) {
  const int src = pos & 63;
  T out = v[0];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const T x = __shfl(v[r], src);
    out = ((pos >> 6) == r) ? x : out;
  }
  return out;
}

// value of v at sorted element e + k (e = t*64 + lane, 1 <= k < 64; slot
// t + 1 for the lanes that wrap; `fill` past the last slot)
// (every lane executes both cross-lane reads: a lane that is not active
// does not provide its value to them)
template <int R, typename T>
SHCI_DEV T wave_ahead(const T (&v)[R], int t, int k, T fill) {
  const int lane = lane_id();
  const int src = (lane + k) & 63;
  const T a = __shfl(v[t], src);
  const T b = __shfl(v[t + 1 < R ? t + 1 : t], src);
  return (lane + k < 64) ? a : ((t + 1 < R) ? b : fill);
}

// value of v at the previous sorted element (element e - 1 for e = t*64 + lane)
template <int R, typename T>
SHCI_DEV T wave_prev(const T (&v)[R], int t, T fill) {
  const int lane = lane_id();
  const T x = __shfl(v[t], (lane + 63) & 63);
  const T y = __shfl(v[t > 0 ? t - 1 : 0], 63);
  return lane > 0 ? x : (t > 0 ? y : fill);
}

// Returns false if the bucket was handed to the block kernel.  Contributions
// accumulate in acc (per lane).
template <int KW, int R, bool SAMPLE, typename VT>
SHCI_DEV bool wave_bucket(const RedArgs& a, int64_t b, int64_t lo, int M, const WaveRedArgs& A, SegAcc& acc) {
  using VB = typename std::conditional<sizeof(VT) == 4, uint32_t, uint64_t>::type;  // value bits
  const int lane = lane_id();
  const int n = a.n;
  const int bh = a.G.bits_hash;
  const int aw = a.auxbit >> 6;
  const uint64_t am = 1ull << (a.auxbit & 63);
  const VT* vin = static_cast<const VT*>(a.in.v);
  const VT* v2in = static_cast<const VT*>(a.in.v2);
  // ---- stage: every record read once, by position ----
  uint64_t kr[KW][R], hr[R], hh[R];
  VB vr[R], v2r[R];
  uint32_t fr[R], sk[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int j = r * 64 + lane;
    sk[r] = ~0u;
    hr[r] = hh[r] = 0;
    vr[r] = v2r[r] = 0;
    fr[r] = 0;
#pragma unroll
    for (int w = 0; w < KW; ++w) kr[w][r] = 0;
    if (j < M) {
      uint64_t k[KW];
      load_key<KW>(a.in, lo + j, k);
      uint64_t fw = 0;
#pragma unroll
      for (int w = 0; w < KW; ++w) fw = (w == aw) ? k[w] : fw;
      clear_aux<KW>(k, a.auxbit);
#pragma unroll
      for (int w = 0; w < KW; ++w) kr[w][r] = k[w];
      const uint64_t h = det_hash<KW>(k, n);
      hh[r] = h;
      const uint64_t fm = vfilt_bits(h);
      const uint64_t fword = a.V.filt[h >> (64 - a.V.fbits)];
      fr[r] = ((fw & am) ? 1u : 0u) | (((fword & fm) == fm) ? 2u : 0u);
      vr[r] = __builtin_bit_cast(VB, vin[lo + j]);
      if constexpr (SAMPLE) v2r[r] = __builtin_bit_cast(VB, v2in[lo + j]);
      hr[r] = (uint64_t)__double_as_longlong(a.in.haa[lo + j]);
      sk[r] = ((uint32_t)((h << bh) >> 32) & ~0xffu) | (uint32_t)j;
    }
  }
  wave_bitonic<R>(sk);
  // ---- every sorted element takes its record from the lane that holds it ----
  uint64_t ks[KW][R], hs[R], hsh[R];
  VB vs[R], v2s[R];
  uint32_t fs[R], psk[R];
#pragma unroll
  for (int t = 0; t < R; ++t) {
    const int pos = (int)(sk[t] & 0xffu);
#pragma unroll
    for (int w = 0; w < KW; ++w) ks[w][t] = wave_fetch<R>(kr[w], pos);
    hs[t] = wave_fetch<R>(hr, pos);
    hsh[t] = wave_fetch<R>(hh, pos);
    vs[t] = wave_fetch<R>(vr, pos);
    if constexpr (SAMPLE) v2s[t] = wave_fetch<R>(v2r, pos);
    fs[t] = wave_fetch<R>(fr, pos);
  }
#pragma unroll
  for (int t = 0; t < R; ++t) psk[t] = wave_prev<R>(sk, t, ~0u);
  // ---- equal sort bits must mean equal determinants ----
  bool clash = false;
#pragma unroll
  for (int t = 0; t < R; ++t) {
    const int e = t * 64 + lane;
    const bool same = e > 0 && e < M && (sk[t] >> 8) == (psk[t] >> 8);
    if (ballot(same)) {
#pragma unroll
      for (int w = 0; w < KW; ++w) {
        const uint64_t pk = wave_prev<R>(ks[w], t, ~(uint64_t)0);
        clash = clash || (same && pk != ks[w][t]);
      }
    }
  }
  if (ballot(clash)) {
    if (lane == 0) {
      A.slow_list[atomicAdd(A.slow_count, 1u)] = (uint32_t)b;
      atomicOr(&A.slow_bits[b >> 5], 1u << (b & 31));
    }
    return false;
  }
  // ---- segments: each head adds the values of the following lanes ----
  int nbefore = 0;
#pragma unroll
  for (int t = 0; t < R; ++t) {
    const int e0 = t * 64 + lane;
    const uint32_t s0 = sk[t];
    const bool head = e0 < M && (e0 == 0 || (s0 >> 8) != (psk[t] >> 8));
    const uint64_t hb = ballot(head);
    SegSum<VT> sum;
    if (head) {
      if constexpr (SAMPLE)
        sum.add_sample(__builtin_bit_cast(VT, vs[t]), __builtin_bit_cast(VT, v2s[t]), (fs[t] & 1u) != 0);
      else
        sum.add(__builtin_bit_cast(VT, vs[t]), (fs[t] & 1u) != 0);
    }
    int cnt = 1;
    bool open = head;
    for (int k = 1; k < 64 * R; ++k) {
      const uint32_t sa = wave_ahead<R>(sk, t, k, ~0u);
      open = open && (e0 + k < M) && (sa >> 8) == (s0 >> 8);
      if (!ballot(open)) break;
      const VB va = wave_ahead<R>(vs, t, k, (VB)0);
      const uint32_t fa = wave_ahead<R>(fs, t, k, 0u);
      if constexpr (SAMPLE) {
        const VB va2 = wave_ahead<R>(v2s, t, k, (VB)0);
        if (open) sum.add_sample(__builtin_bit_cast(VT, va), __builtin_bit_cast(VT, va2), (fa & 1u) != 0);
      } else {
        if (open) sum.add(__builtin_bit_cast(VT, va), (fa & 1u) != 0);
      }
      cnt += open ? 1 : 0;
    }
    bool inv = false;
    double g = 0.0;
    if (head) {
      sum.finish();
      const double X = sum.X;
      uint64_t k[KW], dk[KW];
#pragma unroll
      for (int w = 0; w < KW; ++w) k[w] = dk[w] = ks[w][t];
      mask_det<KW>(dk, n);  // determinant bits only (no sample id)
      const uint64_t h = hsh[t];
      inv = (fs[t] & 2u) && vset_probe<KW>(a.V, dk, h, n);
      acc.ngen += cnt;
      double Dd = 0.0, gd = 0.0, gG = 0.0;
      if (!inv) {
        const double haa = __longlong_as_double((long long)hs[t]);
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
        acc.nterm += cnt;
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
        a.U.cnt[o] = inv ? -cnt : cnt;
      }
    }
    if constexpr (!SAMPLE) {
      // keep-mode adjoint: every record of the segment gets t * 2 A_a / D_a
      if (a.contrib) {
        const uint32_t pos0 = sk[t] & 0xffu;
        if (head) a.contrib[a.in.pay[lo + pos0]] = inv ? 0.0 : (double)__builtin_bit_cast(VT, vs[t]) * g;
        bool op = head;
        for (int k = 1; k < 64 * R; ++k) {
          const uint32_t sa = wave_ahead<R>(sk, t, k, ~0u);
          op = op && (e0 + k < M) && (sa >> 8) == (s0 >> 8);
          if (!ballot(op)) break;
          const VB va = wave_ahead<R>(vs, t, k, (VB)0);
          if (op) a.contrib[a.in.pay[lo + (sa & 0xffu)]] = inv ? 0.0 : (double)__builtin_bit_cast(VT, va) * g;
        }
      }
    }
    nbefore += __popcll(hb);
  }
  if (a.want_u && lane == 0) {
    a.P.nseg[b] = nbefore;
    a.U.start[b] = (uint64_t)lo;
  }
  return true;
}

template <int KW, bool SAMPLE, typename VT>
__global__ void __launch_bounds__(64 * WRED_WAVES) __attribute__((amdgpu_waves_per_eu(4, 8)))
k_reduce_wave(WaveRedArgs A) {
  const RedArgs& a = A.r;
  const int t = threadIdx.x;
  const int wv = t >> 6;
  const int lane = t & 63;
  const int64_t wave = (int64_t)blockIdx.x * WRED_WAVES + wv;
  const int bh = a.G.bits_hash;
  SegAcc acc;
  // sample mode: the buckets of a sample that this wavefront visits are
  // consecutive in its sequence; the accumulators are written once per
  // sample into slot [sample][wave], zeros into the slots of samples it
  // skips
  int64_t cur_s = -1, next_s = 0;
  // each wavefront takes a contiguous range of buckets: the memory line that
  // two neighbouring buckets share is read once, and the sample of its
  // buckets never decreases
  const int64_t per = (a.G.nbucket + A.nwaves - 1) / A.nwaves;
  const int64_t b_lo = wave * per, b_hi = min(a.G.nbucket, b_lo + per);
  int64_t lo_n = 0, hi_n = 0;  // bounds of the next bucket, loaded one bucket ahead
  if (b_lo < b_hi) {
    lo_n = (int64_t)A.bstart[b_lo];
    hi_n = (int64_t)A.bstart[b_lo + 1];
  }
  for (int64_t b = b_lo; b < b_hi; ++b) {
    const int64_t lo = lo_n, M = hi_n - lo_n;
    if (b + 1 < b_hi) {
      lo_n = hi_n;
      hi_n = (int64_t)A.bstart[b + 2];
    }
    if constexpr (SAMPLE) {
      const int64_t s = b >> bh;
      if (s != cur_s) {
        if (cur_s >= 0) {
          wave_write_partials(A.Pw, cur_s * A.nwaves + wave, acc);
          acc = SegAcc();
          next_s = cur_s + 1;
        }
        if (lane == 0)
          for (int64_t z = next_s; z < s; ++z) wave_zero_partials(A.Pw, z * A.nwaves + wave);
        next_s = s;
        cur_s = s;
      }
    }
    if (M > WCAP) {
      if (lane == 0) {
        A.slow_list[atomicAdd(A.slow_count, 1u)] = (uint32_t)b;
        atomicOr(&A.slow_bits[b >> 5], 1u << (b & 31));
      }
      continue;
    }
    if (M == 0) {
      if (a.want_u && lane == 0) {
        a.P.nseg[b] = 0;
        a.U.start[b] = (uint64_t)lo;
      }
      continue;
    }
    if (M <= 64)
      wave_bucket<KW, 1, SAMPLE, VT>(a, b, lo, (int)M, A, acc);
    else
      wave_bucket<KW, 2, SAMPLE, VT>(a, b, lo, (int)M, A, acc);
  }
  if constexpr (SAMPLE) {
    if (cur_s >= 0) {
      wave_write_partials(A.Pw, cur_s * A.nwaves + wave, acc);
      next_s = cur_s + 1;
    }
    if (lane == 0)
      for (int64_t z = next_s; z < A.nsamp; ++z) wave_zero_partials(A.Pw, z * A.nwaves + wave);
  } else {
    wave_write_partials(A.Pw, wave, acc);
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
