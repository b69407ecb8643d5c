// Host side of the C ABI declared in include/shci_pt2.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <functional>
#include <mutex>
#include <string>
#include <thread>
#include <new>
#include <vector>

#include "../../include/shci_pt2.h"
#include "alias.hpp"
#include "group.hpp"
#include "hashsplit.hpp"
#include "hc.hpp"
#include "reduce_wave.hpp"
#include "scan.hpp"

using namespace shci;

namespace {

thread_local char g_msg[512] = "";

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_msg, sizeof g_msg, fmt, ap);
  va_end(ap);
  return code;
}

#define HIPCHK(x)                                                                     \
  do {                                                                                \
    hipError_t e_ = (x);                                                              \
    if (e_ != hipSuccess)                                                             \
      return fail(SHCI_ERR_HIP, "%s failed: %s (%s:%d)", #x, hipGetErrorString(e_),  \
                  __FILE__, __LINE__);                                                \
  } while (0)

#define CHK(...)                    \
  do {                              \
    int s_ = (__VA_ARGS__);         \
    if (s_ != SHCI_OK) return s_;   \
  } while (0)

// grow-only device buffer (the context's memory when the caller passes no
// workspace); growing waits for the calling stream, then reallocates
struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
  int ensure(size_t bytes, size_t limit, hipStream_t st) {
    if (bytes <= cap) return SHCI_OK;
    if (limit && bytes > limit)
      return fail(SHCI_ERR_WORKSPACE, "workspace of %zu bytes exceeds the limit of %zu", bytes, limit);
    if (p) {
      hipError_t e = hipStreamSynchronize(st);
      if (e != hipSuccess) return fail(SHCI_ERR_HIP, "hipStreamSynchronize: %s", hipGetErrorString(e));
      (void)hipFree(p);
      p = nullptr;
      cap = 0;
    }
    size_t want = bytes + bytes / 8 + (1u << 20);
    if (hipMalloc(&p, want) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
      if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        p = nullptr;
        return fail(SHCI_ERR_WORKSPACE, "cannot allocate %zu bytes of device workspace", bytes);
      }
      want = bytes;
    }
    cap = want;
    return SHCI_OK;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
  }
};

// bump allocator over a region (two passes: size, then carve)
struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* b) : base(static_cast<char*>(b)) {}
  template <class T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* r = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return r;
  }
};

// Regions of device memory a call uses, by purpose.  With a caller
// workspace every region is carved from it in call order (stack discipline:
// mark / reset), and the call allocates nothing; without one, each region is
// the context's grow-only buffer of that purpose.
enum Slot {
  SL_V, SL_ITEMS, SL_SPLIT, SL_FILT, SL_HASH, SL_HASH2, SL_REC, SL_SAMPLE, SL_DRAWS, SL_ALIAS, SL_TABLE, SL_SEL,
  SL_HC, SL_HCL0, SL_HCL1, NSLOT
};

constexpr size_t WS_ALIGN = 256;

int ceil_log2(uint64_t x) {
  int b = 0;
  while ((1ull << b) < x) ++b;
  return b;
}

}  // namespace

namespace {
// What one evaluation in flight uses besides its workspace: device scratch
// words, events, the grow-only buffers of context memory and the split's
// size estimates.  The context is lane 0; a second lane lets two sample
// chunks run at once.
struct Lane {
  DevBuf slot[NSLOT];
  double split_rate[2] = {0.0, 0.0};  // kept terms per work item of the last job that could split (det, sample)
  double split_rep[2] = {0.0, 0.0};   // repeated hashes per listed hash of the last split job
  uint32_t* dflag = nullptr;   // device scratch words (flags, counters)
  unsigned long long* dctr = nullptr;  // device 64-bit counters: hash-list claims, repeated hashes
  DevResult* dres = nullptr;
  hipEvent_t ev[10] = {};
  hipEvent_t evp[16] = {};  // around the partition scatter launches of a job (first 8 passes)
  hipEvent_t evh[2] = {};   // around the singleton split (hash partition, repeat finder, marks)
};
}  // namespace

struct shci_pt2_ctx : Lane {
  int device = 0;
  Tables T;
  DevBuf tables;
  size_t ws_limit = 0;
  int64_t rec_limit = 0;  // records per pass (0: from device memory)
  int grouping = SHCI_GROUP_AUTO;
  int lanes = 2;                  // sample chunks in flight at once with a caller workspace
  int64_t split_bucket = HDUP_MEAN;  // hashes a repeat-finder bucket aims at
  Lane lane1;                     // second lane (sample chunks two at a time)
  hipStream_t lane1_stream = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};

namespace {

struct Arena {
  shci_pt2_ctx* X = nullptr;
  Lane* L = nullptr;     // whose grow-only buffers serve context memory
  hipStream_t st = nullptr;
  char* base = nullptr;  // caller workspace, or nullptr: the context's buffers
  size_t cap = 0, off = 0;
  Arena(shci_pt2_ctx* x, hipStream_t s, void* ws, size_t bytes, Lane* lane = nullptr)
      : X(x), L(lane ? lane : x), st(s), base(static_cast<char*>(ws)), cap(ws ? bytes : 0) {}
  bool caller() const { return base != nullptr; }
  size_t mark() const { return off; }
  void reset(size_t m) { off = m; }
  // bytes still free in the caller workspace
  size_t remaining() const {
    const size_t o = (off + WS_ALIGN - 1) & ~(WS_ALIGN - 1);
    return cap > o ? cap - o : 0;
  }
  int take(int slot, size_t bytes, void** p) {
    if (caller()) {
      const size_t o = (off + WS_ALIGN - 1) & ~(WS_ALIGN - 1);
      if (o + bytes > cap)
        return fail(SHCI_ERR_WORKSPACE, "the workspace of %zu bytes is too small (%zu more needed)", cap,
                    o + bytes - cap);
      *p = base + o;
      off = o + bytes;
      return SHCI_OK;
    }
    CHK(L->slot[slot].ensure(bytes, X->ws_limit, st));
    *p = L->slot[slot].p;
    return SHCI_OK;
  }
};

// carve a planned layout from a region of the arena: plan(cv) runs once to
// size it and once on the region
template <class Plan>
int carve_region(Arena& A, int slot, Plan&& plan) {
  Carver cv(nullptr);
  plan(cv);
  void* p = nullptr;
  CHK(A.take(slot, std::max<size_t>(cv.off, 1), &p));
  Carver cv2(p);
  plan(cv2);
  return SHCI_OK;
}

constexpr int GEN_BLOCKS_PER_CU = 32;  // many more blocks than resident: blocks that finish early are replaced
constexpr int RED_BLOCKS_PER_CU = 8;

int num_cus(int dev) {
  static int cus = 0;
  if (!cus) {
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) == hipSuccess) cus = p.multiProcessorCount;
    if (cus <= 0) cus = 256;
  }
  return cus;
}

int key_words(int n, int sbits) { return (2 * n + sbits + 1 + 63) / 64; }

// ----------------------------------------------------------------------------
// Small device utilities
// ----------------------------------------------------------------------------
__global__ void k_fill_u64(uint64_t* p, int64_t n, uint64_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void k_zero_result(DevResult* r) {
  r->e2 = 0.0;
  r->de0 = 0.0;
  r->e2sq = 0.0;
  r->mind = INFINITY;
  r->nterm = r->ngen = r->nuniq = r->nintr = r->nzero = 0;
  r->overflow = 0;
  r->flags = 0;
}

// flags: 1 bad det, 2 non-finite c, 4 duplicate, 8 hash set full, 16 draw out of range
__global__ void k_validate(const uint64_t* dets, const double* c, int64_t nd, int n, int na, int nb,
                           uint32_t* flag) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= nd) return;
  uint64_t m0, m1;
  low_mask(n, m0, m1);
  const uint64_t a0 = dets[4 * i], a1 = dets[4 * i + 1], b0 = dets[4 * i + 2], b1 = dets[4 * i + 3];
  bool ok = (__popcll(a0) + __popcll(a1) == na) && (__popcll(b0) + __popcll(b1) == nb);
  ok = ok && !(a0 & ~m0) && !(a1 & ~m1) && !(b0 & ~m0) && !(b1 & ~m1);
  if (!ok) atomicOr(flag, 1u);
  const double v = c[i];
  if (!(v - v == 0.0)) atomicOr(flag, 2u);
}

// deterministic sum of |c| (fixed per-thread chunks, fixed tree)
__global__ void __launch_bounds__(1024) k_sum_abs(const double* c, int64_t nd, double* out) {
  __shared__ double r[1024];
  const int t = threadIdx.x;
  const int64_t chunk = (nd + 1023) / 1024;
  double s = 0.0;
  for (int64_t i = t * chunk; i < min(nd, (int64_t)(t + 1) * chunk); ++i) s += fabs(c[i]);
  r[t] = s;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if (t < o) r[t] += r[t + o];
    __syncthreads();
  }
  if (t == 0) *out = r[0];
}

// Per sample: sort the draws in LDS, run-length encode, write (det, weight)
// at [s * nd + k] and the number of distinct dets.
constexpr int MAX_DRAWS = 4096;
__global__ void __launch_bounds__(256) k_sample_items(const uint32_t* draws, int32_t nd, int64_t ndet,
                                                     uint32_t* it_det, uint32_t* it_w, uint32_t* ucount,
                                                     uint32_t* flag) {
  __shared__ SortBufs<MAX_DRAWS> B;
  __shared__ SplitScratch S;
  __shared__ uint32_t scan_sh[256];
  __shared__ uint16_t heads[MAX_DRAWS + 1];
  const int t = threadIdx.x;
  const int s = blockIdx.x;
  S.wcnt[0][t] = S.wcnt[1][t] = S.wcnt[2][t] = S.wcnt[3][t] = 0;
  for (int j = t; j < nd; j += 256) {
    uint32_t v = draws[(int64_t)s * nd + j];
    if ((int64_t)v >= ndet) {
      atomicOr(flag, 16u);
      v = 0;
    }
    B.h2a[j] = v;
    B.ia[j] = (uint16_t)j;
  }
  __syncthreads();
  for (int pass = 0; pass < 4; ++pass) {
    const int sh = pass * 8;
    if ((pass & 1) == 0)
      lds_pass<MAX_DRAWS>(nd, B.h2a, B.ia, B.h2b, B.ib, S, scan_sh,
                          [&](int j) { return (B.h2a[j] >> sh) & 0xffu; });
    else
      lds_pass<MAX_DRAWS>(nd, B.h2b, B.ib, B.h2a, B.ia, S, scan_sh,
                          [&](int j) { return (B.h2b[j] >> sh) & 0xffu; });
  }
  const int per = (nd + 255) / 256;
  const int j_lo = t * per, j_hi = min(nd, j_lo + per);
  uint32_t cnt = 0;
  for (int j = j_lo; j < j_hi; ++j) cnt += (j == 0) || (B.h2a[j] != B.h2a[j - 1]);
  uint32_t tot;
  uint32_t idx = block_scan256(cnt, scan_sh, &tot);
  for (int j = j_lo; j < j_hi; ++j)
    if ((j == 0) || (B.h2a[j] != B.h2a[j - 1])) heads[idx++] = (uint16_t)j;
  if (t == 0) heads[tot] = (uint16_t)nd;
  __syncthreads();
  for (uint32_t u = t; u < tot; u += 256) {
    it_det[(int64_t)s * nd + u] = B.h2a[heads[u]];
    it_w[(int64_t)s * nd + u] = (uint32_t)(heads[u + 1] - heads[u]);
  }
  if (t == 0) ucount[s] = tot;
}

__global__ void k_sample_compact(const uint32_t* it_det, const uint32_t* it_w, const uint32_t* ucount,
                                 const uint64_t* uoff, int32_t nd, int32_t s0, uint32_t* o_det,
                                 uint32_t* o_w, uint32_t* o_s) {
  const int s = blockIdx.x;
  const uint64_t base = uoff[s];
  for (uint32_t u = threadIdx.x; u < ucount[s]; u += blockDim.x) {
    o_det[base + u] = it_det[(int64_t)s * nd + u];
    o_w[base + u] = it_w[(int64_t)s * nd + u];
    o_s[base + u] = (uint32_t)(s - s0);
  }
}

// Selection of new determinants: flag[i] = 1 if exported unique i meets the
// criterion (HCI: every a reached at the generation threshold; CIPSI:
// |A_a^2 / D_a| > threshold), value[i] = A_a (HCI) or A_a^2 / D_a (CIPSI).
__global__ void k_select_flags(const double* A, const double* D, int64_t n, int mode, double thr, uint32_t* flag,
                               double* value) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double e = A[i] * A[i] / D[i];
    const bool keep = (mode == SHCI_SELECT_HCI) ? true : fabs(e) > thr;
    flag[i] = keep ? 1u : 0u;
    value[i] = (mode == SHCI_SELECT_HCI) ? A[i] : e;
  }
}

__global__ void k_select_compact(const uint64_t* keys, const double* value, const uint32_t* flag,
                                 const uint64_t* pos, int64_t n, uint64_t* out_keys, double* out_val) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    if (!flag[i]) continue;
    const uint64_t o = pos[i];
    for (int w = 0; w < 4; ++w) out_keys[4 * o + w] = keys[4 * i + w];
    out_val[o] = value[i];
  }
}

// Unique export: copy the non-V uniques of every bucket to dense arrays.
template <int KW>
__global__ void k_export_uniq(Uniq U, const int32_t* nseg, const uint64_t* boff, int64_t nb, int n,
                              uint64_t* keys, double* A, double* D, int32_t* cnt, int64_t cap) {
  for (int64_t b = blockIdx.x; b < nb; b += gridDim.x) {
    const uint64_t lo = U.start[b];
    const int ns = nseg[b];
    // non-V uniques before each: sequential scan by thread 0 into the loop below
    uint64_t o = boff[b];
    for (int s = 0; s < ns; ++s) {
      const int32_t c = U.cnt[lo + s];
      if (c < 0) continue;
      if (threadIdx.x == 0 && (int64_t)o < cap) {
        uint64_t k[KW];
#pragma unroll
        for (int w = 0; w < KW; ++w) k[w] = U.k[w][lo + s];
        uint64_t a0, a1, b0, b1;
        unpack_det<KW>(k, n, a0, a1, b0, b1);
        keys[4 * o] = a0;
        keys[4 * o + 1] = a1;
        keys[4 * o + 2] = b0;
        keys[4 * o + 3] = b1;
        A[o] = U.A[lo + s];
        D[o] = U.D[lo + s];
        cnt[o] = c;
      }
      ++o;
    }
  }
}

template <int KW, typename VT>
__global__ void k_export_terms(Recs R, int64_t nrec, int n, uint64_t* keys, uint32_t* idx, double* val,
                               int64_t cap) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < nrec && j < cap;
       j += (int64_t)gridDim.x * blockDim.x) {
    uint64_t k[KW];
#pragma unroll
    for (int w = 0; w < KW; ++w) k[w] = R.k[w][j];
    uint64_t a0, a1, b0, b1;
    unpack_det<KW>(k, n, a0, a1, b0, b1);
    keys[4 * j] = a0;
    keys[4 * j + 1] = a1;
    keys[4 * j + 2] = b0;
    keys[4 * j + 3] = b1;
    idx[j] = R.pay[j];
    val[j] = (double)static_cast<const VT*>(R.v)[j];
  }
}

// number of non-V uniques of every bucket, from the unique store
__global__ void k_nonv_counts(Uniq U, const int32_t* nseg, int64_t nb, uint64_t* out) {
  for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < nb; b += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t lo = U.start[b];
    uint64_t c = 0;
    for (int s = 0; s < nseg[b]; ++s) c += U.cnt[lo + s] > 0;
    out[b] = c;
  }
}

// ----------------------------------------------------------------------------
// One evaluation (deterministic or one chunk of samples)
// ----------------------------------------------------------------------------
// internal status: the records of a job exceed its max_records
constexpr int JOB_TOO_BIG = 1;

struct Job {
  shci_pt2_ctx* ctx;
  hipStream_t st;
  const uint64_t* dets;
  const double* c;
  int64_t ndet;
  double e0, eps2, eps2_d;
  int precision;
  bool sample;
  int sbits;
  int32_t nsamp;   // samples in this chunk
  double nd;       // draws per sample
  double sum_abs;  // device pointer value read by the kernels is passed by value
  // items (sample mode)
  const uint32_t* it_det = nullptr;
  const uint32_t* it_w = nullptr;
  const uint32_t* it_s = nullptr;
  int64_t n_items;
  // options
  bool want_u = false;
  bool want_pay = false;
  double* per_sample = nullptr;  // device [nsamp]
  double* per_sample_de0 = nullptr;  // device [nsamp], nullable: dS_s/dE0
  const uint64_t* samp_off = nullptr;  // host [nsamp + 1]: item range of each sample of the chunk
  double grad_scale = 1.0;             // sample mode: weight of this chunk's adjoint
  Arena* ar = nullptr;           // device memory of the call
  int64_t max_records = 0;       // > 0: give up after the count pass if exceeded
  int64_t max_records_eff = 0;   // on JOB_TOO_BIG: the records that would have fit
  bool keep = false;             // adjoint from the forward records (record positions carried)
  double* contrib = nullptr;     // keep mode: per record t * 2 A_a / D_a (records' generation order)
  uint32_t bmask = 0, bsel = 0;  // hash batch of a
  const int32_t* sbatch = nullptr;  // device: batch of each sample of the chunk (sample mode)
  double sample_scale = 1.0;        // factor on every per-sample result (number of batches)
  bool grad_accumulate = false;  // add this batch's adjoint to grad
  double* grad = nullptr;        // device [ndet]
  shci_pt2_export* ex = nullptr;
  // results
  DevResult res;
  int32_t nbucket = 0, retries = 0;
  float ms_gen = 0, ms_sort = 0, ms_reduce = 0, ms_k_count = 0, ms_k_write = 0, ms_k_reduce = 0, ms_k_part = 0;
  int32_t n_part = 0;
  int64_t n_part_rec = 0;
  int64_t nrec = 0;
  int kw = 0, vbytes = 0;
  int32_t nbatch = 1;
  // singleton split
  int64_t nrec_all = 0;  // kept terms (records or in place)
  int64_t nhash = 0;     // listed hashes (fillers included)
  int64_t nmulti = 0;    // terms written as records
  float ms_k_split = 0;  // hash partition, repeat finder and marks
  Lane* lane = nullptr;  // scratch words, events and estimates (nullptr: the context's own)
};

// Layout of the record region of one pass.
struct BigDims {
  int kw = 0, vsize = 8;
  bool v2 = false, pay = false, want_u = false, keep = false;
  int64_t nrec = 0, nbucket = 1, ntiles = 1;
  int64_t npart = 1;  // per-wavefront partial slots (waves, times the sample slots in sample mode)
  int64_t nqslot = 1536;  // first-level slots of the final sums
  int npass = 0;
};
struct BigPlan {
  Recs A, B;
  uint32_t *hist = nullptr, *hoffs = nullptr;
  ScanTmp hsc;
  Partials P, Pq, Pw;
  Uniq U;
  uint64_t *boff = nullptr, *bst = nullptr;
  uint32_t* slow = nullptr;
  uint32_t* slow_bits = nullptr;  // bitmap of the block kernel's buckets
  double* contrib = nullptr;      // keep mode: per-record adjoint terms
};

template <class CV>
void plan_partials(CV& cv, Partials& P, int64_t m, bool nseg) {
  P.e2 = cv.template take<double>(m);
  P.de0 = cv.template take<double>(m);
  P.e2sq = cv.template take<double>(m);
  P.nterm = cv.template take<int64_t>(m);
  P.ngen = cv.template take<int64_t>(m);
  P.nuniq = cv.template take<int32_t>(m);
  P.nintr = cv.template take<int32_t>(m);
  P.nzero = cv.template take<int32_t>(m);
  P.mind = cv.template take<double>(m);
  P.nseg = nseg ? cv.template take<int32_t>(m) : nullptr;
}

template <class CV>
void plan_recs(CV& cv, Recs& R, const BigDims& d) {
  const int64_t m = d.nrec;
  for (int w = 0; w < d.kw; ++w) R.k[w] = cv.template take<uint64_t>(m);
  R.v = d.vsize == 4 ? (void*)cv.template take<float>(m) : (void*)cv.template take<double>(m);
  R.v2 = d.v2 ? (d.vsize == 4 ? (void*)cv.template take<float>(m) : (void*)cv.template take<double>(m)) : nullptr;
  R.pay = d.pay ? cv.template take<uint32_t>(m) : nullptr;
  R.bid = cv.template take<uint32_t>(m);
  R.haa = cv.template take<double>(m);
}

template <class CV>
void plan_big(CV& cv, const BigDims& d, BigPlan& o) {
  const int64_t nb = d.nbucket;
  plan_recs(cv, o.A, d);
  if (d.npass > 0) plan_recs(cv, o.B, d);
  o.bst = cv.template take<uint64_t>(nb + 1);
  o.slow = cv.template take<uint32_t>(nb + 1);
  o.slow_bits = cv.template take<uint32_t>(nb / 32 + 1);
  o.hist = cv.template take<uint32_t>((size_t)256 * d.ntiles);
  o.hoffs = cv.template take<uint32_t>((size_t)256 * d.ntiles + 1);
  o.hsc.carve(cv, std::max<int64_t>((int64_t)256 * d.ntiles, nb + 1));
  plan_partials(cv, o.P, nb, true);
  plan_partials(cv, o.Pw, d.npart, false);
  plan_partials(cv, o.Pq, d.nqslot, false);
  if (d.want_u) {
    for (int w = 0; w < d.kw; ++w) o.U.k[w] = cv.template take<uint64_t>(d.nrec);
    o.U.h2 = cv.template take<uint32_t>(d.nrec);
    o.U.A = cv.template take<double>(d.nrec);
    o.U.D = cv.template take<double>(d.nrec);
    o.U.g = cv.template take<double>(d.nrec);
    o.U.cnt = cv.template take<int32_t>(d.nrec);
    o.U.start = cv.template take<uint64_t>(nb + 1);
    o.boff = cv.template take<uint64_t>(nb + 1);
  }
  o.contrib = d.keep ? cv.template take<double>(d.nrec) : nullptr;
}

// hash set of V: 2^ceil(log2 2N) slots; presence filter of 2^fbits 64-bit
// words, at least 32 bits per member
void vset_dims(int64_t ndet, uint64_t& vcap, int& fbits, int64_t& fwords) {
  vcap = 1024;
  while (vcap < 2 * (uint64_t)ndet) vcap <<= 1;
  fbits = 8;
  while (fbits < 40 && ((uint64_t)64 << fbits) < 32 * (uint64_t)ndet) ++fbits;
  fwords = (int64_t)1 << fbits;
}

struct Phase0 {  // per source: work split; hash set of V
  uint32_t* nsplit = nullptr;
  uint64_t *soff = nullptr, *vtab = nullptr, *total = nullptr;
  uint64_t* vfilt = nullptr;
  ScanTmp sc0;
};
template <class CV>
void plan_phase0(CV& cv, Phase0& p, int64_t nsrc, uint64_t vcap, int64_t fwords) {
  p.nsplit = cv.template take<uint32_t>(nsrc + 1);
  p.soff = cv.template take<uint64_t>(nsrc + 1);
  p.vtab = cv.template take<uint64_t>(vcap);
  p.vfilt = cv.template take<uint64_t>(fwords);
  p.total = cv.template take<uint64_t>(4);
  p.sc0.carve(cv, nsrc + 1);
}

struct Phase1 {  // per work item: source, pair range, count, offset, adjoint parts
  uint32_t *w_src = nullptr, *w_rng = nullptr, *counts = nullptr;
  uint64_t* offs = nullptr;
  double *gpart = nullptr, *gitem = nullptr;
  ScanTmp sc;
};
template <class CV>
void plan_phase1(CV& cv, Phase1& p, int64_t ni, int64_t nsrc, bool grad, bool sample) {
  p.w_src = cv.template take<uint32_t>(ni + 1);
  p.w_rng = cv.template take<uint32_t>(ni + 1);
  p.counts = cv.template take<uint32_t>(ni + 1);
  p.offs = cv.template take<uint64_t>(ni + 1);
  p.gpart = grad ? cv.template take<double>(ni + 1) : nullptr;
  p.gitem = (grad && sample) ? cv.template take<double>(nsrc + 1) : nullptr;
  p.sc.carve(cv, ni + 1);
}

// ---- singleton split (hashsplit.hpp) ----
// the list takes 12 bytes a slot, twice (partition), plus the filter (at
// most half a byte a slot), tile histograms and bucket bounds
constexpr double HASH_BYTES_PER_ENTRY = 25.5;
// SHCI_GROUP_AUTO: a deterministic pass with fewer kept terms groups them all
// as records (measured: 6.4e6 terms 2.1 ms as records against 3.8 ms split;
// 4.9e7 terms 43 ms against 45 ms); sampling passes always split
constexpr int64_t SPLIT_MIN_DET_TERMS = 100000000;
constexpr uint64_t HASH_CAP = (uint64_t)1000000000;  // slots of one list

struct SplitPlan {
  int64_t ni = 0;
  uint32_t* mcount = nullptr;  // [ni + 1] terms of each work item written as records
  uint64_t* moffs = nullptr;   // [ni + 1] their exclusive scan, moffs[ni] = total
  ScanTmp msc;
  Partials PI;                 // [ni] in-place sums of each work item
  uint64_t* ib = nullptr;      // [nsamp + 1] sample mode: first work item of each sample
  uint64_t* filt = nullptr;    // filter of repeated hashes: fwords_max words, 2^fbits in use
  uint64_t fwords_max = 0;
  int fbits = 0;
};
template <class CV>
void plan_split(CV& cv, SplitPlan& p, int64_t ni, int32_t nsamp) {
  p.ni = ni;
  p.mcount = cv.template take<uint32_t>(ni + 1);
  p.moffs = cv.template take<uint64_t>(ni + 1);
  p.msc.carve(cv, ni + 1);
  plan_partials(cv, p.PI, std::max<int64_t>(ni, 1), false);
  p.ib = cv.template take<uint64_t>((int64_t)nsamp + 2);
}
struct HashList {
  uint64_t* k = nullptr;
  uint32_t* i = nullptr;
};
template <class CV>
void plan_hash_list(CV& cv, HashList& h, int64_t n) {
  h.k = cv.template take<uint64_t>(std::max<int64_t>(n, 1));
  h.i = cv.template take<uint32_t>(std::max<int64_t>(n, 1));
}

// the split needs no per-a output: no unique store, no records kept for an
// adjoint or an export
bool split_allowed(const Job& J) {
  return J.ctx->grouping != SHCI_GROUP_RECORDS && !J.want_u && !J.want_pay && !J.keep && !J.grad;
}

// list slots the memory allows: what the caller workspace has left, or a
// share of free device memory (plus the context's list buffers)
int64_t split_budget(const Arena& A) {
  shci_pt2_ctx* X = A.X;
  double avail;
  if (A.caller()) {
    const double r = (double)A.remaining() - (double)(64u << 20);
    avail = r > 0 ? r : 0.0;
  } else {
    size_t fr = 0, tt = 0;
    if (hipMemGetInfo(&fr, &tt) != hipSuccess) {
      (void)hipGetLastError();
      fr = 0;
    }
    double a = (double)fr + (double)A.L->slot[SL_FILT].cap + (double)A.L->slot[SL_HASH].cap +
               (double)A.L->slot[SL_HASH2].cap;
    if (X->ws_limit) a = std::min(a, (double)X->ws_limit);
    avail = 0.6 * a;
  }
  return (int64_t)(avail / HASH_BYTES_PER_ENTRY);
}

// Partition of the hash list, repeated hashes into the filter, marks per
// work item and their scan; J.nmulti = terms that become records.
int find_repeats(Job& J, SplitPlan& SP, HashList& HL, int64_t nent, hipStream_t st, int cus) {
  shci_pt2_ctx* X = J.ctx;
  Lane& R = J.lane ? *J.lane : *X;
  Arena& AR = *J.ar;
  // buckets of ~12k hashes (one LDS table fill each): 16 bits, two passes,
  // up to ~8e8 hashes.  The bits follow the number of listed terms, not the
  // list's length (its fillers depend on the run sizes, which follow earlier
  // calls): the hashes that share a bucket and a tag, which the filter takes
  // as repeated, then depend on the hashes alone.
  const int64_t nreal = std::max<int64_t>(1, J.nrec_all);
  const int64_t per = X->split_bucket;
  const int nbits = std::min(30, std::max(1, ceil_log2((uint64_t)((nreal + per - 1) / per))));
  const int npass = (nbits + 7) / 8;
  const int64_t nbucket = (int64_t)1 << nbits;
  const int64_t ntiles = std::max<int64_t>(1, (nent + PTILE - 1) / PTILE);
  HashList HB;
  uint32_t *hist = nullptr, *hoffs = nullptr;
  ScanTmp hsc;
  uint64_t* bst = nullptr;
  CHK(carve_region(AR, SL_HASH2, [&](Carver& cv) {
    plan_hash_list(cv, HB, nent);
    hist = cv.take<uint32_t>((size_t)256 * ntiles);
    hoffs = cv.take<uint32_t>((size_t)256 * ntiles + 1);
    hsc.carve(cv, (int64_t)256 * ntiles);
    bst = cv.take<uint64_t>(nbucket + 1);
  }));
  HIPCHK(hipEventRecord(R.evh[0], st));
  HashList* cur = &HL;
  HashList* oth = &HB;
  int shift = 0;
  const int pgrid = (int)(8 * ((ntiles + 7) / 8));
  for (int pass = 0; pass < npass; ++pass) {
    const int dbits = nbits / npass + (pass < nbits % npass ? 1 : 0);
    HPassArgs pa{};
    pa.kin = cur->k;
    pa.iin = cur->i;
    pa.kout = oth->k;
    pa.iout = oth->i;
    pa.n = nent;
    pa.nbits = nbits;
    pa.shift = shift;
    pa.dbits = dbits;
    pa.hist = hist;
    pa.offs = hoffs;
    pa.ntiles = (int)ntiles;
    k_hpart_hist<<<pgrid, 256, 0, st>>>(pa);
    CHK(scan_exclusive<uint32_t, uint32_t>(hist, hoffs, ((int64_t)1 << dbits) * ntiles, hsc, nullptr, st));
    if (pass == 0)
      k_hpart_scatter_first<<<pgrid, PTHREADS, 0, st>>>(pa);
    else
      k_hpart_scatter<<<pgrid, PTHREADS, 0, st>>>(pa);
    HIPCHK(hipGetLastError());
    std::swap(cur, oth);
    shift += dbits;
  }
  k_hbounds<<<(int)((nbucket + 256) / 256), 256, 0, st>>>(cur->k, nent, nbits, nbucket, bst);
  // filter of 32-64 bits per repeated hash: its size is a function of the
  // number of repeated hashes (so the records, and the sums, do not depend on
  // an earlier call); first guessed from the last job's rate, then again if
  // the guess was not that size
  const int sidx = J.sample ? 1 : 0;
  // at most ~4 bits per kept term (a cap that depends on the terms only)
  uint64_t wcap = 1024;
  while (wcap < SP.fwords_max && (double)wcap * 16.0 < (double)J.nrec_all) wcap <<= 1;
  auto words_for = [&](double rep) {
    uint64_t w = 1024;
    while (w < wcap && (double)w * 2.0 < rep) w <<= 1;
    return w;
  };
  uint64_t words = words_for(R.split_rep[sidx] * (double)nent);
  const int64_t dblocks = std::min<int64_t>(nbucket, (int64_t)cus * 4);
  unsigned long long nrep = 0;
  for (int attempt = 0;; ++attempt) {
    const int fbits = ceil_log2(words);
    k_fill_u64<<<(int)std::min<int64_t>(4096, ((int64_t)words + 255) / 256), 256, 0, st>>>(SP.filt, (int64_t)words,
                                                                                           0ull);
    k_fill_u64<<<1, 64, 0, st>>>(reinterpret_cast<uint64_t*>(R.dctr + 1), 1, 0ull);
    HDupArgs da{};
    da.g = cur->k;
    da.bstart = bst;
    da.n = nent;
    da.nbits = nbits;
    da.nbucket = nbucket;
    da.filt = SP.filt;
    da.fbits = fbits;
    da.nrep = R.dctr + 1;
    k_hdup<<<(int)dblocks, HDUP_THREADS, 0, st>>>(da);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(&nrep, R.dctr + 1, sizeof nrep, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    SP.fbits = fbits;
    const uint64_t want = words_for((double)nrep);
    if (want != words && attempt == 0) {
      words = want;
      continue;
    }
    break;
  }
  R.split_rep[sidx] = nent > 0 ? (double)nrep / (double)nent : 0.0;
  k_fill_u32<<<(int)std::min<int64_t>(4096, (SP.ni + 256) / 256), 256, 0, st>>>(SP.mcount, SP.ni + 1, 0u);
  k_hmark<<<(int)std::min<int64_t>(8192, (nent + 255) / 256 + 1), 256, 0, st>>>(cur->k, cur->i, nent, SP.filt,
                                                                                SP.fbits, SP.mcount);
  CHK(scan_exclusive<uint32_t, uint64_t>(SP.mcount, SP.moffs, SP.ni, SP.msc, SP.moffs + SP.ni, st));
  HIPCHK(hipEventRecord(R.evh[1], st));
  HIPCHK(hipGetLastError());
  uint64_t nm = 0;
  HIPCHK(hipMemcpyAsync(&nm, SP.moffs + SP.ni, sizeof nm, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  J.nmulti = (int64_t)nm;
  float ms = 0;
  HIPCHK(hipEventElapsedTime(&ms, R.evh[0], R.evh[1]));
  J.ms_k_split = ms;
  return SHCI_OK;
}

template <int KW, typename VT, bool SAMPLE>
int run_job(Job& J) {
  shci_pt2_ctx* X = J.ctx;
  Lane& R = J.lane ? *J.lane : *X;
  const Tables& T = X->T;
  const int n = T.n;
  hipStream_t st = J.st;
  constexpr int C = (KW <= 2) ? 2048 : 1024;
  const int auxbit = 2 * n + J.sbits;
  const int cus = num_cus(X->device);

  // ---- phase 0: validation, hash set of V, work split per source ----
  const int64_t nsrc = J.n_items;
  uint64_t vcap;
  int fbits;
  int64_t fwords;
  vset_dims(J.ndet, vcap, fbits, fwords);
  Phase0 p0;
  Arena& AR = *J.ar;
  const size_t job_mark = AR.mark();
  CHK(carve_region(AR, SL_V, [&](Carver& cv) { plan_phase0(cv, p0, nsrc, vcap, fwords); }));
  uint32_t* nsplit = p0.nsplit;
  uint64_t *soff = p0.soff, *vtab = p0.vtab, *total = p0.total;
  uint64_t* vfilt = p0.vfilt;
  ScanTmp& sc0 = p0.sc0;
  uint32_t* dflag = R.dflag;
  uint32_t* counter = R.dflag + 1;
  uint32_t* overflow = R.dflag + 2;

  HIPCHK(hipEventRecord(R.ev[0], st));
  k_fill_u32<<<1, 64, 0, st>>>(dflag, 4, 0u);
  k_validate<<<(int)((J.ndet + 255) / 256), 256, 0, st>>>(J.dets, J.c, J.ndet, n, T.na, T.nb, dflag);
  VSet V;
  V.tab = vtab;
  V.mask = vcap - 1;
  V.filt = vfilt;
  V.fbits = fbits;
  k_fill_u64<<<(int)std::min<int64_t>(4096, (fwords + 255) / 256), 256, 0, st>>>(vfilt, fwords, 0ull);
  V.dets = J.dets;
  k_fill_u64<<<std::min<int64_t>(4096, (vcap + 255) / 256), 256, 0, st>>>(vtab, (int64_t)vcap, ~0ull);
  k_vset_insert<KW><<<(int)((J.ndet + 255) / 256), 256, 0, st>>>(V, J.ndet, n, dflag);
  const int npairs = T.na * (T.na - 1) / 2 + T.nb * (T.nb - 1) / 2 + T.na * T.nb;
  {
    SplitArgs sa{};
    sa.n = n;
    sa.na = T.na;
    sa.nb = T.nb;
    sa.nss = T.nss;
    sa.lss = T.lss;
    sa.los = T.los;
    sa.c = J.c;
    sa.it_det = J.it_det;
    sa.n_src = nsrc;
    sa.eps2 = J.eps2;
    sa.mag_cum = T.mag_cum;
    sa.nsplit = nsplit;
    k_split_count<<<(int)((nsrc + 255) / 256), 256, 0, st>>>(sa);
  }
  CHK(scan_exclusive<uint32_t, uint64_t>(nsplit, soff, nsrc, sc0, total, st));
  uint64_t hostv[2] = {0, 0};
  uint32_t hflags = 0;
  HIPCHK(hipMemcpyAsync(hostv, total, sizeof(uint64_t), hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(&hflags, dflag, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (hflags & 1u) return fail(SHCI_ERR_DET, "a determinant has a wrong electron count or an orbital >= n_orb");
  if (hflags & 2u) return fail(SHCI_ERR_NONFINITE, "c contains a non-finite value");
  if (hflags & 4u) return fail(SHCI_ERR_DUP, "the variational space contains a duplicate determinant");
  if (hflags & 8u) return fail(SHCI_ERR_WORKSPACE, "hash set of V overflowed");
  const int64_t ni = (int64_t)hostv[0];  // work items
  if (ni >= (int64_t)0xffffffffll) return fail(SHCI_ERR_WORKSPACE, "too many work items");

  // ---- phase 1: work items, count pass ----
  Phase1 p1;
  CHK(carve_region(AR, SL_ITEMS, [&](Carver& cv) { plan_phase1(cv, p1, ni, nsrc, J.grad != nullptr, SAMPLE); }));
  uint32_t *w_src = p1.w_src, *w_rng = p1.w_rng, *counts = p1.counts;
  uint64_t* offs = p1.offs;
  double* gpart = p1.gpart;
  double* gitem = p1.gitem;  // sample mode: adjoint per item before the scatter to determinants
  ScanTmp& sc = p1.sc;
  k_split_fill<<<(int)((nsrc + 255) / 256), 256, 0, st>>>(nsplit, soff, nsrc, npairs, w_src, w_rng);

  GenArgs g{};
  g.n = n;
  g.na = T.na;
  g.nb = T.nb;
  g.dets = J.dets;
  g.c = J.c;
  g.n_items = ni;
  g.w_src = w_src;
  g.w_rng = w_rng;
  g.it_det = J.it_det;
  g.it_w = J.it_w;
  g.it_s = J.it_s;
  g.sum_abs = J.sum_abs;
  g.nd = J.nd;
  g.eps2 = J.eps2;
  g.eps2_d = J.eps2_d;
  g.T = T;
  g.counts = counts;
  g.offs = offs;
  g.flag = dflag;
  g.counter = counter;
  g.sbits = J.sbits;
  g.auxbit = auxbit;
  g.bmask = J.bmask;
  g.bsel = J.bsel;
  g.sbatch = J.sbatch;
  g.ref = J.dets;
  g.Fref = T.fref;
  g.smarg = 8.0 * (2 * n + 2 + 2 * DL_CAP) * 0x1p-53;
  g.pay_pos = J.keep ? 1 : 0;
  singles_ref(T, J.dets, st);
  const int gen_grid = cus * GEN_BLOCKS_PER_CU;
  const int64_t gen_waves = (int64_t)gen_grid * 4;

  // ---- count walk; with the singleton split it also lists the grouping
  // hashes (hashsplit.hpp) ----
  bool split = split_allowed(J);
  const bool split0 = split;
  SplitPlan SP;
  HashList HL;
  uint64_t hcap = 0;
  double& rate = R.split_rate[SAMPLE ? 1 : 0];  // kept terms per work item, last job that could split
  // runs of 64 to 512 slots (a run must take one emission of up to 64
  // terms), shorter for fewer terms: the unused tails of the runs (at most
  // one per wavefront) are partitioned too
  double run_terms = 0.0;  // expected terms, for the run length
  auto pick_run = [&](double terms) {
    int r = 512;
    while (r > 64 && (double)r * (double)gen_waves * 16.0 > terms) r >>= 1;
    return r;
  };
  if (split) {
    CHK(carve_region(AR, SL_SPLIT, [&](Carver& cv) { plan_split(cv, SP, ni, J.nsamp); }));
    // list capacity: what the caller workspace has left, or (context memory)
    // an estimate from the last job of this kind; none: a plain count first
    const uint64_t lim = std::min<uint64_t>(HASH_CAP, (uint64_t)split_budget(AR));
    run_terms = rate > 0.0 ? 1.3 * rate * (double)ni : (double)lim;
    if (AR.caller())
      hcap = lim;
    else if (rate > 0.0)
      hcap = std::min<uint64_t>(lim, (uint64_t)run_terms + (uint64_t)gen_waves * (uint64_t)pick_run(run_terms));
  }
  int hrun = 0;
  size_t list_mark = 0;
  auto count_walk = [&](bool list) -> int {
    hrun = 0;
    g.hkey = nullptr;
    g.hitem = nullptr;
    g.hcap = 0;
    if (list) {
      hrun = pick_run(std::min((double)hcap, run_terms));
      // the filter (kept for the write walk), then the list
      uint64_t fw = 1024;
      while (fw < ((uint64_t)1 << 27) && fw * 16 < hcap) fw <<= 1;
      SP.fwords_max = fw;
      CHK(carve_region(AR, SL_FILT, [&](Carver& cv) { SP.filt = cv.take<uint64_t>(fw); }));
      list_mark = AR.mark();
      CHK(carve_region(AR, SL_HASH, [&](Carver& cv) { plan_hash_list(cv, HL, (int64_t)hcap); }));
      g.hkey = HL.k;
      g.hitem = HL.i;
      g.hcap = hcap;
      g.hclaim = R.dctr;
      g.hrun = hrun;
    }
    k_fill_u32<<<1, 64, 0, st>>>(counter, 1, 0u);
    k_fill_u64<<<1, 64, 0, st>>>(reinterpret_cast<uint64_t*>(R.dctr), 4, 0ull);
    HIPCHK(hipEventRecord(R.ev[4], st));
    k_gen_count<KW, SAMPLE, VT><<<gen_grid, 256, 0, st>>>(g);
    HIPCHK(hipEventRecord(R.ev[5], st));
    HIPCHK(hipGetLastError());
    // offs[ni] = total: the write walk checks every item's end against it
    CHK(scan_exclusive<uint32_t, uint64_t>(counts, offs, ni, sc, offs + ni, st));
    HIPCHK(hipMemcpyAsync(hostv, offs + ni, sizeof(uint64_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(hostv + 1, R.dctr, sizeof(uint64_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return SHCI_OK;
  };
  const size_t hash_mark = AR.mark();
  bool counted = false;
  // "auto" groups a small deterministic pass as records (decided on the exact
  // count): when the last pass of this kind was small, count first without
  // the list
  const bool det_auto = !SAMPLE && X->grouping == SHCI_GROUP_AUTO;
  const bool guess_small = det_auto && rate > 0.0 && rate * (double)ni < 0.5 * (double)SPLIT_MIN_DET_TERMS;
  if (split && (hcap == 0 || guess_small)) {
    // no estimate yet (or a small pass expected): count first, then size the
    // list for every term
    CHK(count_walk(false));
    counted = true;
    if (det_auto && hostv[0] < (uint64_t)SPLIT_MIN_DET_TERMS) {
      split = false;
    } else {
      run_terms = (double)hostv[0];
      hcap = std::min<uint64_t>(std::min<uint64_t>(HASH_CAP, (uint64_t)split_budget(AR)),
                                hostv[0] + (uint64_t)gen_waves * (uint64_t)pick_run(run_terms));
    }
  }
  // a caller workspace with too little room for a list of runs of 64 slots:
  // every term becomes a record
  if (split && AR.caller() && hcap < (uint64_t)gen_waves * 64 * 2) split = false;
  if (split) {
    CHK(count_walk(true));
    counted = true;
    if (hostv[1] > hcap && !AR.caller() && hcap < HASH_CAP) {
      // the estimate was short: list again with room for every term
      AR.reset(hash_mark);
      run_terms = (double)hostv[0];
      hcap = std::min<uint64_t>(std::min<uint64_t>(HASH_CAP, (uint64_t)split_budget(AR)),
                                hostv[0] + (uint64_t)gen_waves * (uint64_t)pick_run(run_terms));
      CHK(count_walk(true));
    }
  }
  if (!counted) CHK(count_walk(false));
  const int64_t nrec_all = (int64_t)hostv[0];
  if (split && det_auto && nrec_all < SPLIT_MIN_DET_TERMS) {
    // a small deterministic pass: every term a record (the counts per work
    // item are the same; the list is dropped)
    split = false;
    AR.reset(hash_mark);
  }
  if (split0 && ni > 0) rate = std::max(1.0, (double)nrec_all / (double)ni);
  const int64_t lim_rec = split ? X->rec_limit : J.max_records;
  if (lim_rec > 0 && nrec_all > lim_rec) {
    J.nrec = nrec_all;
    J.max_records_eff = lim_rec;
    AR.reset(job_mark);
    return JOB_TOO_BIG;
  }
  int64_t nrec = nrec_all;
  J.nrec_all = nrec_all;
  J.nhash = 0;
  J.ms_k_split = 0;
  if (split) {
    const uint64_t nent = hostv[1];
    if (nent > hcap) {
      // the list did not fit: hash batches or smaller sample chunks, sized
      // by the terms that would have fit
      J.nrec = nrec_all;
      J.max_records_eff = std::max<int64_t>(1, (int64_t)hcap - gen_waves * hrun);
      AR.reset(job_mark);
      return JOB_TOO_BIG;
    }
    CHK(find_repeats(J, SP, HL, (int64_t)nent, st, cus));
    nrec = J.nmulti;
    J.nhash = (int64_t)nent;
    // the hash list is not read again: the records take its memory
    AR.reset(list_mark);
    g.offs = SP.moffs;
    g.mfilt = SP.filt;
    g.mfbits = SP.fbits;
    g.V = V;
    g.e0 = J.e0;
    g.inv_ndd = SAMPLE ? 1.0 / (J.nd * (J.nd - 1.0)) : 0.0;
    g.PI = SP.PI;
  }
  if (nrec >= (int64_t)0xffffffffll)
    return fail(SHCI_ERR_WORKSPACE, "%lld screened terms exceed the 2^32-1 records of one pass", (long long)nrec);

  // ---- plan the grouping ----
  GroupPlan G;
  G.sbits = J.sbits;
  {
    // buckets of 64-128 records on average; one more hash bit (32-64) when
    // it costs no extra partition pass: smaller buckets sort in fewer
    // register slots in the reduce
    const int64_t per_sample_rec = SAMPLE ? std::max<int64_t>(1, nrec / std::max(1, J.nsamp)) : nrec;
    G.bits_hash = std::min(26, std::max(0, ceil_log2((uint64_t)((per_sample_rec + 127) / 128))));
    const int nb0 = G.bits_hash + G.sbits;
    if (G.bits_hash < 26 && per_sample_rec >= ((int64_t)64 << G.bits_hash) && (nb0 + 1 + 7) / 8 == (nb0 + 7) / 8)
      G.bits_hash += 1;
  }

  const size_t big_mark = AR.mark();
  for (int attempt = 0;; ++attempt) {
    AR.reset(big_mark);
    G.nbits = G.bits_hash + G.sbits;
    G.nbucket = (int64_t)1 << G.nbits;
    const int npass = (G.nbits + 7) / 8;
    const int64_t ntiles = std::max<int64_t>(1, (nrec + PTILE - 1) / PTILE);
    const bool v2 = SAMPLE;
    const bool pay = J.want_pay || J.keep;
    BigDims bd;
    bd.kw = KW;
    bd.vsize = (int)sizeof(VT);
    bd.v2 = v2;
    bd.pay = pay;
    bd.want_u = J.want_u;
    bd.keep = J.keep;
    bd.nrec = nrec;
    bd.nbucket = G.nbucket;
    bd.ntiles = ntiles;
    bd.npass = npass;
    // reduce launch: wavefronts, and the sample slots of the chunk's key bits
    const int64_t wblocks =
        std::min<int64_t>((G.nbucket + WRED_WAVES - 1) / WRED_WAVES, (int64_t)cus * RED_BLOCKS_PER_CU);
    const int64_t nwv = wblocks * WRED_WAVES;
    const int64_t nslots = SAMPLE ? ((int64_t)1 << G.sbits) : 1;
    bd.npart = nwv * nslots;
    bd.nqslot = std::max<int64_t>(1536, nslots);
    BigPlan BP;
    if (AR.caller()) {
      // the records must fit what the workspace has left; otherwise report
      // how many would have fit (hash batches / smaller sample chunks)
      Carver cv(nullptr);
      plan_big(cv, bd, BP);
      if (cv.off > AR.remaining()) {
        J.nrec = nrec;
        J.max_records_eff = std::max<int64_t>(
            1, (int64_t)(0.95 * (double)nrec * (double)AR.remaining() / (double)cv.off));
        AR.reset(job_mark);
        return JOB_TOO_BIG;
      }
    }
    CHK(carve_region(AR, SL_REC, [&](Carver& cv) { plan_big(cv, bd, BP); }));
    Recs& A = BP.A;
    Recs& B = BP.B;
    uint32_t* hist = BP.hist;
    uint32_t* hoffs = BP.hoffs;
    ScanTmp& hsc = BP.hsc;
    Partials& P = BP.P;
    Partials& Pq = BP.Pq;
    Partials& Pw = BP.Pw;
    Uniq& U = BP.U;
    uint64_t* boff = BP.boff;
    uint64_t* bst = BP.bst;
    uint32_t* slow = BP.slow;
    {
      // ---- generation (write pass; repeated after a re-plan, same records) ----
      g.out = A;
      g.bits_hash = G.bits_hash;
      k_fill_u32<<<1, 64, 0, st>>>(counter, 1, 0u);
      HIPCHK(hipEventRecord(R.ev[6], st));
      if constexpr (SAMPLE)
        k_gen_write_sample<KW, VT><<<gen_grid, 256, 0, st>>>(g);
      else
        k_gen_write<KW, VT><<<gen_grid, 256, 0, st>>>(g);
      HIPCHK(hipEventRecord(R.ev[7], st));
      HIPCHK(hipGetLastError());
      if (J.ex && J.ex->t_keys && J.ex->t_cap > 0 && pay) {
        k_export_terms<KW, VT><<<1024, 256, 0, st>>>(A, nrec, n, J.ex->t_keys, J.ex->t_i, J.ex->t_val,
                                                      J.ex->t_cap);
      }
    }
    HIPCHK(hipEventRecord(R.ev[1], st));
    // ---- hash partition (LSD over the bucket id) ----
    Recs* cur = &A;
    Recs* oth = &B;
    {
      int shift = 0;
      for (int pass = 0; pass < npass; ++pass) {
        const int dbits = G.nbits / npass + (pass < G.nbits % npass ? 1 : 0);
        PassArgs pa{};
        pa.in = *cur;
        pa.out = *oth;
        pa.n = nrec;
        pa.G = G;
        pa.nbits_n = n;
        pa.auxbit = auxbit;
        pa.shift = shift;
        pa.dbits = dbits;
        pa.hist = hist;
        pa.offs = hoffs;
        pa.ntiles = (int)ntiles;
        const int pgrid = (int)(8 * ((ntiles + 7) / 8));
        k_part_hist<KW><<<pgrid, 256, 0, st>>>(pa);
        CHK(scan_exclusive<uint32_t, uint32_t>(hist, hoffs, ((int64_t)1 << dbits) * ntiles, hsc, nullptr, st));
        if (pass < 8) HIPCHK(hipEventRecord(R.evp[2 * pass], st));
        if (pay)
          k_part_scatter<KW, VT, SAMPLE, true><<<pgrid, PTHREADS, 0, st>>>(pa);
        else
          k_part_scatter<KW, VT, SAMPLE, false><<<pgrid, PTHREADS, 0, st>>>(pa);
        if (pass < 8) HIPCHK(hipEventRecord(R.evp[2 * pass + 1], st));
        HIPCHK(hipGetLastError());
        std::swap(cur, oth);
        shift += dbits;
      }
    }
    if (npass > 0) {
      const int64_t m = nrec + 1;
      k_bucket_bounds<<<(int)std::min<int64_t>(8192, (m + 255) / 256), 256, 0, st>>>(cur->bid, nrec, G.nbucket, bst);
    } else {
      const uint64_t hb[2] = {0, (uint64_t)nrec};
      HIPCHK(hipMemcpyAsync(bst, hb, sizeof hb, hipMemcpyHostToDevice, st));
    }
    HIPCHK(hipEventRecord(R.ev[2], st));
    // ---- bucket reduce ----
    RedArgs ra{};
    ra.in = *cur;
    ra.nrec = nrec;
    ra.G = G;
    ra.n = n;
    ra.auxbit = auxbit;
    ra.e0 = J.e0;
    ra.nd = J.nd;
    ra.V = V;
    ra.P = P;
    ra.U = U;
    ra.overflow = overflow;
    ra.want_u = J.want_u ? 1 : 0;
    ra.bstart = bst;
    ra.contrib = (J.keep && !SAMPLE) ? BP.contrib : nullptr;
    uint32_t* slow_count = R.dflag + 3;
    WaveRedArgs wa;
    wa.r = ra;
    wa.bstart = bst;
    wa.slow_list = slow;
    wa.slow_count = slow_count;
    wa.slow_bits = BP.slow_bits;
    wa.Pw = Pw;
    wa.nwaves = nwv;
    wa.nsamp = (int32_t)nslots;
    k_fill_u32<<<1, 64, 0, st>>>(overflow, 1, 0u);
    k_fill_u32<<<1, 64, 0, st>>>(slow_count, 1, 0u);
    {
      const int64_t nw = G.nbucket / 32 + 1;
      k_fill_u32<<<(int)std::min<int64_t>(4096, (nw + 255) / 256), 256, 0, st>>>(BP.slow_bits, nw, 0u);
    }
    HIPCHK(hipEventRecord(R.ev[8], st));
    k_reduce_wave<KW, SAMPLE, VT><<<(int)wblocks, 64 * WRED_WAVES, 0, st>>>(wa);
    // buckets the wavefront kernel could not take: block kernel with a full-key sort
    ra.blist = slow;
    ra.nlist = slow_count;
    {
      const int rgrid = (int)std::min<int64_t>(G.nbucket, (int64_t)cus * 2);
      k_reduce<KW, C, SAMPLE, VT><<<rgrid, 256, 0, st>>>(ra);
    }
    HIPCHK(hipEventRecord(R.ev[9], st));
    HIPCHK(hipGetLastError());
    k_zero_result<<<1, 1, 0, st>>>(R.dres);
    if (SAMPLE) {
      if (split)
        k_item_bounds<<<(J.nsamp + 256) / 256, 256, 0, st>>>(w_src, J.it_s, ni, J.nsamp, SP.ib);
      // slices per sample: up to 32, within the 1536 slots of Pq
      const int gs = (int)std::max<int64_t>(1, std::min<int64_t>(32, 1536 / std::max<int32_t>(1, J.nsamp)));
      k_final_sample_part<<<J.nsamp * gs, 256, 0, st>>>(Pw, nwv, P, BP.slow_bits, G.bits_hash, SP.PI,
                                                          split ? SP.ib : nullptr, gs, Pq);
      k_final_sample_sum<<<(J.nsamp + 255) / 256, 256, 0, st>>>(Pq, gs, J.nsamp, R.dres, J.per_sample,
                                                                 J.per_sample_de0, J.sample_scale);
    } else {
      // the block kernel's bucket partials (through the bitmap, in bucket
      // order) and the per-wavefront partials, summed in a fixed order
      const int64_t fchunk = std::max<int64_t>(8192, ((G.nbucket + 511) / 512 + 31) / 32 * 32);
      const int64_t fblocks = (G.nbucket + fchunk - 1) / fchunk;
      const int64_t wchunk = std::max<int64_t>(256, (nwv + 511) / 512);
      const int64_t wfblocks = (nwv + wchunk - 1) / wchunk;
      Partials Q = Pq, Q2 = Pq;
      Q2.e2 += fblocks; Q2.de0 += fblocks; Q2.e2sq += fblocks; Q2.nterm += fblocks; Q2.ngen += fblocks;
      Q2.nuniq += fblocks; Q2.nintr += fblocks; Q2.nzero += fblocks; Q2.mind += fblocks;
      k_final_partial_marked<<<(int)fblocks, 256, 0, st>>>(P, BP.slow_bits, G.nbucket, fchunk, Q);
      k_final_partial<<<(int)wfblocks, 256, 0, st>>>(Pw, nwv, wchunk, Q2);
      // and the in-place partials of the work items (singleton split)
      int64_t ifblocks = 0;
      if (split && ni > 0) {
        const int64_t ichunk = std::max<int64_t>(4096, ((ni + 255) / 256 + 31) / 32 * 32);
        ifblocks = (ni + ichunk - 1) / ichunk;
        Partials Q3 = Pq;
        const int64_t o3 = fblocks + wfblocks;
        Q3.e2 += o3; Q3.de0 += o3; Q3.e2sq += o3; Q3.nterm += o3; Q3.ngen += o3;
        Q3.nuniq += o3; Q3.nintr += o3; Q3.nzero += o3; Q3.mind += o3;
        k_final_partial<<<(int)ifblocks, 256, 0, st>>>(SP.PI, ni, ichunk, Q3);
      }
      k_final<<<1, 1024, 0, st>>>(Q, fblocks + wfblocks + ifblocks, 0, 1, overflow, dflag, R.dres, nullptr, 0,
                                   nullptr, 1.0);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipEventRecord(R.ev[3], st));
    uint32_t hov = 0;
    HIPCHK(hipMemcpyAsync(&J.res, R.dres, sizeof(DevResult), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(&hov, overflow, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (J.res.flags & 32u)
      return fail(SHCI_ERR_HIP, "internal error: the write walk kept a different number of terms than the count walk");
    if (hov) {
      // a bucket held more records than fit in LDS: plan again with one more
      // hash bit; the write pass regenerates the same records
      if (G.bits_hash >= 30 || attempt >= 6)
        return fail(SHCI_ERR_WORKSPACE, "a perturbative determinant has more kept terms than one bucket holds");
      G.bits_hash += 1;
      J.retries++;
      continue;
    }
    float ms;
    HIPCHK(hipEventElapsedTime(&ms, R.ev[0], R.ev[1]));
    J.ms_gen = ms;
    HIPCHK(hipEventElapsedTime(&ms, R.ev[1], R.ev[2]));
    J.ms_sort = ms;
    HIPCHK(hipEventElapsedTime(&ms, R.ev[2], R.ev[3]));
    J.ms_reduce = ms;
    HIPCHK(hipEventElapsedTime(&ms, R.ev[4], R.ev[5]));
    J.ms_k_count = ms;
    HIPCHK(hipEventElapsedTime(&ms, R.ev[6], R.ev[7]));
    J.ms_k_write = ms;
    HIPCHK(hipEventElapsedTime(&ms, R.ev[8], R.ev[9]));
    J.ms_k_reduce = ms;
    J.ms_k_part = 0;
    for (int p = 0; p < std::min(npass, 8); ++p) {
      HIPCHK(hipEventElapsedTime(&ms, R.evp[2 * p], R.evp[2 * p + 1]));
      J.ms_k_part += ms;
    }
    J.n_part = npass;
    J.n_part_rec = nrec * npass;
    J.nrec = nrec;
    if (!split) J.nmulti = nrec;
    J.kw = KW;
    J.vbytes = (int)sizeof(VT) * (SAMPLE ? 2 : 1);
    J.nbucket = (int32_t)G.nbucket;

    if (J.keep && J.grad && !SAMPLE) {
      // adjoint from the forward records: per work item, the sum of its
      // records' t * 2 A_a / D_a; per source, divided by c_i
      k_keep_item_sum<<<(int)((ni + 3) / 4), 256, 0, st>>>(offs, ni, BP.contrib, gpart);
      k_grad_sum<<<(int)((nsrc + 255) / 256), 256, 0, st>>>(nsplit, soff, gpart, nsrc, J.grad,
                                                              J.grad_accumulate ? 1 : 0, J.c);
      HIPCHK(hipGetLastError());
    } else if (J.want_u && J.grad) {
      LookupArgs L;
      L.U = U;
      L.nseg = P.nseg;
      L.G = G;
      g.L = L;
      g.grad = gpart;
      k_fill_u32<<<1, 64, 0, st>>>(counter, 1, 0u);
      k_gen_grad<KW, SAMPLE, VT><<<gen_grid, 256, 0, st>>>(g);
      if constexpr (SAMPLE) {
        k_grad_sum<<<(int)((nsrc + 255) / 256), 256, 0, st>>>(nsplit, soff, gpart, nsrc, gitem, 0);
        for (int32_t smp = 0; smp < J.nsamp; ++smp) {
          const int64_t o0 = (int64_t)(J.samp_off[smp] - J.samp_off[0]);
          const int64_t cnt = (int64_t)(J.samp_off[smp + 1] - J.samp_off[smp]);
          if (cnt > 0)
            k_grad_scatter<<<(int)((cnt + 255) / 256), 256, 0, st>>>(gitem + o0, J.it_det + o0, cnt,
                                                                      J.grad_scale, J.grad);
        }
      } else {
        k_grad_sum<<<(int)((nsrc + 255) / 256), 256, 0, st>>>(nsplit, soff, gpart, nsrc, J.grad,
                                                                J.grad_accumulate ? 1 : 0);
      }
      HIPCHK(hipGetLastError());
    }
    if (J.want_u && J.ex && J.ex->u_keys) {
      k_nonv_counts<<<256, 256, 0, st>>>(U, P.nseg, G.nbucket, boff);
      CHK(scan_exclusive<uint64_t, uint64_t>(boff, boff, G.nbucket, hsc, nullptr, st));
      k_export_uniq<KW><<<1024, 64, 0, st>>>(U, P.nseg, boff, G.nbucket, n, J.ex->u_keys, J.ex->u_A,
                                             J.ex->u_D, J.ex->u_cnt, J.ex->u_cap);
      HIPCHK(hipGetLastError());
    }
    if (J.ex) {
      J.ex->u_n = J.res.nuniq;
      J.ex->t_n = split ? nrec_all : nrec;
    }
    HIPCHK(hipStreamSynchronize(st));
    AR.reset(job_mark);
    return SHCI_OK;
  }
}

template <typename VT, bool SAMPLE>
int dispatch_kw(Job& J) {
  const int kw = key_words(J.ctx->T.n, J.sbits);
  switch (kw) {
    case 1: return run_job<1, VT, SAMPLE>(J);
    case 2: return run_job<2, VT, SAMPLE>(J);
    case 3: return run_job<3, VT, SAMPLE>(J);
    case 4: return run_job<4, VT, SAMPLE>(J);
    default: return fail(SHCI_ERR_NORB, "key of %d words unsupported", kw);
  }
}

int dispatch(Job& J) {
  if (J.sample)
    return J.precision == SHCI_FP32C ? dispatch_kw<float, true>(J) : dispatch_kw<double, true>(J);
  return J.precision == SHCI_FP32C ? dispatch_kw<float, false>(J) : dispatch_kw<double, false>(J);
}

int common_checks(shci_pt2_ctx* ctx, const uint64_t* dets, const double* c, int64_t n_det, double e0,
                  double eps2, int precision) {
  if (!ctx) return fail(SHCI_ERR_ARG, "ctx is NULL");
  if (!dets || !c) return fail(SHCI_ERR_ARG, "dets or c is NULL");
  if (n_det < 1) return fail(SHCI_ERR_ARG, "n_det must be >= 1");
  if (n_det >= (int64_t)0xffffffffll) return fail(SHCI_ERR_ARG, "n_det must be < 2^32-1");
  if (!std::isfinite(e0)) return fail(SHCI_ERR_NONFINITE, "E0 is not finite");
  if (!(eps2 >= 0.0) || !std::isfinite(eps2)) return fail(SHCI_ERR_ARG, "eps2 must be finite and >= 0");
  if (precision != SHCI_FP64 && precision != SHCI_FP32C) return fail(SHCI_ERR_ARG, "unknown precision");
  HIPCHK(hipSetDevice(ctx->device));
  return SHCI_OK;
}

void fill_stats(shci_pt2_stats* st, const Job& J, float ms_total) {
  if (!st) return;
  st->n_terms = J.res.nterm;
  st->n_terms_gen = J.res.ngen;
  st->n_unique = J.res.nuniq;
  st->n_intruder = J.res.nintr;
  st->min_abs_denom = J.res.mind;
  st->n_buckets = J.nbucket;
  st->n_retries = J.retries;
  st->ms_gen = J.ms_gen;
  st->ms_sort = J.ms_sort;
  st->ms_reduce = J.ms_reduce;
  st->ms_total = ms_total;
  st->ms_k_count = J.ms_k_count;
  st->ms_k_write = J.ms_k_write;
  st->ms_k_reduce = J.ms_k_reduce;
  st->n_records = J.nrec;
  st->key_words = J.kw;
  st->value_bytes = J.vbytes;
  st->n_chunks = J.nbatch;
  st->n_part_launches = J.n_part;
  st->ms_k_part = J.ms_k_part;
  st->n_part_records = J.n_part_rec;
  st->n_terms_all = J.nrec_all;
  st->n_hashes = J.nhash;
  st->n_singletons = J.nrec_all - J.nmulti;
  st->ms_k_split = J.ms_k_split;
}

// Records one pass may materialise: the record limit if set, else what free
// device memory (plus the reusable record workspace), or the workspace limit,
// takes at `per_rec` bytes per record (two record buffers, bucket ids, the
// unique store when kept, per-bucket arrays), after a fixed reserve for the
// per-wavefront partials.
// Default cap on the records of one pass: larger passes partition more
// slowly (scattered writes over a larger working set) and gain nothing.
constexpr int64_t REC_CAP_AUTO = (int64_t)3 << 29;  // 1.61e9

int64_t record_budget(const Arena& A, double per_rec) {
  shci_pt2_ctx* X = A.X;
  if (X->rec_limit > 0) return X->rec_limit;
  size_t avail;
  if (A.caller()) {
    // an estimate for sizing; run_job checks the exact layout against the
    // workspace after its count pass
    avail = A.remaining();
  } else {
    size_t fr = 0, tt = 0;
    if (hipMemGetInfo(&fr, &tt) != hipSuccess) {
      (void)hipGetLastError();
      fr = 0;
    }
    avail = fr + A.L->slot[SL_REC].cap;
    if (X->ws_limit) avail = std::min(avail, X->ws_limit);
  }
  const size_t reserve = (size_t)(num_cus(X->device) * RED_BLOCKS_PER_CU * WRED_WAVES + 1024) * 64 + (2u << 20);
  avail = avail > reserve ? avail - reserve : 0;
  const int64_t m = (int64_t)((A.caller() ? 0.9 : 0.75) * (double)avail / per_rec);
  return std::max<int64_t>(1, std::min<int64_t>(m, REC_CAP_AUTO));
}

double record_bytes(int kw, int vbytes, bool pay, bool uniq, bool keep = false) {
  // two record buffers (keys, values, payload, bucket id, H_aa), then slack
  // for the bucket tables and the per-unique output (and the keep-mode
  // per-record adjoint terms)
  pay = pay || keep;
  return 2.0 * (8.0 * kw + vbytes + (pay ? 4.0 : 0.0) + 4.0 + 8.0) + 2.0 + (uniq ? 8.0 * kw + 40.0 : 0.0) +
         (keep ? 8.0 : 0.0);
}

// Deterministic evaluation within the record budget.  When the screened
// terms do not fit, they are split into B = 2^k hash batches of a (the low
// bits of the determinant hash; the bucket id uses the high bits): batch b
// regenerates every term and keeps those whose a falls in b, so every a is
// reduced whole inside one batch and E2 = sum over batches of E2_b.
int run_det_batched(const Job& proto, Job& acc) {
  shci_pt2_ctx* X = proto.ctx;
  const int kw = key_words(X->T.n, 0);
  const int vb = proto.precision == SHCI_FP32C ? 4 : 8;
  const int64_t max_rec = record_budget(*proto.ar, record_bytes(kw, vb, proto.want_pay, proto.want_u, proto.keep));
  uint32_t nb = 1;
  for (;;) {
    acc = Job{};
    acc.res.mind = INFINITY;
    bool again = false;
    for (uint32_t b = 0; b < nb; ++b) {
      Job J = proto;
      J.bmask = nb - 1;
      J.bsel = b;
      // with a caller workspace the job checks its exact layout against what
      // is left of it after its count pass
      J.max_records = (proto.ar->caller() && X->rec_limit == 0) ? REC_CAP_AUTO : max_rec;
      J.grad_accumulate = b > 0;
      shci_pt2_export exb{};
      if (proto.ex) {
        exb = *proto.ex;
        const int64_t ub = std::min<int64_t>(acc.res.nuniq, exb.u_cap);
        const int64_t tb = std::min<int64_t>(acc.nrec, exb.t_cap);
        if (exb.u_keys) {
          exb.u_keys += 4 * ub;
          exb.u_A += ub;
          exb.u_D += ub;
          exb.u_cnt += ub;
          exb.u_cap -= ub;
        }
        if (exb.t_keys) {
          exb.t_keys += 4 * tb;
          exb.t_i += tb;
          exb.t_val += tb;
          exb.t_cap -= tb;
        }
        J.ex = &exb;
      }
      const int r = dispatch(J);
      if (r == JOB_TOO_BIG) {
        // batches needed at this batch's size, with a margin for unevenness
        const double need = 1.3 * (double)J.nrec * nb / (double)std::max<int64_t>(1, J.max_records_eff);
        uint32_t nn = nb;
        while (nn < need) nn <<= 1;
        if (nn == nb) nn <<= 1;
        if (nn > 256)
          return fail(SHCI_ERR_WORKSPACE, "%lld screened terms need more than 256 hash batches of %lld records",
                      (long long)((double)J.nrec * nb), (long long)J.max_records_eff);
        nb = nn;
        again = true;
        break;
      }
      if (r) return r;
      acc.res.e2 += J.res.e2;
      acc.res.de0 += J.res.de0;
      acc.res.nterm += J.res.nterm;
      acc.res.ngen += J.res.ngen;
      acc.res.nuniq += J.res.nuniq;
      acc.res.nintr += J.res.nintr;
      acc.res.nzero += J.res.nzero;
      acc.res.mind = std::min(acc.res.mind, J.res.mind);
      acc.nbucket = std::max(acc.nbucket, J.nbucket);
      acc.retries += J.retries;
      acc.ms_gen += J.ms_gen;
      acc.ms_sort += J.ms_sort;
      acc.ms_reduce += J.ms_reduce;
      acc.ms_k_count += J.ms_k_count;
      acc.ms_k_write += J.ms_k_write;
      acc.ms_k_reduce += J.ms_k_reduce;
      acc.ms_k_part += J.ms_k_part;
      acc.n_part += J.n_part;
      acc.n_part_rec += J.n_part_rec;
      acc.nrec += J.nrec;
      acc.nrec_all += J.nrec_all;
      acc.nhash += J.nhash;
      acc.nmulti += J.nmulti;
      acc.ms_k_split += J.ms_k_split;
      acc.kw = J.kw;
      acc.vbytes = J.vbytes;
    }
    if (!again) break;
  }
  acc.nbatch = (int32_t)nb;
  if (proto.ex) {
    proto.ex->u_n = acc.res.nuniq;
    proto.ex->t_n = acc.nrec;
  }
  return SHCI_OK;
}

}  // namespace

// Workspace of shci_pt2_det_static: a file-scope device array, one copy per
// GPU, held until the process ends.  Host code never uses the array's name as
// an address: the device address comes from hipGetSymbolAddress, once per
// device, with that device current (at context creation).
constexpr size_t STATIC_WS_BYTES = (size_t)128 << 20;
constexpr int64_t STATIC_WS_MAX_DETS = 500000;
static __device__ __align__(256) unsigned char scratch[STATIC_WS_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
bool g_scratch_done[MAX_DEVICES] = {};
hipError_t g_scratch_err[MAX_DEVICES] = {};
void* g_scratch_ptr[MAX_DEVICES] = {};

// device address of `scratch` on device `dev`, which must be current; the
// symbol lookup runs once per device
int scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= MAX_DEVICES) return fail(SHCI_ERR_HIP, "device %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_done[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) (void)hipGetLastError();
    g_scratch_err[dev] = e;
    g_scratch_ptr[dev] = e == hipSuccess ? p : nullptr;
    g_scratch_done[dev] = true;
  }
  if (g_scratch_err[dev] != hipSuccess)
    return fail(SHCI_ERR_HIP, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                hipGetErrorString(g_scratch_err[dev]));
  *out = g_scratch_ptr[dev];
  return SHCI_OK;
}

int ws_check(const void* ws, size_t ws_bytes) {
  if (ws && ((uintptr_t)ws & (WS_ALIGN - 1)))
    return fail(SHCI_ERR_ARG, "ws must be aligned to %zu bytes", WS_ALIGN);
  if (ws && ws_bytes == 0) return fail(SHCI_ERR_ARG, "ws_bytes must be > 0 when ws is given");
  return SHCI_OK;
}

// Alias table of p_i = |c_i| / sum_j |c_j| (thresholds and aliases, device
// arrays of n); temporaries from the arena, released on return.
struct AliasTmp {
  AliasArgs a;
  ScanTmp s1, s2, s3;
};
template <class CV>
void plan_alias(CV& cv, AliasTmp& t, int64_t n) {
  const int64_t nblk = (n + 4095) / 4096;
  t.a.maxbits = cv.template take<uint64_t>(2);
  t.a.w = cv.template take<u128>(n);
  t.a.tsum = cv.template take<u128>(nblk);
  t.a.tot = cv.template take<u128>(1);
  t.a.isl = cv.template take<uint32_t>(n);
  t.a.lpos = cv.template take<uint64_t>(n + 1);
  t.a.hidx = cv.template take<uint32_t>(n);
  t.a.dl = cv.template take<u128>(n + 1);
  t.a.xh = cv.template take<u128>(n + 1);
  t.s1.carve(cv, n + 1);
  t.s2.carve(cv, n + 1, 2);
  t.s3.carve(cv, n + 1, 2);
}

int build_alias(Arena& A, const double* c, int64_t n, uint64_t* thr, uint32_t* alias, hipStream_t st) {
  AliasTmp t;
  const size_t m = A.mark();
  CHK(carve_region(A, SL_ALIAS, [&](Carver& cv) { plan_alias(cv, t, n); }));
  AliasArgs& a = t.a;
  a.c = c;
  a.n = n;
  a.K = 127 - 2 * ceil_log2((uint64_t)n);
  a.thr = thr;
  a.alias = alias;
  a.flag = A.X->dflag;
  const int64_t nblk = (n + 4095) / 4096;
  const int grid = (int)std::min<int64_t>(8192, (n + 255) / 256);
  k_fill_u64<<<1, 64, 0, st>>>(a.maxbits, 1, 0ull);
  k_alias_max<<<grid, 256, 0, st>>>(c, n, a.maxbits, a.flag);
  k_alias_weights<<<(int)nblk, 256, 0, st>>>(a);
  k_alias_total<<<1, 256, 0, st>>>(a, nblk);
  k_alias_classify<<<grid, 256, 0, st>>>(a);
  CHK(scan_exclusive<uint32_t, uint64_t>(a.isl, a.lpos, n, t.s1, a.lpos + n, st));
  k_alias_heavies<<<grid, 256, 0, st>>>(a);
  CHK(scan_exclusive<u128, u128>(a.dl, a.dl, n, t.s2, a.dl + n, st));
  CHK(scan_exclusive<u128, u128>(a.xh, a.xh, n, t.s3, a.xh + n, st));
  k_alias_assemble<<<grid, 256, 0, st>>>(a);
  HIPCHK(hipGetLastError());
  // later regions may reuse the temporaries: they run after these kernels
  // on the same stream
  A.reset(m);
  return SHCI_OK;
}

// batch of P of each sample on the seed path: the top log2(n_batches) bits
// of SplitMix64 output 2 N_s N_d + s + 1 (after the outputs of the draws)
__global__ void k_seed_batches(uint64_t seed, int32_t ns, int32_t nd, int32_t n_batches, int32_t* out) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= ns) return;
  const uint64_t r = splitmix64_out(seed, 2 * (uint64_t)ns * (uint64_t)nd + (uint64_t)s + 1);
  out[s] = (int32_t)__umul64hi(r, (uint64_t)n_batches);
}

__global__ void k_check_batches(const int32_t* sb, int32_t ns, int32_t n_batches, uint32_t* flag) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < ns && (sb[s] < 0 || sb[s] >= n_batches)) atomicOr(flag, 128u);
}

// draws [ns][nd] of the stochastic samples from the seed
int seed_draws(Arena& A, const double* c, int64_t n, uint64_t seed, int32_t ns, int32_t nd, uint32_t* draws,
               hipStream_t st) {
  uint64_t* thr = nullptr;
  uint32_t* al = nullptr;
  const size_t m = A.mark();
  CHK(carve_region(A, SL_TABLE, [&](Carver& cv) {
    thr = cv.take<uint64_t>(n);
    al = cv.take<uint32_t>(n);
  }));
  CHK(build_alias(A, c, n, thr, al, st));
  const int64_t tot = (int64_t)ns * nd;
  k_alias_draw<<<(int)std::min<int64_t>(16384, (tot + 255) / 256), 256, 0, st>>>(thr, al, n, seed, ns, nd, draws);
  HIPCHK(hipGetLastError());
  A.reset(m);
  return SHCI_OK;
}

// bytes of the job regions (validation / V set, work items, records)
size_t job_bytes(int kw, int vsize, bool sample, bool grad, bool keep, bool want_u, int64_t ndet, int64_t nsrc,
                 int64_t ni, int64_t nrec, int32_t nsamp, int cus) {
  uint64_t vcap;
  int fbits;
  int64_t fwords;
  vset_dims(ndet, vcap, fbits, fwords);
  size_t tot = 0;
  {
    Carver cv(nullptr);
    Phase0 p;
    plan_phase0(cv, p, nsrc, vcap, fwords);
    tot += cv.off + WS_ALIGN;
  }
  {
    Carver cv(nullptr);
    Phase1 p;
    plan_phase1(cv, p, ni, nsrc, grad, sample);
    tot += cv.off + WS_ALIGN;
  }
  {
    GroupPlan G;
    G.sbits = sample ? std::max(1, ceil_log2((uint64_t)std::max(1, nsamp))) : 0;
    const int64_t per = sample ? std::max<int64_t>(1, nrec / std::max(1, nsamp)) : nrec;
    G.bits_hash = std::min(26, std::max(0, ceil_log2((uint64_t)((per + 127) / 128))));
    G.nbits = G.bits_hash + G.sbits;
    BigDims d;
    d.kw = kw;
    d.vsize = vsize;
    d.v2 = sample;
    d.pay = keep;
    d.want_u = want_u;
    d.keep = keep;
    d.nrec = nrec;
    // one re-plan with an extra hash bit is allowed for
    d.nbucket = (int64_t)1 << (G.nbits + 1);
    d.ntiles = std::max<int64_t>(1, (nrec + PTILE - 1) / PTILE);
    d.npass = (G.nbits + 1 + 7) / 8;
    d.npart = (int64_t)cus * RED_BLOCKS_PER_CU * WRED_WAVES * (sample ? ((int64_t)1 << G.sbits) : 1);
    Carver cv(nullptr);
    BigPlan o;
    plan_big(cv, d, o);
    tot += cv.off + WS_ALIGN;
  }
  return tot;
}

}  // namespace

extern "C" {

const char* shci_pt2_last_error(void) { return g_msg; }

const char* shci_pt2_version(void) { return "shci_pt2 0.2 (gfx950)"; }

int shci_pt2_ctx_create(int n_orb, int n_alpha, int n_beta, const double* h1, const double* eri, void* stream,
                        shci_pt2_ctx** out) {
  if (!out) return fail(SHCI_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!h1 || !eri) return fail(SHCI_ERR_ARG, "h1 or eri is NULL");
  if (n_orb < 2 || n_orb > 127) return fail(SHCI_ERR_NORB, "n_orb must be in [2, 127]");
  if (n_alpha < 1 || n_alpha >= n_orb || n_beta < 1 || n_beta >= n_orb)
    return fail(SHCI_ERR_NORB, "electron counts must be in [1, n_orb - 1]");
  shci_pt2_ctx* X = new (std::nothrow) shci_pt2_ctx();
  if (!X) return fail(SHCI_ERR_WORKSPACE, "out of host memory");
  hipStream_t st = static_cast<hipStream_t>(stream);
  auto bail = [&](int code) {
    shci_pt2_ctx_destroy(X);
    return code;
  };
  if (hipGetDevice(&X->device) != hipSuccess) return bail(fail(SHCI_ERR_HIP, "hipGetDevice failed"));
  {
    // set-up of the allocation-free entry point on this device (its errors
    // are reported by that entry point)
    void* sp = nullptr;
    (void)scratch_address(X->device, &sp);
    g_msg[0] = 0;
  }
  Tables& T = X->T;
  const int n = n_orb;
  T.n = n;
  T.na = n_alpha;
  T.nb = n_beta;
  T.nss = n * (n - 1) / 2;
  T.lss = (int64_t)(n - 2) * (n - 3) / 2;
  T.los = (int64_t)(n - 1) * (n - 1);
  const int64_t n2 = (int64_t)n * n, n3 = n2 * n;
  const int64_t nhb = (int64_t)T.nss * T.lss + n2 * T.los;
  auto plan = [&](Carver& cv) {
    T.h1 = cv.take<double>(n2);
    T.sD = cv.take<double>(n3);
    T.sJ = cv.take<double>(n3);
    T.ubound = cv.take<double>(n2);
    T.fref = cv.take<double>(2 * n2);
    T.diag = cv.take<double>(diag_table_doubles(n));
    T.hpp = T.diag;
    T.jtri = T.diag + n;
    T.sstri = T.diag + n + n * (n + 1) / 2;
    T.hb_val = cv.take<double>(nhb);
    T.hb_rs = cv.take<uint16_t>(nhb);
    T.hb_max = cv.take<double>(T.nss + n2);
    T.mag_cum = cv.take<double>(144);
    {
      const int64_t npair = (int64_t)n * (n + 1) / 2;
      T.g8 = cv.take<double>(npair * (npair + 1) / 2);
    }
    X->dflag = cv.take<uint32_t>(16);
    X->dctr = cv.take<unsigned long long>(4);
    X->dres = cv.take<DevResult>(1);
    X->lane1.dflag = cv.take<uint32_t>(16);
    X->lane1.dctr = cv.take<unsigned long long>(4);
    X->lane1.dres = cv.take<DevResult>(1);

  };
  {
    Carver cv(nullptr);
    plan(cv);
    int s = X->tables.ensure(cv.off, 0, st);
    if (s) return bail(s);
    Carver cv2(X->tables.p);
    plan(cv2);
  }
  for (auto& e : X->ev)
    if (hipEventCreate(&e) != hipSuccess) return bail(fail(SHCI_ERR_HIP, "hipEventCreate failed"));
  for (auto& e : X->evp)
    if (hipEventCreate(&e) != hipSuccess) return bail(fail(SHCI_ERR_HIP, "hipEventCreate failed"));
  for (auto& e : X->evh)
    if (hipEventCreate(&e) != hipSuccess) return bail(fail(SHCI_ERR_HIP, "hipEventCreate failed"));
  for (Lane* l : {static_cast<Lane*>(&X->lane1)}) {
    for (auto& e : l->ev)
      if (hipEventCreate(&e) != hipSuccess) return bail(fail(SHCI_ERR_HIP, "hipEventCreate failed"));
    for (auto& e : l->evp)
      if (hipEventCreate(&e) != hipSuccess) return bail(fail(SHCI_ERR_HIP, "hipEventCreate failed"));
    for (auto& e : l->evh)
      if (hipEventCreate(&e) != hipSuccess) return bail(fail(SHCI_ERR_HIP, "hipEventCreate failed"));
  }
  if (hipEventCreateWithFlags(&X->fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&X->join, hipEventDisableTiming) != hipSuccess ||
      hipStreamCreateWithFlags(&X->lane1_stream, hipStreamNonBlocking) != hipSuccess)
    return bail(fail(SHCI_ERR_HIP, "stream or event creation failed"));
  k_fill_u32<<<1, 64, 0, st>>>(X->lane1.dflag, 16, 0u);
  if (hipMemcpyAsync(T.h1, h1, n2 * sizeof(double), hipMemcpyDeviceToDevice, st) != hipSuccess)
    return bail(fail(SHCI_ERR_HIP, "copy of h1 failed"));
  k_fill_u32<<<1, 64, 0, st>>>(X->dflag, 16, 0u);
  if (build_tables(T, h1, eri, st, X->dflag) != 0)
    return bail(fail(SHCI_ERR_HIP, "table build launch failed: %s", hipGetErrorString(hipGetLastError())));
  uint32_t hf = 0;
  if (hipMemcpyAsync(&hf, X->dflag, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return bail(fail(SHCI_ERR_HIP, "table build failed"));
  if (hf) return bail(fail(SHCI_ERR_NONFINITE, "an integral is not finite"));
  *out = X;
  return SHCI_OK;
}

void shci_pt2_ctx_destroy(shci_pt2_ctx* ctx) {
  if (!ctx) return;
  (void)hipDeviceSynchronize();
  for (auto& e : ctx->ev)
    if (e) (void)hipEventDestroy(e);
  for (auto& e : ctx->evp)
    if (e) (void)hipEventDestroy(e);
  for (auto& e : ctx->evh)
    if (e) (void)hipEventDestroy(e);
  for (Lane* l : {static_cast<Lane*>(&ctx->lane1)}) {
    for (auto& e : l->ev)
      if (e) (void)hipEventDestroy(e);
    for (auto& e : l->evp)
      if (e) (void)hipEventDestroy(e);
    for (auto& e : l->evh)
      if (e) (void)hipEventDestroy(e);
    for (auto& b : l->slot) b.release();
  }
  if (ctx->fork) (void)hipEventDestroy(ctx->fork);
  if (ctx->join) (void)hipEventDestroy(ctx->join);
  if (ctx->lane1_stream) (void)hipStreamDestroy(ctx->lane1_stream);
  ctx->tables.release();
  for (auto& b : ctx->slot) b.release();
  delete ctx;
}

int shci_pt2_ctx_set_record_limit(shci_pt2_ctx* ctx, int64_t max_records) {
  if (!ctx) return fail(SHCI_ERR_ARG, "ctx is NULL");
  if (max_records < 0) return fail(SHCI_ERR_ARG, "max_records must be >= 0");
  ctx->rec_limit = max_records;
  return SHCI_OK;
}

int shci_pt2_ctx_set_grouping(shci_pt2_ctx* ctx, int mode) {
  if (!ctx) return fail(SHCI_ERR_ARG, "ctx is NULL");
  if (mode != SHCI_GROUP_AUTO && mode != SHCI_GROUP_RECORDS && mode != SHCI_GROUP_SPLIT)
    return fail(SHCI_ERR_ARG, "unknown grouping mode");
  ctx->grouping = mode;
  return SHCI_OK;
}

int shci_pt2_ctx_set_split_bucket(shci_pt2_ctx* ctx, int64_t hashes) {
  if (!ctx) return fail(SHCI_ERR_ARG, "ctx is NULL");
  if (hashes < 64 || hashes > ((int64_t)1 << 24)) return fail(SHCI_ERR_ARG, "bucket size must lie in [64, 2^24]");
  ctx->split_bucket = hashes;
  return SHCI_OK;
}

int shci_pt2_ctx_set_lanes(shci_pt2_ctx* ctx, int lanes) {
  if (!ctx) return fail(SHCI_ERR_ARG, "ctx is NULL");
  if (lanes != 1 && lanes != 2) return fail(SHCI_ERR_ARG, "lanes must be 1 or 2");
  ctx->lanes = lanes;
  return SHCI_OK;
}

int shci_pt2_ctx_set_workspace_limit(shci_pt2_ctx* ctx, size_t bytes) {
  if (!ctx) return fail(SHCI_ERR_ARG, "ctx is NULL");
  ctx->ws_limit = bytes;
  return SHCI_OK;
}

int shci_pt2_workspace_size(const shci_pt2_ctx* ctx, int op, int64_t n_det, int64_t n_records, int32_t n_samples,
                            int32_t n_draws, int precision, size_t* bytes) {
  if (!ctx || !bytes) return fail(SHCI_ERR_ARG, "ctx and bytes must be non-NULL");
  if (n_det < 1 || n_det >= (int64_t)0xffffffffll) return fail(SHCI_ERR_ARG, "n_det must be in [1, 2^32 - 1)");
  if (n_records < 0) return fail(SHCI_ERR_ARG, "n_records must be >= 0");
  if (precision != SHCI_FP64 && precision != SHCI_FP32C) return fail(SHCI_ERR_ARG, "unknown precision");
  const bool sample = op == SHCI_OP_SAMPLE || op == SHCI_OP_SAMPLE_GRAD;
  if (op < SHCI_OP_DET || op > SHCI_OP_DRAWS) return fail(SHCI_ERR_ARG, "unknown op");
  if ((sample || op == SHCI_OP_DRAWS) && (n_samples < 1 || n_draws < 1))
    return fail(SHCI_ERR_ARG, "sample ops need n_samples >= 1 and n_draws >= 1");
  const int vsize = precision == SHCI_FP32C ? 4 : 8;
  const int cus = num_cus(ctx->device);
  const int64_t nrec = std::max<int64_t>(n_records, 1024);
  const int64_t cap = sample || op == SHCI_OP_DRAWS ? (int64_t)n_samples * n_draws : 0;
  size_t tot = 0;
  // seed path: draws and sample batches, then the alias table and its
  // temporaries (released before the samples are evaluated)
  size_t draws_b = 0, alias_b = 0;
  if (cap) {
    Carver cv(nullptr);
    cv.take<uint32_t>(cap);
    cv.take<int32_t>(n_samples);
    draws_b = cv.off + WS_ALIGN;
    Carver ca(nullptr);
    ca.take<uint64_t>(n_det);
    ca.take<uint32_t>(n_det);
    AliasTmp t;
    plan_alias(ca, t, n_det);
    alias_b = ca.off + 2 * WS_ALIGN;
  }
  if (op == SHCI_OP_DRAWS) {
    *bytes = draws_b + alias_b;
    return SHCI_OK;
  }
  if (sample) {
    Carver cv(nullptr);
    for (int k = 0; k < 5; ++k) cv.take<uint32_t>(cap);
    cv.take<uint32_t>(n_samples + 1);
    cv.take<uint64_t>(n_samples + 1);
    cv.take<double>(4);
    cv.take<double>(n_samples + 1);
    ScanTmp tmp;
    tmp.carve(cv, n_samples + 1);
    const size_t items_b = cv.off + WS_ALIGN;
    const int kw = key_words(ctx->T.n, std::max(1, ceil_log2((uint64_t)n_samples)));
    const size_t job = job_bytes(kw, vsize, true, op == SHCI_OP_SAMPLE_GRAD, false, op == SHCI_OP_SAMPLE_GRAD,
                                 n_det, cap, cap + cap / 2, nrec, n_samples, cus);
    tot = draws_b + std::max(alias_b, items_b + job);
  } else {
    const int kw = key_words(ctx->T.n, 0);
    const bool keep = op == SHCI_OP_GRAD_KEEP;
    const bool grad = op == SHCI_OP_GRAD || keep;
    tot = job_bytes(kw, vsize, false, grad, keep, op == SHCI_OP_GRAD, n_det, n_det, 2 * n_det, nrec, 1, cus);
  }
  *bytes = tot;
  return SHCI_OK;
}

int shci_pt2_det(shci_pt2_ctx* ctx, const uint64_t* dets, const double* c, int64_t n_det, double e0,
                 double eps2, int precision, void* ws, size_t ws_bytes, void* stream, double* e2,
                 shci_pt2_stats* st, shci_pt2_export* ex) {
  CHK(common_checks(ctx, dets, c, n_det, e0, eps2, precision));
  CHK(ws_check(ws, ws_bytes));
  if (!e2) return fail(SHCI_ERR_ARG, "e2 is NULL");
  Arena AR(ctx, static_cast<hipStream_t>(stream), ws, ws_bytes);
  Job J{};
  J.ctx = ctx;
  J.ar = &AR;
  J.st = static_cast<hipStream_t>(stream);
  J.dets = dets;
  J.c = c;
  J.ndet = n_det;
  J.e0 = e0;
  J.eps2 = eps2;
  J.eps2_d = INFINITY;
  J.precision = precision;
  J.sample = false;
  J.sbits = 0;
  J.nsamp = 1;
  J.nd = 0.0;
  J.n_items = n_det;
  J.ex = ex;
  J.want_u = ex && ex->u_keys;
  J.want_pay = ex && ex->t_keys;
  Job R;
  CHK(run_det_batched(J, R));
  *e2 = R.res.e2;
  fill_stats(st, R, R.ms_gen + R.ms_sort + R.ms_reduce);
  if (R.res.nzero) return fail(SHCI_ERR_SINGULAR, "%lld kept determinants have E0 - H_aa == 0",
                               (long long)R.res.nzero);
  return SHCI_OK;
}

int shci_pt2_det_static(shci_pt2_ctx* ctx, const uint64_t* dets, const double* c, int64_t n_det, double e0,
                        double eps2, int precision, void* stream, double* e2, shci_pt2_stats* st) {
  CHK(common_checks(ctx, dets, c, n_det, e0, eps2, precision));
  if (n_det > STATIC_WS_MAX_DETS)
    return fail(SHCI_ERR_WORKSPACE, "shci_pt2_det_static takes at most %lld determinants (got %lld)",
                (long long)STATIC_WS_MAX_DETS, (long long)n_det);
  void* ws = nullptr;
  CHK(scratch_address(ctx->device, &ws));
  return shci_pt2_det(ctx, dets, c, n_det, e0, eps2, precision, ws, STATIC_WS_BYTES, stream, e2, st, nullptr);
}

int shci_pt2_grad(shci_pt2_ctx* ctx, const uint64_t* dets, const double* c, int64_t n_det, double e0,
                  double eps2, int precision, int mode, void* ws, size_t ws_bytes, void* stream, double* e2,
                  double* de2_dc, double* de2_de0, shci_pt2_stats* st) {
  CHK(common_checks(ctx, dets, c, n_det, e0, eps2, precision));
  CHK(ws_check(ws, ws_bytes));
  if (!de2_dc) return fail(SHCI_ERR_ARG, "de2_dc is NULL");
  if (mode != SHCI_GRAD_AUTO && mode != SHCI_GRAD_KEEP && mode != SHCI_GRAD_RECOMPUTE)
    return fail(SHCI_ERR_ARG, "unknown adjoint mode");
  Arena AR(ctx, static_cast<hipStream_t>(stream), ws, ws_bytes);
  Job J{};
  J.ctx = ctx;
  J.ar = &AR;
  J.st = static_cast<hipStream_t>(stream);
  J.dets = dets;
  J.c = c;
  J.ndet = n_det;
  J.e0 = e0;
  J.eps2 = eps2;
  J.eps2_d = INFINITY;
  J.precision = precision;
  J.nsamp = 1;
  J.n_items = n_det;
  J.grad = de2_dc;
  // keep: records carry their position, the reduce writes each record's
  // adjoint term (no second generation pass); recompute: the unique store
  // is kept and the adjoint walks the connections again.  auto takes keep
  // when one pass holds every record, recompute when hash batches are needed.
  bool keep = mode == SHCI_GRAD_KEEP;
  if (mode == SHCI_GRAD_AUTO) {
    J.keep = true;
    J.want_u = false;
    J.max_records = 0;
    Job probe = J;
    // one keep-mode pass if it fits; otherwise recompute over hash batches
    const int kw = key_words(ctx->T.n, 0);
    probe.max_records = record_budget(AR, record_bytes(kw, precision == SHCI_FP32C ? 4 : 8, false, false, true));
    if (AR.caller() && ctx->rec_limit == 0) probe.max_records = REC_CAP_AUTO;
    const int r = dispatch(probe);
    if (r == SHCI_OK) {
      probe.nbatch = 1;
      if (e2) *e2 = probe.res.e2;
      if (de2_de0) *de2_de0 = probe.res.de0;
      fill_stats(st, probe, probe.ms_gen + probe.ms_sort + probe.ms_reduce);
      if (probe.res.nzero) return fail(SHCI_ERR_SINGULAR, "%lld kept determinants have E0 - H_aa == 0",
                                       (long long)probe.res.nzero);
      return SHCI_OK;
    }
    if (r != JOB_TOO_BIG) return r;
    keep = false;
  }
  J.keep = keep;
  J.want_u = !keep;
  Job R;
  CHK(run_det_batched(J, R));
  if (e2) *e2 = R.res.e2;
  if (de2_de0) *de2_de0 = R.res.de0;
  fill_stats(st, R, R.ms_gen + R.ms_sort + R.ms_reduce);
  if (R.res.nzero) return fail(SHCI_ERR_SINGULAR, "%lld kept determinants have E0 - H_aa == 0",
                               (long long)R.res.nzero);
  return SHCI_OK;
}

static int sample_impl(shci_pt2_ctx* ctx, const uint64_t* dets, const double* c, int64_t n_det, double e0,
                       double eps2, double eps2_d, int32_t n_samples, int32_t n_draws, const uint32_t* draws,
                       uint64_t seed, int precision, void* ws, size_t ws_bytes, void* stream, double* per_sample,
                       double* mean, double* sem, shci_pt2_stats* st, double* grad, double* de2_de0,
                       int32_t n_batches = 1, const int32_t* sample_batch = nullptr) {
  CHK(common_checks(ctx, dets, c, n_det, e0, eps2, precision));
  CHK(ws_check(ws, ws_bytes));
  if (!per_sample) return fail(SHCI_ERR_ARG, "per_sample is NULL");
  if (n_samples < 1 || n_draws < 2) return fail(SHCI_ERR_ARG, "need n_samples >= 1 and n_draws >= 2");
  if (n_draws > MAX_DRAWS) return fail(SHCI_ERR_ARG, "n_draws must be <= %d", MAX_DRAWS);
  if ((int64_t)n_samples * n_draws >= ((int64_t)1 << 31))
    return fail(SHCI_ERR_ARG, "n_samples * n_draws must be < 2^31");
  if (!(eps2_d >= eps2)) return fail(SHCI_ERR_ARG, "eps2_d must be >= eps2");
  if (n_batches < 1 || n_batches > 65536 || (n_batches & (n_batches - 1)))
    return fail(SHCI_ERR_ARG, "n_batches must be a power of two in [1, 65536]");
  const int sbits = std::max(1, ceil_log2((uint64_t)n_samples));
  if (2 * ctx->T.n + sbits + 1 > 256) return fail(SHCI_ERR_NORB, "too many samples for this n_orb");
  hipStream_t s = static_cast<hipStream_t>(stream);
  Arena AR(ctx, s, ws, ws_bytes);
  k_fill_u32<<<1, 64, 0, s>>>(ctx->dflag, 4, 0u);
  // seed path: draws (and sample batches) made on the device
  const uint32_t* dr = draws;
  const int32_t* sbatch = sample_batch;
  if (!draws || (n_batches > 1 && !sample_batch)) {
    uint32_t* own_d = nullptr;
    int32_t* own_b = nullptr;
    CHK(carve_region(AR, SL_DRAWS, [&](Carver& cv) {
      own_d = cv.take<uint32_t>((int64_t)n_samples * n_draws);
      own_b = cv.take<int32_t>(n_samples);
    }));
    if (!draws) {
      CHK(seed_draws(AR, c, n_det, seed, n_samples, n_draws, own_d, s));
      dr = own_d;
    }
    if (n_batches > 1 && !sample_batch) {
      k_seed_batches<<<(n_samples + 255) / 256, 256, 0, s>>>(seed, n_samples, n_draws, n_batches, own_b);
      sbatch = own_b;
    }
  }
  if (n_batches > 1 && sample_batch)
    k_check_batches<<<(n_samples + 255) / 256, 256, 0, s>>>(sample_batch, n_samples, n_batches, ctx->dflag);
  // items: distinct dets per sample
  const int64_t cap = (int64_t)n_samples * n_draws;
  uint32_t *t_det, *t_w, *ucount, *o_det, *o_w, *o_s;
  uint64_t* uoff;
  double *dsum, *psde0;
  ScanTmp tmp;
  CHK(carve_region(AR, SL_SAMPLE, [&](Carver& cv) {
    t_det = cv.take<uint32_t>(cap);
    t_w = cv.take<uint32_t>(cap);
    ucount = cv.take<uint32_t>(n_samples + 1);
    uoff = cv.take<uint64_t>(n_samples + 1);
    o_det = cv.take<uint32_t>(cap);
    o_w = cv.take<uint32_t>(cap);
    o_s = cv.take<uint32_t>(cap);
    dsum = cv.take<double>(4);
    psde0 = cv.take<double>(n_samples + 1);
    tmp.carve(cv, n_samples + 1);
  }));
  auto done = [&](int code) {
    (void)hipStreamSynchronize(s);
    return code;
  };
  k_sample_items<<<n_samples, 256, 0, s>>>(dr, n_draws, n_det, t_det, t_w, ucount, ctx->dflag);
  k_sum_abs<<<1, 1024, 0, s>>>(c, n_det, dsum);
  uint64_t* tot = uoff + n_samples;
  int sc = scan_exclusive<uint32_t, uint64_t>(ucount, uoff, n_samples, tmp, tot, s);
  if (sc) return done(sc);
  double hsum = 0.0;
  uint32_t hf = 0;
  std::vector<uint64_t> hoff(n_samples + 1);
  if (hipMemcpyAsync(hoff.data(), uoff, (n_samples + 1) * sizeof(uint64_t), hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      hipMemcpyAsync(&hsum, dsum, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipMemcpyAsync(&hf, ctx->dflag, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return done(fail(SHCI_ERR_HIP, "sample preparation failed"));
  if (hf & 2u) return done(fail(SHCI_ERR_NONFINITE, "c contains a non-finite value"));
  if (hf & 64u) return done(fail(SHCI_ERR_NONFINITE, "every coefficient is zero"));
  if (hf & 16u) return done(fail(SHCI_ERR_ARG, "a draw is >= n_det"));
  if (hf & 128u) return done(fail(SHCI_ERR_ARG, "sample_batch entries must lie in [0, n_batches)"));
  if (!(hsum > 0.0) || !std::isfinite(hsum)) return done(fail(SHCI_ERR_NONFINITE, "sum |c| is not positive and finite"));

  // Samples are evaluated in chunks of consecutive samples: one generation /
  // grouping launch sequence per chunk covers all its samples (sample id in
  // the key).  The first chunk (up to 8 samples) sets the terms per sample;
  // the others then take as many samples as a pass holds (a power of two).
  // With a caller workspace the later chunks run two at a time on two lanes
  // (this thread and the caller's stream; a second thread and stream), each
  // with half of what is left of the workspace: one chunk's grouping (HBM
  // bound) runs beside another's generation (VALU bound).  The chunk plan
  // depends on the inputs and sizes only, so results do not depend on the
  // timing; a chunk whose terms do not fit is evaluated as two halves.
  // (with the singleton split a term takes a list slot, not a record)
  const bool split_ok = ctx->grouping != SHCI_GROUP_RECORDS && grad == nullptr;
  auto max_rec_of = [&](const Arena& A) -> int64_t {
    return split_ok ? (ctx->rec_limit > 0 ? ctx->rec_limit
                                          : std::max<int64_t>(1, std::min<int64_t>((int64_t)(0.9 * (double)HASH_CAP),
                                                                                   split_budget(A))))
                    : record_budget(A, record_bytes(key_words(ctx->T.n, sbits), precision == SHCI_FP32C ? 8 : 16,
                                                    false, grad != nullptr));
  };
  if (grad) k_fill_u64<<<(int)std::min<int64_t>(4096, (n_det + 255) / 256), 256, 0, s>>>(
      reinterpret_cast<uint64_t*>(grad), n_det, 0ull);
  auto pow2_floor = [](int64_t v) {
    int32_t p = 1;
    while ((int64_t)p * 2 <= v) p *= 2;
    return p;
  };
  auto add_stats = [](Job& acc, const Job& J) {
    acc.res.nterm += J.res.nterm;
    acc.res.ngen += J.res.ngen;
    acc.res.nuniq += J.res.nuniq;
    acc.res.nintr += J.res.nintr;
    acc.res.nzero += J.res.nzero;
    acc.res.mind = std::min(acc.res.mind, J.res.mind);
    acc.nbucket = std::max(acc.nbucket, J.nbucket);
    acc.retries += J.retries;
    acc.ms_gen += J.ms_gen;
    acc.ms_sort += J.ms_sort;
    acc.ms_reduce += J.ms_reduce;
    acc.ms_k_count += J.ms_k_count;
    acc.ms_k_write += J.ms_k_write;
    acc.ms_k_reduce += J.ms_k_reduce;
    acc.ms_k_part += J.ms_k_part;
    acc.n_part += J.n_part;
    acc.n_part_rec += J.n_part_rec;
    acc.nrec += J.nrec;
    acc.nrec_all += J.nrec_all;
    acc.nhash += J.nhash;
    acc.nmulti += J.nmulti;
    acc.ms_k_split += J.ms_k_split;
    acc.kw = std::max(acc.kw, J.kw);
    acc.vbytes = J.vbytes;
  };
  // one chunk [s0, s0 + k) on an arena, lane and stream; halves when its
  // terms do not fit
  std::function<int(int32_t, int32_t, Arena&, Lane*, hipStream_t, int64_t, Job&)> run_chunk =
      [&](int32_t s0, int32_t k, Arena& A, Lane* lane, hipStream_t strm, int64_t max_rec, Job& acc) -> int {
    k_sample_compact<<<k, 256, 0, strm>>>(t_det + (int64_t)s0 * n_draws, t_w + (int64_t)s0 * n_draws,
                                            ucount + s0, uoff + s0, n_draws, 0, o_det, o_w, o_s);
    Job J{};
    J.ctx = ctx;
    J.ar = &A;
    J.lane = lane;
    J.st = strm;
    J.dets = dets;
    J.c = c;
    J.ndet = n_det;
    J.e0 = e0;
    J.eps2 = eps2;
    J.eps2_d = eps2_d;
    J.precision = precision;
    J.sample = true;
    J.sbits = std::max(1, ceil_log2((uint64_t)k));
    J.nsamp = k;
    J.nd = (double)n_draws;
    J.sum_abs = hsum;
    J.it_det = o_det + hoff[s0];
    J.it_w = o_w + hoff[s0];
    J.it_s = o_s + hoff[s0];
    J.n_items = (int64_t)(hoff[s0 + k] - hoff[s0]);
    J.per_sample = per_sample + s0;
    J.per_sample_de0 = psde0 + s0;
    J.max_records = (A.caller() && ctx->rec_limit == 0) ? REC_CAP_AUTO : max_rec;
    J.samp_off = hoff.data() + s0;
    if (n_batches > 1) {
      // one batch of P per sample, the estimate scaled by the number of batches
      J.bmask = (uint32_t)(n_batches - 1);
      J.sbatch = sbatch + s0;
      J.sample_scale = (double)n_batches;
    }
    if (grad) {
      J.want_u = true;
      J.grad = grad;
      J.grad_scale = (double)n_batches / (double)n_samples;
    }
    const int r = dispatch(J);
    if (r == JOB_TOO_BIG) {
      if (k == 1)
        return fail(SHCI_ERR_WORKSPACE, "one sample has %lld screened terms; the workspace holds %lld",
                    (long long)J.nrec, (long long)J.max_records_eff);
      const int32_t h = k / 2;
      CHK(run_chunk(s0, h, A, lane, strm, max_rec, acc));
      return run_chunk(s0 + h, k - h, A, lane, strm, max_rec, acc);
    }
    if (r) return r;
    add_stats(acc, J);
    acc.nbatch += 1;  // chunks evaluated
    return SHCI_OK;
  };
  Job acc{};
  acc.res.mind = INFINITY;
  acc.nbatch = 0;
  const int64_t max_rec0 = max_rec_of(AR);
  const int32_t k0 = std::min<int32_t>(n_samples, 8);
  if (int r = run_chunk(0, k0, AR, nullptr, s, max_rec0, acc)) return done(r);
  if (k0 < n_samples) {
    const bool two = AR.caller() && ctx->lanes == 2;
    // the rest: chunks of kr samples (the budget of one lane when two run)
    Arena half0(ctx, s, nullptr, 0), half1(ctx, ctx->lane1_stream, nullptr, 0, &ctx->lane1);
    if (two) {
      const size_t o = (AR.off + WS_ALIGN - 1) & ~(WS_ALIGN - 1);
      const size_t left = AR.cap > o ? AR.cap - o : 0;
      const size_t h = (left / 2) & ~(WS_ALIGN - 1);
      half0 = Arena(ctx, s, AR.base + o, h);
      half1 = Arena(ctx, ctx->lane1_stream, AR.base + o + h, left - h, &ctx->lane1);
    }
    const int64_t max_rec = two ? max_rec_of(half0) : max_rec0;
    const double per = (double)std::max<int64_t>(1, acc.nrec_all) / k0;
    const int32_t kr = pow2_floor(std::max<int64_t>(1, (int64_t)std::min<double>(n_samples, 0.9 * (double)max_rec / per)));
    std::vector<std::pair<int32_t, int32_t>> plan;
    for (int32_t s0 = k0; s0 < n_samples; s0 += kr) plan.emplace_back(s0, std::min<int32_t>(kr, n_samples - s0));
    if (!two || plan.size() < 2) {
      for (auto& ch : plan)
        if (int r = run_chunk(ch.first, ch.second, two ? half0 : AR, nullptr, s, max_rec, acc)) return done(r);
    } else {
      // lane 1 starts after the work queued so far on the caller's stream
      if (hipEventRecord(ctx->fork, s) != hipSuccess || hipStreamWaitEvent(ctx->lane1_stream, ctx->fork, 0) != hipSuccess)
        return done(fail(SHCI_ERR_HIP, "stream fork failed"));
      Job acc1{};
      acc1.res.mind = INFINITY;
      acc1.nbatch = 0;
      int r1 = SHCI_OK;
      std::string msg1;
      std::thread t1([&] {
        if (hipSetDevice(ctx->device) != hipSuccess) {
          r1 = fail(SHCI_ERR_HIP, "hipSetDevice failed");
        } else {
          for (size_t i = 1; i < plan.size() && r1 == SHCI_OK; i += 2)
            r1 = run_chunk(plan[i].first, plan[i].second, half1, &ctx->lane1, ctx->lane1_stream, max_rec, acc1);
        }
        if (r1) msg1 = shci_pt2_last_error();
        (void)hipStreamSynchronize(ctx->lane1_stream);
      });
      int r0 = SHCI_OK;
      for (size_t i = 0; i < plan.size() && r0 == SHCI_OK; i += 2)
        r0 = run_chunk(plan[i].first, plan[i].second, half0, nullptr, s, max_rec, acc);
      t1.join();
      // the caller's stream continues after lane 1's work
      if (hipEventRecord(ctx->join, ctx->lane1_stream) != hipSuccess || hipStreamWaitEvent(s, ctx->join, 0) != hipSuccess)
        return done(fail(SHCI_ERR_HIP, "stream join failed"));
      if (r0) return done(r0);
      if (r1) return done(fail(r1, "%s", msg1.c_str()));
      // lane 0 took the even chunks, lane 1 the odd ones
      add_stats(acc, acc1);
      acc.nbatch += acc1.nbatch;
    }
  }
  const int64_t chunks = acc.nbatch;
  std::vector<double> ps(n_samples);
  if (hipMemcpyAsync(ps.data(), per_sample, n_samples * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return done(fail(SHCI_ERR_HIP, "copy of per-sample results failed"));
  double m = 0.0;
  for (double v : ps) m += v;
  m /= n_samples;
  if (de2_de0) {
    std::vector<double> pd(n_samples);
    if (hipMemcpyAsync(pd.data(), psde0, n_samples * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return done(fail(SHCI_ERR_HIP, "copy of per-sample E0 derivatives failed"));
    double d = 0.0;
    for (double v : pd) d += v;
    *de2_de0 = d / n_samples;
  }
  double var = 0.0;
  for (double v : ps) var += (v - m) * (v - m);
  if (mean) *mean = m;
  if (sem) *sem = n_samples > 1 ? std::sqrt(var / (n_samples - 1)) / std::sqrt((double)n_samples) : 0.0;
  fill_stats(st, acc, acc.ms_gen + acc.ms_sort + acc.ms_reduce);
  if (st) st->n_chunks = (int32_t)chunks;  // sample chunks
  if (acc.res.nzero) return done(fail(SHCI_ERR_SINGULAR, "%lld kept determinants have E0 - H_aa == 0",
                                      (long long)acc.res.nzero));
  return done(SHCI_OK);
}

int shci_pt2_sample(shci_pt2_ctx* ctx, const uint64_t* dets, const double* c, int64_t n_det, double e0,
                    double eps2, double eps2_d, int32_t n_samples, int32_t n_draws, const uint32_t* draws,
                    uint64_t seed, int precision, void* ws, size_t ws_bytes, void* stream, double* per_sample,
                    double* mean, double* sem, shci_pt2_stats* st) {
  return sample_impl(ctx, dets, c, n_det, e0, eps2, eps2_d, n_samples, n_draws, draws, seed, precision, ws,
                     ws_bytes, stream, per_sample, mean, sem, st, nullptr, nullptr);
}

int shci_pt2_sample_grad(shci_pt2_ctx* ctx, const uint64_t* dets, const double* c, int64_t n_det, double e0,
                         double eps2, double eps2_d, int32_t n_samples, int32_t n_draws, const uint32_t* draws,
                         uint64_t seed, int precision, void* ws, size_t ws_bytes, void* stream, double* per_sample,
                         double* mean, double* sem, double* de2_dc, double* de2_de0, shci_pt2_stats* st) {
  if (!de2_dc) return fail(SHCI_ERR_ARG, "de2_dc is NULL");
  return sample_impl(ctx, dets, c, n_det, e0, eps2, eps2_d, n_samples, n_draws, draws, seed, precision, ws,
                     ws_bytes, stream, per_sample, mean, sem, st, de2_dc, de2_de0);
}

int shci_pt2_sample_batched(shci_pt2_ctx* ctx, const uint64_t* dets, const double* c, int64_t n_det, double e0,
                            double eps2, double eps2_d, int32_t n_samples, int32_t n_draws,
                            const uint32_t* draws, int32_t n_batches, const int32_t* sample_batch, uint64_t seed,
                            int precision, void* ws, size_t ws_bytes, void* stream, double* per_sample,
                            double* mean, double* sem, shci_pt2_stats* st) {
  return sample_impl(ctx, dets, c, n_det, e0, eps2, eps2_d, n_samples, n_draws, draws, seed, precision, ws,
                     ws_bytes, stream, per_sample, mean, sem, st, nullptr, nullptr, n_batches, sample_batch);
}

int shci_pt2_det_batches(shci_pt2_ctx* ctx, const uint64_t* dets, const double* c, int64_t n_det, double e0,
                         double eps2, double eps2_hi, int32_t n_batches, const int32_t* batches, int32_t n_list,
                         int precision, void* ws, size_t ws_bytes, void* stream, shci_pt2_batch* out,
                         shci_pt2_stats* st) {
  CHK(common_checks(ctx, dets, c, n_det, e0, eps2, precision));
  CHK(ws_check(ws, ws_bytes));
  if (!batches || !out || n_list < 1) return fail(SHCI_ERR_ARG, "batches and out must be non-NULL, n_list >= 1");
  if (n_batches < 1 || n_batches > 65536 || (n_batches & (n_batches - 1)))
    return fail(SHCI_ERR_ARG, "n_batches must be a power of two in [1, 65536]");
  if (!(eps2_hi >= eps2)) return fail(SHCI_ERR_ARG, "eps2_hi must be >= eps2 (INFINITY for one threshold)");
  for (int32_t k = 0; k < n_list; ++k)
    if (batches[k] < 0 || batches[k] >= n_batches) return fail(SHCI_ERR_ARG, "batch index out of range");
  Arena AR(ctx, static_cast<hipStream_t>(stream), ws, ws_bytes);
  Job proto{};
  proto.ctx = ctx;
  proto.ar = &AR;
  proto.st = static_cast<hipStream_t>(stream);
  proto.dets = dets;
  proto.c = c;
  proto.ndet = n_det;
  proto.e0 = e0;
  proto.eps2 = eps2;
  proto.eps2_d = eps2_hi;
  proto.precision = precision;
  proto.sample = false;
  proto.sbits = 0;
  proto.nsamp = 1;
  proto.n_items = n_det;
  const int kw = key_words(ctx->T.n, 0);
  proto.max_records = (AR.caller() && ctx->rec_limit == 0)
                          ? REC_CAP_AUTO
                          : record_budget(AR, record_bytes(kw, precision == SHCI_FP32C ? 4 : 8, false, false));
  Job acc{};
  acc.res.mind = INFINITY;
  for (int32_t k = 0; k < n_list; ++k) {
    Job J = proto;
    J.bmask = (uint32_t)(n_batches - 1);
    J.bsel = (uint32_t)batches[k];
    const int r = dispatch(J);
    if (r == JOB_TOO_BIG)
      return fail(SHCI_ERR_WORKSPACE, "batch %d has %lld terms, above the %lld records that fit; use more batches",
                  batches[k], (long long)J.nrec, (long long)J.max_records_eff);
    if (r) return r;
    out[k].sum = J.res.e2;
    out[k].sumsq = J.res.e2sq;
    out[k].n_unique = J.res.nuniq;
    out[k].n_terms = J.res.nterm;
    acc.res.nterm += J.res.nterm;
    acc.res.ngen += J.res.ngen;
    acc.res.nuniq += J.res.nuniq;
    acc.res.nintr += J.res.nintr;
    acc.res.nzero += J.res.nzero;
    acc.res.mind = std::min(acc.res.mind, J.res.mind);
    acc.nbucket = std::max(acc.nbucket, J.nbucket);
    acc.ms_gen += J.ms_gen;
    acc.ms_sort += J.ms_sort;
    acc.ms_reduce += J.ms_reduce;
    acc.ms_k_count += J.ms_k_count;
    acc.ms_k_write += J.ms_k_write;
    acc.ms_k_reduce += J.ms_k_reduce;
    acc.ms_k_part += J.ms_k_part;
    acc.n_part += J.n_part;
    acc.n_part_rec += J.n_part_rec;
    acc.nrec += J.nrec;
    acc.kw = J.kw;
    acc.vbytes = J.vbytes;
  }
  acc.nbatch = n_list;
  fill_stats(st, acc, acc.ms_gen + acc.ms_sort + acc.ms_reduce);
  if (acc.res.nzero) return fail(SHCI_ERR_SINGULAR, "%lld kept determinants have E0 - H_aa == 0",
                                 (long long)acc.res.nzero);
  return SHCI_OK;
}

int shci_pt2_three_step(shci_pt2_ctx* ctx, const uint64_t* dets, const double* c, int64_t n_det, double e0,
                        double eps2_dtm, double eps2_psto, double eps2, double target_error, int32_t nb_psto,
                        int32_t nb_sto, int32_t n_samples, int32_t n_draws, const uint32_t* draws,
                        const int32_t* sample_batch, uint64_t seed, int precision, void* ws, size_t ws_bytes,
                        void* stream, double* per_sample, shci_pt2_3step_result* res) {
  if (!res || !per_sample) return fail(SHCI_ERR_ARG, "res and per_sample must be non-NULL");
  if (!(eps2 <= eps2_psto && eps2_psto <= eps2_dtm)) return fail(SHCI_ERR_ARG, "need eps2 <= eps2_psto <= eps2_dtm");
  if (!(target_error > 0.0)) return fail(SHCI_ERR_ARG, "target_error must be > 0");
  if (nb_psto < 1 || nb_sto < 1) return fail(SHCI_ERR_ARG, "nb_psto and nb_sto must be >= 1");
  *res = shci_pt2_3step_result{};
  // 1. deterministic step at eps2_dtm, every batch of P (hash batches when
  //    the records do not fit)
  CHK(shci_pt2_det(ctx, dets, c, n_det, e0, eps2_dtm, precision, ws, ws_bytes, stream, &res->e2_dtm, nullptr,
                   nullptr));
  // 2. pseudo-stochastic step: batches of P in order; per batch the
  //    corrections (A(eps2_psto)^2 - A(eps2_dtm)^2) / D of its unique a.  The
  //    total is estimated from the evaluated a; its standard error is that of
  //    the sum over the a not yet evaluated.  Stop below 40% of the target.
  double S = 0.0, SS = 0.0;
  int64_t nev = 0;
  int32_t b = 0;
  double est = 0.0, sig = 0.0;
  for (; b < nb_psto;) {
    shci_pt2_batch o{};
    const int32_t idx = b;
    CHK(shci_pt2_det_batches(ctx, dets, c, n_det, e0, eps2_psto, eps2_dtm, nb_psto, &idx, 1, precision, ws,
                             ws_bytes, stream, &o, nullptr));
    ++b;
    S += o.sum;
    SS += o.sumsq;
    nev += o.n_unique;
    if (b == nb_psto || nev == 0) {
      est = S * (double)nb_psto / (double)b;
      sig = 0.0;
      if (b == nb_psto) break;
      continue;
    }
    const double mean = S / (double)nev;
    const double var = std::max(0.0, SS / (double)nev - mean * mean);
    const double nrest = (double)nev * ((double)nb_psto / (double)b - 1.0);
    est = S + nrest * mean;
    sig = std::sqrt(nrest * var);
    if (sig < 0.4 * target_error) break;
  }
  res->e2_psto = est;
  res->err_psto = sig;
  res->psto_batches_used = b;
  // 3. stochastic step: samples of V, one random batch of P per sample
  double mean = 0.0, sem = 0.0;
  CHK(shci_pt2_sample_batched(ctx, dets, c, n_det, e0, eps2, eps2_psto, n_samples, n_draws, draws, nb_sto,
                              sample_batch, seed, precision, ws, ws_bytes, stream, per_sample, &mean, &sem,
                              nullptr));
  res->e2_sto = mean;
  res->err_sto = sem;
  res->e2 = res->e2_dtm + res->e2_psto + res->e2_sto;
  res->err = std::sqrt(res->err_psto * res->err_psto + res->err_sto * res->err_sto);
  return SHCI_OK;
}

int shci_pt2_select(shci_pt2_ctx* ctx, const uint64_t* dets, const double* c, int64_t n_det, double e0,
                double eps_gen, int mode, double threshold, int precision, void* stream, uint64_t* out_keys,
                double* out_val, int64_t cap, int64_t* n_out, shci_pt2_stats* st) {
  if (!ctx) return fail(SHCI_ERR_ARG, "ctx is NULL");
  if (mode != SHCI_SELECT_HCI && mode != SHCI_SELECT_CIPSI) return fail(SHCI_ERR_ARG, "unknown selection mode");
  if (!out_keys || !out_val || !n_out || cap < 1) return fail(SHCI_ERR_ARG, "out_keys, out_val, n_out, cap >= 1");
  if (mode == SHCI_SELECT_CIPSI && !(threshold >= 0.0)) return fail(SHCI_ERR_ARG, "threshold must be >= 0");
  hipStream_t s = static_cast<hipStream_t>(stream);
  // every unique a of the pass, exported into the context's selection buffer
  uint64_t *k, *pos;
  double *A, *D, *val;
  int32_t* cnt;
  uint32_t* flag;
  ScanTmp sc;
  Arena AR(ctx, s, nullptr, 0);
  CHK(carve_region(AR, SL_SEL, [&](Carver& cv) {
    k = cv.take<uint64_t>(4 * cap);
    A = cv.take<double>(cap);
    D = cv.take<double>(cap);
    cnt = cv.take<int32_t>(cap);
    flag = cv.take<uint32_t>(cap + 1);
    val = cv.take<double>(cap);
    pos = cv.take<uint64_t>(cap + 1);
    sc.carve(cv, cap + 1);
  }));
  shci_pt2_export ex{};
  ex.u_keys = k;
  ex.u_A = A;
  ex.u_D = D;
  ex.u_cnt = cnt;
  ex.u_cap = cap;
  double e2 = 0.0;
  int r = shci_pt2_det(ctx, dets, c, n_det, e0, eps_gen, precision, nullptr, 0, stream, &e2, st, &ex);
  if (r) return r;
  if (ex.u_n > cap)
    return fail(SHCI_ERR_WORKSPACE, "%lld perturbative determinants exceed cap = %lld", (long long)ex.u_n,
                (long long)cap);
  const int64_t nu = ex.u_n;
  *n_out = 0;
  if (nu == 0) return SHCI_OK;
  const int grid = (int)std::min<int64_t>(4096, (nu + 255) / 256);
  k_select_flags<<<grid, 256, 0, s>>>(A, D, nu, mode, threshold, flag, val);
  r = scan_exclusive<uint32_t, uint64_t>(flag, pos, nu, sc, pos + nu, s);
  if (r) return r;
  k_select_compact<<<grid, 256, 0, s>>>(k, val, flag, pos, nu, out_keys, out_val);
  uint64_t h = 0;
  if (hipMemcpyAsync(&h, pos + nu, sizeof h, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return fail(SHCI_ERR_HIP, "selection count copy failed");
  *n_out = (int64_t)h;
  return SHCI_OK;
}

int shci_pt2_alias_table(shci_pt2_ctx* ctx, const double* c, int64_t n_det, void* ws, size_t ws_bytes,
                         void* stream, uint64_t* threshold, uint32_t* alias) {
  if (!ctx || !c || !threshold || !alias) return fail(SHCI_ERR_ARG, "ctx, c, threshold and alias must be non-NULL");
  if (n_det < 1 || n_det >= (int64_t)0xffffffffll) return fail(SHCI_ERR_ARG, "n_det must be in [1, 2^32 - 1)");
  CHK(ws_check(ws, ws_bytes));
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  Arena AR(ctx, s, ws, ws_bytes);
  k_fill_u32<<<1, 64, 0, s>>>(ctx->dflag, 4, 0u);
  CHK(build_alias(AR, c, n_det, threshold, alias, s));
  uint32_t hf = 0;
  HIPCHK(hipMemcpyAsync(&hf, ctx->dflag, 4, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (hf & 2u) return fail(SHCI_ERR_NONFINITE, "c contains a non-finite value");
  if (hf & 64u) return fail(SHCI_ERR_NONFINITE, "every coefficient is zero");
  return SHCI_OK;
}

int shci_pt2_draws(shci_pt2_ctx* ctx, const double* c, int64_t n_det, uint64_t seed, int32_t n_samples,
                   int32_t n_draws, void* ws, size_t ws_bytes, void* stream, uint32_t* draws) {
  if (!ctx || !c || !draws) return fail(SHCI_ERR_ARG, "ctx, c and draws must be non-NULL");
  if (n_det < 1 || n_det >= (int64_t)0xffffffffll) return fail(SHCI_ERR_ARG, "n_det must be in [1, 2^32 - 1)");
  if (n_samples < 1 || n_draws < 1) return fail(SHCI_ERR_ARG, "need n_samples >= 1 and n_draws >= 1");
  if ((int64_t)n_samples * n_draws >= ((int64_t)1 << 31))
    return fail(SHCI_ERR_ARG, "n_samples * n_draws must be < 2^31");
  CHK(ws_check(ws, ws_bytes));
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  Arena AR(ctx, s, ws, ws_bytes);
  k_fill_u32<<<1, 64, 0, s>>>(ctx->dflag, 4, 0u);
  CHK(seed_draws(AR, c, n_det, seed, n_samples, n_draws, draws, s));
  uint32_t hf = 0;
  HIPCHK(hipMemcpyAsync(&hf, ctx->dflag, 4, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (hf & 2u) return fail(SHCI_ERR_NONFINITE, "c contains a non-finite value");
  if (hf & 64u) return fail(SHCI_ERR_NONFINITE, "every coefficient is zero");
  return SHCI_OK;
}

int shci_pt2_hc(shci_pt2_ctx* ctx, const uint64_t* dets, const double* c, int64_t n_det, void* stream,
                double* y, uint32_t* n_conn, double* e_var, shci_pt2_stats* st) {
  if (!ctx || !dets || !c || !y) return fail(SHCI_ERR_ARG, "ctx, dets, c and y must be non-NULL");
  if (n_det < 1 || n_det >= (int64_t)0x7fffffff) return fail(SHCI_ERR_ARG, "n_det must be in [1, 2^31 - 1)");
  if (st) *st = shci_pt2_stats{};
  hipStream_t s = static_cast<hipStream_t>(stream);
  const Tables& T = ctx->T;
  const int64_t n = n_det;
  const uint64_t cap = 1ull << ceil_log2((uint64_t)(2 * n));
  const int64_t ntiles = (n + PAIR_TILE - 1) / PAIR_TILE;
  int passes = 0;
  while (passes < 4 && ((uint64_t)(n - 1) >> (8 * passes)) != 0) ++passes;
  if (passes == 0) passes = 1;
  // workspace: string tables, groups, two pair-sort buffer sets per spin,
  // histograms, group starts, singles counts and offsets
  struct Plan {
    uint32_t *slot[2], *grp[2], *k0[2], *v0[2], *k1[2], *v1[2], *hist, *hoffs, *scnt[2], *cnt_tmp, *pval;
    uint64_t *start[2], *soff[2], *tot, *oth0[2], *oth1[2], *pkey;
    uint32_t* othf[2];
    double* dots;
    ScanTmp sh, ss;
  } P{};
  auto plan = [&](Carver& cv) {
    for (int sp = 0; sp < 2; ++sp) {
      P.slot[sp] = cv.take<uint32_t>(cap);
      P.grp[sp] = cv.take<uint32_t>(n);
      P.k0[sp] = cv.take<uint32_t>(n);
      P.v0[sp] = cv.take<uint32_t>(n);
      P.k1[sp] = cv.take<uint32_t>(n);
      P.v1[sp] = cv.take<uint32_t>(n);
      P.start[sp] = cv.take<uint64_t>(n + 1);
      P.scnt[sp] = cv.take<uint32_t>(n + 1);
      P.soff[sp] = cv.take<uint64_t>(n + 1);
      P.oth0[sp] = cv.take<uint64_t>(n);
      P.oth1[sp] = cv.take<uint64_t>(n);
      P.othf[sp] = cv.take<uint32_t>(n);
    }
    P.pkey = cv.take<uint64_t>(cap);
    P.pval = cv.take<uint32_t>(cap);
    P.hist = cv.take<uint32_t>(256 * ntiles);
    P.hoffs = cv.take<uint32_t>(256 * ntiles);
    P.cnt_tmp = cv.take<uint32_t>(n);
    P.tot = cv.take<uint64_t>(2);
    P.dots = cv.take<double>(2);
    P.sh.carve(cv, 256 * ntiles);
    P.ss.carve(cv, n + 1);
  };
  // the context's grow-only buffers (no allocation once they are large enough)
  Arena AR(ctx, s, nullptr, 0);
  CHK(carve_region(AR, SL_HC, plan));
  auto done = [&](int code) {
    (void)hipStreamSynchronize(s);
    return code;
  };
  const int g1 = (int)((n + 255) / 256);
  const int gw = (int)std::min<int64_t>((n + 3) / 4, (int64_t)num_cus(ctx->device) * 16);
  HIPCHK(hipEventRecord(ctx->ev[0], s));
  k_fill_u32<<<1, 64, 0, s>>>(ctx->dflag, 4, 0u);
  k_validate<<<g1, 256, 0, s>>>(dets, c, n, T.n, T.na, T.nb, ctx->dflag);
  for (int sp = 0; sp < 2; ++sp) {
    StrTab tab{P.slot[sp], cap - 1};
    k_fill_u32<<<(int)std::min<uint64_t>(4096, (cap + 255) / 256), 256, 0, s>>>(P.slot[sp], (int64_t)cap, STR_EMPTY);
    k_str_insert<<<g1, 256, 0, s>>>(dets, n, sp, tab);
    k_str_group<<<g1, 256, 0, s>>>(dets, n, sp, tab, P.grp[sp]);
    // members of each group in index order: stable sort of (group, index)
    k_pair_init<<<g1, 256, 0, s>>>(P.grp[sp], n, P.k0[sp], P.v0[sp]);
    uint32_t *kin = P.k0[sp], *vin = P.v0[sp], *kout = P.k1[sp], *vout = P.v1[sp];
    const int pg = (int)((ntiles + 3) / 4);
    for (int pass = 0; pass < passes; ++pass) {
      k_pair_count<<<pg, 256, 0, s>>>(kin, n, 8 * pass, ntiles, P.hist);
      int r = scan_exclusive<uint32_t, uint32_t>(P.hist, P.hoffs, 256 * ntiles, P.sh, nullptr, s);
      if (r) return done(r);
      k_pair_place<<<pg, 256, 0, s>>>(kin, vin, n, 8 * pass, ntiles, P.hoffs, kout, vout);
      std::swap(kin, kout);
      std::swap(vin, vout);
    }
    // kin: sorted groups, vin: members
    P.k0[sp] = kin;
    P.v0[sp] = vin;
    k_bucket_bounds<<<(int)std::min<int64_t>(8192, (n + 256) / 256), 256, 0, s>>>(kin, n, n, P.start[sp]);
    // the other-spin string of each member, in member order
    k_pack_other<<<g1, 256, 0, s>>>(vin, dets, n, 1 - sp, P.oth0[sp], P.oth1[sp], P.othf[sp]);
  }
  // (alpha group, beta group) -> determinant
  PairTab pt{P.pkey, P.pval, cap - 1};
  k_fill_u64<<<(int)std::min<uint64_t>(4096, (cap + 255) / 256), 256, 0, s>>>(P.pkey, (int64_t)cap, PAIR_EMPTY);
  k_fill_u32<<<(int)std::min<uint64_t>(4096, (cap + 255) / 256), 256, 0, s>>>(P.pval, (int64_t)cap, STR_EMPTY);
  k_pairtab_insert<<<g1, 256, 0, s>>>(P.grp[0], P.grp[1], n, pt);
  // alpha- and beta-singles lists of the groups
  SinglesArgs sa[2];
  uint64_t nsl[2] = {0, 0};
  for (int sp = 0; sp < 2; ++sp) {
    sa[sp] = SinglesArgs{dets, n, T.n, sp ? T.nb : T.na, sp, StrTab{P.slot[sp], cap - 1}, P.grp[sp], P.scnt[sp],
                         P.soff[sp], nullptr};
    k_fill_u32<<<g1 + 1, 256, 0, s>>>(P.scnt[sp], n + 1, 0u);
    k_str_singles<false><<<gw, 256, 0, s>>>(sa[sp]);
    int r = scan_exclusive<uint32_t, uint64_t>(P.scnt[sp], P.soff[sp], n + 1, P.ss, nullptr, s);
    if (r) return done(r);
  }
  uint32_t hf = 0;
  if (hipMemcpyAsync(&nsl[0], P.soff[0] + n, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipMemcpyAsync(&nsl[1], P.soff[1] + n, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipMemcpyAsync(&hf, ctx->dflag, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return done(fail(SHCI_ERR_HIP, "string list preparation failed"));
  if (hf & 1u) return done(fail(SHCI_ERR_DET, "a determinant has a wrong electron count or an orbital >= n_orb"));
  if (hf & 2u) return done(fail(SHCI_ERR_NONFINITE, "c holds a NaN or Inf"));
  for (int sp = 0; sp < 2; ++sp) {
    void* lp = nullptr;
    if (int r = AR.take(sp ? SL_HCL1 : SL_HCL0, std::max<uint64_t>(1, nsl[sp]) * sizeof(uint32_t), &lp))
      return done(r);
    sa[sp].list = static_cast<uint32_t*>(lp);
    if (nsl[sp]) k_str_singles<true><<<gw, 256, 0, s>>>(sa[sp]);
  }
  HcArgs ha{};
  ha.T = T;
  ha.dets = dets;
  ha.c = c;
  ha.nd = n;
  ha.grpA = P.grp[0];
  ha.grpB = P.grp[1];
  ha.memA = P.v0[0];
  ha.memB = P.v0[1];
  ha.startA = P.start[0];
  ha.startB = P.start[1];
  ha.soff = P.soff[0];
  ha.slist = sa[0].list;
  ha.soffB = P.soff[1];
  ha.slistB = sa[1].list;
  ha.bOfA0 = P.oth0[0];
  ha.bOfA1 = P.oth1[0];
  ha.aOfB0 = P.oth0[1];
  ha.aOfB1 = P.oth1[1];
  ha.bOfAf = P.othf[0];
  ha.aOfBf = P.othf[1];
  ha.pt = pt;
  ha.y = y;
  ha.nconn = n_conn ? n_conn : P.cnt_tmp;
  ha.flag = ctx->dflag;
  HIPCHK(hipEventRecord(ctx->ev[1], s));
  k_hc_rows<<<gw, 256, 0, s>>>(ha);
  HIPCHK(hipEventRecord(ctx->ev[2], s));
  k_sum_u32<<<1, 1024, 0, s>>>(ha.nconn, n, P.tot);
  k_dot2<<<1, 1024, 0, s>>>(c, y, n, P.dots);
  HIPCHK(hipEventRecord(ctx->ev[3], s));
  HIPCHK(hipGetLastError());
  double dots[2] = {0.0, 0.0};
  uint64_t nconn_tot = 0;
  if (hipMemcpyAsync(dots, P.dots, sizeof dots, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipMemcpyAsync(&nconn_tot, P.tot, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipMemcpyAsync(&hf, ctx->dflag, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return done(fail(SHCI_ERR_HIP, "H c failed: %s", hipGetErrorString(hipGetLastError())));
  if (hf & 4u) return done(fail(SHCI_ERR_DUP, "the variational space contains a duplicate determinant"));
  if (e_var) *e_var = dots[0] / dots[1];
  if (st) {
    float a = 0.f, b = 0.f, t = 0.f;
    (void)hipEventElapsedTime(&a, ctx->ev[0], ctx->ev[1]);
    (void)hipEventElapsedTime(&b, ctx->ev[1], ctx->ev[2]);
    (void)hipEventElapsedTime(&t, ctx->ev[0], ctx->ev[3]);
    st->n_terms = (int64_t)nconn_tot;
    st->n_records = (int64_t)(nsl[0] + nsl[1]);
    st->ms_gen = a;
    st->ms_reduce = b;
    st->ms_total = t;
  }
  return done(SHCI_OK);
}

}  // extern "C"
