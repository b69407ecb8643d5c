// Integral-derived tables, built once per integral set on the device.
//
//  * Heat-bath tables (paper, section II.A: for every pair of occupied
//    orbitals, the magnitudes of all double-excitation matrix elements from it,
//    sorted in decreasing order with their target pair, so that a walk can
//    stop at the first entry below the cutoff; section II.B reuses them for
//    eps2).  Keyed by spatial pair:
//      same spin  p<q   : entries r<s, r,s not in {p,q}, value (pr|qs)-(ps|qr)
//      opposite   (p,q) : entries r != p, s != q,        value (pr|qs)
//    Each key's list has a fixed length (lss or los) and is sorted by
//    decreasing |value|, ties by ascending entry index (enumeration order).
//  * Single-excitation tables, layout [k][p][r]:
//      sD = (pr|kk) - (pk|kr),  sJ = (pr|kk),
//    and an upper bound of |h_pr + sum_k ...| used to skip hopeless singles.
//  * Diagonal tables (pp|qq) and (pp|qq) - (pq|qp) for H_aa.
#include "kernels.hpp"

namespace shci {

__device__ __forceinline__ double eri_at(const double* eri, int n, int p, int q, int r, int s) {
  return eri[(((size_t)p * n + q) * n + r) * n + s];
}

__global__ void k_check_finite(const double* x, int64_t m, uint32_t* flag) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x) {
    double v = x[i];
    if (!(v - v == 0.0)) atomicOr(flag, 1u);
  }
}

__global__ void k_singles_tables(const double* h1, const double* eri, int n, double* sD,
                                 double* sJ) {
  int64_t m = (int64_t)n * n * n;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < m;
       t += (int64_t)gridDim.x * blockDim.x) {
    int r = (int)(t % n);
    int p = (int)((t / n) % n);
    int k = (int)(t / ((int64_t)n * n));
    double j = eri_at(eri, n, p, r, k, k);
    double x = eri_at(eri, n, p, k, k, r);
    sJ[t] = j;
    sD[t] = j - x;
  }
}

__global__ void k_singles_bound(const double* h1, const double* sD, const double* sJ, int n,
                                double* ub) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * n) return;
  int p = t / n, r = t % n;
  double acc = fabs(h1[(size_t)p * n + r]);
  for (int k = 0; k < n; ++k) {
    size_t o = ((size_t)k * n + p) * n + r;
    acc += fabs(sD[o]) + fabs(sJ[o]);
  }
  // the evaluated element adds at most 2n-1 rounded terms; 1e-9 covers the rounding
  ub[t] = acc * (1.0 + 1e-9);
}

// h_pp; (pp|qq) on the triangle p <= q at q(q+1)/2 + p; (pp|qq) - (pq|qp) on
// p < q at q(q-1)/2 + p
__global__ void k_diag_tables(const double* h1, const double* eri, int n, double* hpp, double* jtri,
                              double* sstri) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * n) return;
  int p = t / n, q = t % n;
  if (p > q) return;
  double j = eri_at(eri, n, p, p, q, q);
  jtri[q * (q + 1) / 2 + p] = j;
  if (p < q) sstri[q * (q - 1) / 2 + p] = j - eri_at(eri, n, p, q, q, p);
  if (p == q) hpp[p] = h1[(size_t)p * n + p];
}

// entry e of a same-spin key (p<q): colex pair (x<y) of the n-2 orbitals
// outside {p,q}; e = y(y-1)/2 + x
__device__ __forceinline__ void ss_entry(int e, int p, int q, int& r, int& s) {
  int y = (int)floor((1.0 + sqrt(1.0 + 8.0 * (double)e)) * 0.5);
  while (y * (y - 1) / 2 > e) --y;
  while ((y + 1) * y / 2 <= e) ++y;
  int x = e - y * (y - 1) / 2;
  r = x + (x >= p);
  r += (r >= q);
  s = y + (y >= p);
  s += (s >= q);
}

// entry e of an opposite-spin key (p,q): e = xr*(n-1) + xs, r = xr skipping p,
// s = xs skipping q
__device__ __forceinline__ void os_entry(int e, int n, int p, int q, int& r, int& s) {
  int xr = e / (n - 1), xs = e % (n - 1);
  r = xr + (xr >= p);
  s = xs + (xs >= q);
}

__device__ __forceinline__ void key_pair(int key, int nss, int n, int& p, int& q, bool& same) {
  if (key < nss) {
    int y = (int)floor((1.0 + sqrt(1.0 + 8.0 * (double)key)) * 0.5);
    while (y * (y - 1) / 2 > key) --y;
    while ((y + 1) * y / 2 <= key) ++y;
    p = key - y * (y - 1) / 2;
    q = y;
    same = true;
  } else {
    int k = key - nss;
    p = k / n;
    q = k % n;
    same = false;
  }
}

// One block per key: values in enumeration order, then an exact rank sort in
// LDS (rank = entries with larger magnitude + equal magnitude and smaller
// index), written back in sorted order.
__global__ void __launch_bounds__(256) k_heatbath(const double* eri, int n, int nss, int64_t lss,
                                                  int64_t los, double* hb_val, uint16_t* hb_rs,
                                                  double* hb_max) {
  extern __shared__ double s_mag[];
  const int key = blockIdx.x;
  int p, q;
  bool same;
  key_pair(key, nss, n, p, q, same);
  const int L = (int)(same ? lss : los);
  const int64_t off = same ? (int64_t)key * lss : (int64_t)nss * lss + (int64_t)(key - nss) * los;
  for (int e = threadIdx.x; e < L; e += blockDim.x) {
    int r, s;
    double v;
    if (same) {
      ss_entry(e, p, q, r, s);
      v = eri_at(eri, n, p, r, q, s) - eri_at(eri, n, p, s, q, r);
    } else {
      os_entry(e, n, p, q, r, s);
      v = eri_at(eri, n, p, r, q, s);
    }
    s_mag[e] = fabs(v);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < L; e += blockDim.x) {
    const double m = s_mag[e];
    int rank = 0;
    for (int f = 0; f < L; ++f) {
      const double o = s_mag[f];
      rank += (o > m) || (o == m && f < e);
    }
    int r, s;
    double v;
    if (same) {
      ss_entry(e, p, q, r, s);
      v = eri_at(eri, n, p, r, q, s) - eri_at(eri, n, p, s, q, r);
    } else {
      os_entry(e, n, p, q, r, s);
      v = eri_at(eri, n, p, r, q, s);
    }
    hb_val[off + rank] = v;
    hb_rs[off + rank] = (uint16_t)(r | (s << 8));
    if (rank == 0) hb_max[key] = m;
  }
  if (L == 0 && threadIdx.x == 0) hb_max[key] = 0.0;
}

__global__ void k_mag_clear(double* h) {
  for (int x = threadIdx.x; x < 144; x += blockDim.x) h[x] = 0.0;
}

// histogram of log2 |value| per table kind, then cumulative from the top
// (entries with |value| >= 2^e); used to size work items
__global__ void k_mag_hist2(const double* hb_val, int64_t n_ss_entries, int64_t n_entries, double* hist) {
  __shared__ unsigned int loc[144];
  for (int x = threadIdx.x; x < 144; x += blockDim.x) loc[x] = 0u;
  __syncthreads();
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n_entries;
       e += (int64_t)gridDim.x * blockDim.x) {
    const double m = fabs(hb_val[e]);
    if (!(m > 0.0)) continue;
    int x = ilogb(m);
    x = x < -64 ? -64 : (x > 7 ? 7 : x);
    atomicAdd(&loc[(e < n_ss_entries ? 0 : 72) + x + 64], 1u);
  }
  __syncthreads();
  for (int x = threadIdx.x; x < 144; x += blockDim.x)
    if (loc[x]) atomicAdd(&hist[x], (double)loc[x]);
}

__global__ void k_mag_cum2(double* hist) {
  if (threadIdx.x < 2) {
    double acc = 0.0;
    for (int x = 71; x >= 0; --x) {
      acc += hist[threadIdx.x * 72 + x];
      hist[threadIdx.x * 72 + x] = acc;
    }
  }
}

// Singles elements of the reference determinant R for every p, r and spin s:
// h_pr + sum_{k in R_s, k != p} sD[k][p][r] + sum_{k in R_s'} sJ[k][p][r]
// (any order; the generator uses them only as a filter with a margin).
__global__ void k_singles_ref(const uint64_t* ref, const double* h1, const double* sD, const double* sJ,
                              int n, double* fref) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 2 * n * n) return;
  const int sp = t / (n * n), p = (t / n) % n, r = t % n;
  const size_t nn = (size_t)n * n, pr = (size_t)p * n + r;
  double h = h1[pr];
  for (int k = 0; k < n; ++k) {
    const bool in_a = (ref[k >> 6] >> (k & 63)) & 1ull;
    const bool in_b = (ref[2 + (k >> 6)] >> (k & 63)) & 1ull;
    const bool same = sp == 0 ? in_a : in_b;
    const bool other = sp == 0 ? in_b : in_a;
    if (same && k != p) h += sD[k * nn + pr];
    if (other) h += sJ[k * nn + pr];
  }
  fref[t] = h;
}

void singles_ref(const Tables& T, const uint64_t* ref, hipStream_t st) {
  const int m = 2 * T.n * T.n;
  k_singles_ref<<<(m + 255) / 256, 256, 0, st>>>(ref, T.h1, T.sD, T.sJ, T.n, T.fref);
}

// (pq|rs) folded by the 8-fold symmetry: entry k of the (P, Q) triangle with
// P = pq and Q = rs pair indices (the integrals are symmetric bit for bit, so
// any representative is exact)
__global__ void k_eri8(const double* eri, int n, int64_t npair, double* g8) {
  const int64_t tot = npair * (npair + 1) / 2;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < tot; k += (int64_t)gridDim.x * blockDim.x) {
    int64_t P, Q, p, q, r, s;
    tri_split(k, P, Q);
    tri_split(P, p, q);
    tri_split(Q, r, s);
    g8[k] = eri_at(eri, n, (int)p, (int)q, (int)r, (int)s);
  }
}

int build_tables(Tables& T, const double* h1, const double* eri, hipStream_t st, uint32_t* dflag) {
  const int n = T.n;
  const int64_t n3 = (int64_t)n * n * n, n4 = n3 * n;
  k_check_finite<<<1024, 256, 0, st>>>(h1, (int64_t)n * n, dflag);
  k_check_finite<<<4096, 256, 0, st>>>(eri, n4, dflag);
  k_singles_tables<<<(int)((n3 + 255) / 256), 256, 0, st>>>(h1, eri, n, T.sD, T.sJ);
  k_singles_bound<<<(n * n + 255) / 256, 256, 0, st>>>(h1, T.sD, T.sJ, n, T.ubound);
  k_diag_tables<<<(n * n + 255) / 256, 256, 0, st>>>(h1, eri, n, T.hpp, T.jtri, T.sstri);
  const int nkeys = T.nss + n * n;
  const int64_t maxl = T.lss > T.los ? T.lss : T.los;
  size_t lds = (size_t)maxl * sizeof(double);
  if (lds < 8) lds = 8;
  if (hipFuncSetAttribute((const void*)k_heatbath, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)lds) != hipSuccess)
    return -1;
  k_heatbath<<<nkeys, 256, lds, st>>>(eri, n, T.nss, T.lss, T.los, T.hb_val, T.hb_rs, T.hb_max);
  k_mag_clear<<<1, 256, 0, st>>>(T.mag_cum);
  const int64_t nss_e = (int64_t)T.nss * T.lss, ntot = nss_e + (int64_t)n * n * T.los;
  k_mag_hist2<<<2048, 256, 0, st>>>(T.hb_val, nss_e, ntot, T.mag_cum);
  k_mag_cum2<<<1, 64, 0, st>>>(T.mag_cum);
  const int64_t npair = (int64_t)n * (n + 1) / 2;
  k_eri8<<<4096, 256, 0, st>>>(eri, n, npair, T.g8);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace shci
