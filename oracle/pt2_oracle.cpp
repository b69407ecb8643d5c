// CPU reference for the screened Epstein-Nesbet PT2 energy (TEST INFRASTRUCTURE).
//
// This file is the oracle: a plain, slow, brute-force implementation used only
// by the test-suite, the smoke check and the CPU-baseline timing.  It shares no
// code with the GPU library and is never called by it.
//
// What it computes (paper, section II.B):
//   * the Epstein-Nesbet partition H0 = H restricted to V plus diag(H_aa)
//     outside V (partition equation) fixes the denominator E0 - H_aa;
//   * the second-order energy sum_a (sum_i H_ai c_i)^2 / (E0 - H_aa) over the
//     perturbative space P, the determinants outside V connected to V by at
//     least one non-zero element (definition of P, section II; PT2 equation);
//   * the screened form, where only terms with |H_ai c_i| > eps2 enter the
//     inner sum (screened PT2 equation; the strict inequality reproduces
//     "non-zero element" at eps2 = 0);
//   * the stochastic estimator on given draws (stochastic PT2 equation, with
//     p_i = |c_i| / sum_j |c_j|, sampling-probability equation);
//   * the gradient dE2/dc_i = sum_a 2 H_ai A_a / D_a and dE2/dE0 =
//     -sum_a A_a^2 / D_a^2 at a frozen screening mask;
//   * helpers that build workload inputs: <c|H|c> and the MP1-like amplitudes
//     H_i0 / (E_HF - H_ii) of the doubles of the Hartree-Fock determinant;
//   * H c on the variational space, row by row over every pair (the product
//     that section III evaluates through alpha/beta string lists).
//
// Method: every single and double excitation of every variational determinant
// is enumerated by brute force (no heat-bath table, no early exit); matrix
// elements come from the Slater-Condon rules; terms are sorted by (a, i) and
// summed with Neumaier's compensated summation in i order; H_aa is evaluated
// from scratch.  All arithmetic is IEEE binary64 with no contraction
// (-ffp-contract=off).
//
// Conventions (readings of points the paper leaves open):
//   * real orbitals, chemists' notation (pq|rs), eri[((p*n+q)*n+r)*n+s];
//   * spin-orbital order alpha_0..alpha_{n-1}, beta_0..beta_{n-1}, so the sign
//     of a_r^+ a_p on a spin string S is (-1)^popcount(S strictly between p
//     and r) and opposite-spin signs factorise;
//   * a same-spin double p<q -> r<s is p->r followed by q->s;
//   * single excitation p->r in spin s:  h_pr + sum over occupied k != p, in
//     ascending spin-orbital order (alpha block, then beta block), of
//     (pr|kk) - (pk|kr) for same-spin k and (pr|kk) for opposite-spin k,
//     accumulated left to right starting from h_pr;
//   * determinant words (alpha_lo, alpha_hi, beta_lo, beta_hi); orbital p at
//     bit (p & 63) of word (p >> 6) of its spin (section V.A).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <quadmath.h>
#include <unordered_map>
#include <unordered_set>
#include <vector>
#include <omp.h>
#include <parallel/algorithm>

namespace {

struct Det {
  uint64_t w[4];
  bool operator==(const Det& o) const {
    return w[0] == o.w[0] && w[1] == o.w[1] && w[2] == o.w[2] && w[3] == o.w[3];
  }
  bool operator<(const Det& o) const {
    for (int k = 3; k >= 0; --k)
      if (w[k] != o.w[k]) return w[k] < o.w[k];
    return false;
  }
};

struct DetHash {
  size_t operator()(const Det& d) const {
    uint64_t h = 0x9e3779b97f4a7c15ull;
    for (int k = 0; k < 4; ++k) {
      h ^= d.w[k] + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2);
    }
    return (size_t)h;
  }
};

struct Neumaier {
  double s = 0.0, c = 0.0;
  void add(double x) {
    double t = s + x;
    if (std::fabs(s) >= std::fabs(x))
      c += (s - t) + x;
    else
      c += (x - t) + s;
    s = t;
  }
  double value() const { return s + c; }
};

struct System {
  int n, na, nb;
  const double* h1;
  const double* eri;
  double h(int p, int q) const { return h1[(size_t)p * n + q]; }
  double g(int p, int q, int r, int s) const {
    return eri[(((size_t)p * n + q) * n + r) * n + s];
  }
};

inline bool bit(const uint64_t* s, int p) { return (s[p >> 6] >> (p & 63)) & 1ull; }
inline void flip(uint64_t* s, int p) { s[p >> 6] ^= (1ull << (p & 63)); }

// number of occupied orbitals of spin string s strictly between p and r
// (population count of the string masked to the orbitals lo+1 .. hi-1)
inline int between(const uint64_t* s, int p, int r) {
  int lo = std::min(p, r), hi = std::max(p, r);
  if (hi - lo < 2) return 0;
  unsigned __int128 str = ((unsigned __int128)s[1] << 64) | s[0];
  unsigned __int128 mask = (((unsigned __int128)1 << hi) - 1) & ~((((unsigned __int128)1 << lo) << 1) - 1);
  unsigned __int128 v = str & mask;
  return __builtin_popcountll((uint64_t)v) + __builtin_popcountll((uint64_t)(v >> 64));
}

inline double sign_of(int parity) { return (parity & 1) ? -1.0 : 1.0; }

std::vector<int> occ_list(const uint64_t* s, int n) {
  std::vector<int> o;
  for (int p = 0; p < n; ++p)
    if (bit(s, p)) o.push_back(p);
  return o;
}
std::vector<int> virt_list(const uint64_t* s, int n) {
  std::vector<int> o;
  for (int p = 0; p < n; ++p)
    if (!bit(s, p)) o.push_back(p);
  return o;
}

// <D_i with p->r in spin `spin`|H|D_i>, without the sign
double single_value(const System& S, const Det& di, int spin, int p, int r) {
  double acc = S.h(p, r);
  for (int ks = 0; ks < 2; ++ks) {
    const uint64_t* str = &di.w[2 * ks];
    for (int k = 0; k < S.n; ++k) {
      if (!bit(str, k)) continue;
      if (ks == spin) {
        if (k == p) continue;
        acc = acc + (S.g(p, r, k, k) - S.g(p, k, k, r));
      } else {
        acc = acc + S.g(p, r, k, k);
      }
    }
  }
  return acc;
}

double diag_value(const System& S, const Det& d) {
  std::vector<int> oa = occ_list(&d.w[0], S.n), ob = occ_list(&d.w[2], S.n);
  double e = 0.0;
  for (int p : oa) e = e + S.h(p, p);
  for (int p : ob) e = e + S.h(p, p);
  for (size_t x = 0; x < oa.size(); ++x)
    for (size_t y = x + 1; y < oa.size(); ++y)
      e = e + (S.g(oa[x], oa[x], oa[y], oa[y]) - S.g(oa[x], oa[y], oa[y], oa[x]));
  for (size_t x = 0; x < ob.size(); ++x)
    for (size_t y = x + 1; y < ob.size(); ++y)
      e = e + (S.g(ob[x], ob[x], ob[y], ob[y]) - S.g(ob[x], ob[y], ob[y], ob[x]));
  for (int p : oa)
    for (int q : ob) e = e + S.g(p, p, q, q);
  return e;
}

// Generic matrix element <a|H|i> by the Slater-Condon rules, evaluated from the
// source determinant i (so that it is bit-identical to the enumeration below).
double hij(const System& S, const Det& a, const Det& i) {
  int nd[2], hole[2][2], part[2][2];
  int total = 0;
  for (int sp = 0; sp < 2; ++sp) {
    nd[sp] = 0;
    int nh = 0, np = 0;
    for (int p = 0; p < S.n; ++p) {
      bool bi = bit(&i.w[2 * sp], p), ba = bit(&a.w[2 * sp], p);
      if (bi && !ba) {
        if (nh < 2) hole[sp][nh] = p;
        ++nh;
      }
      if (!bi && ba) {
        if (np < 2) part[sp][np] = p;
        ++np;
      }
    }
    if (nh != np) return 0.0;
    nd[sp] = nh;
    total += nh;
  }
  if (total == 0) return diag_value(S, i);
  if (total > 2) return 0.0;
  if (total == 1) {
    int sp = nd[0] == 1 ? 0 : 1;
    int p = hole[sp][0], r = part[sp][0];
    double v = single_value(S, i, sp, p, r);
    return sign_of(between(&i.w[2 * sp], p, r)) * v;
  }
  if (nd[0] == 1 && nd[1] == 1) {
    int p = hole[0][0], r = part[0][0], q = hole[1][0], s = part[1][0];
    int par = between(&i.w[0], p, r) + between(&i.w[2], q, s);
    return sign_of(par) * S.g(p, r, q, s);
  }
  int sp = nd[0] == 2 ? 0 : 1;
  int p = hole[sp][0], q = hole[sp][1], r = part[sp][0], s = part[sp][1];
  uint64_t str[2] = {i.w[2 * sp], i.w[2 * sp + 1]};
  int par = between(str, p, r);
  flip(str, p);
  flip(str, r);
  par += between(str, q, s);
  return sign_of(par) * (S.g(p, r, q, s) - S.g(p, s, q, r));
}

struct Term {
  Det a;
  uint32_t i;
  double h;  // H_ai (t = h * c_i)
};

// Enumerate every single and double excitation a of det i with its H_ai.
template <class F>
void for_each_excitation(const System& S, const Det& di, F&& emit) {
  for (int sp = 0; sp < 2; ++sp) {
    const uint64_t* str = &di.w[2 * sp];
    std::vector<int> occ = occ_list(str, S.n), vir = virt_list(str, S.n);
    // singles
    for (int p : occ)
      for (int r : vir) {
        double v = single_value(S, di, sp, p, r);
        double hval = sign_of(between(str, p, r)) * v;
        Det a = di;
        flip(&a.w[2 * sp], p);
        flip(&a.w[2 * sp], r);
        emit(a, hval);
      }
    // same-spin doubles p<q -> r<s
    for (size_t x = 0; x < occ.size(); ++x)
      for (size_t y = x + 1; y < occ.size(); ++y)
        for (size_t u = 0; u < vir.size(); ++u)
          for (size_t v = u + 1; v < vir.size(); ++v) {
            int p = occ[x], q = occ[y], r = vir[u], s = vir[v];
            uint64_t s1[2] = {str[0], str[1]};
            int par = between(s1, p, r);
            flip(s1, p);
            flip(s1, r);
            par += between(s1, q, s);
            double hval = sign_of(par) * (S.g(p, r, q, s) - S.g(p, s, q, r));
            Det a = di;
            flip(&a.w[2 * sp], p);
            flip(&a.w[2 * sp], r);
            flip(&a.w[2 * sp], q);
            flip(&a.w[2 * sp], s);
            emit(a, hval);
          }
  }
  // opposite-spin doubles: p->r (alpha), q->s (beta)
  std::vector<int> oa = occ_list(&di.w[0], S.n), va = virt_list(&di.w[0], S.n);
  std::vector<int> ob = occ_list(&di.w[2], S.n), vb = virt_list(&di.w[2], S.n);
  for (int p : oa)
    for (int r : va) {
      int pa = between(&di.w[0], p, r);
      for (int q : ob)
        for (int s : vb) {
          int par = pa + between(&di.w[2], q, s);
          double hval = sign_of(par) * S.g(p, r, q, s);
          Det a = di;
          flip(&a.w[0], p);
          flip(&a.w[0], r);
          flip(&a.w[2], q);
          flip(&a.w[2], s);
          emit(a, hval);
        }
    }
}

inline bool kept(double hval, double c, double eps2) {
  return std::fabs(hval) * std::fabs(c) > eps2;
}

thread_local char g_err[256] = "";

int validate(const System& S, const Det* dets, const double* c, int64_t nd) {
  if (S.n < 1 || S.n > 128 || S.na < 0 || S.nb < 0 || S.na > S.n || S.nb > S.n) {
    snprintf(g_err, sizeof g_err, "bad shape n=%d na=%d nb=%d", S.n, S.na, S.nb);
    return -2;
  }
  std::unordered_set<Det, DetHash> seen;
  for (int64_t i = 0; i < nd; ++i) {
    const Det& d = dets[i];
    for (int sp = 0; sp < 2; ++sp) {
      int cnt = __builtin_popcountll(d.w[2 * sp]) + __builtin_popcountll(d.w[2 * sp + 1]);
      if (cnt != (sp ? S.nb : S.na)) {
        snprintf(g_err, sizeof g_err, "det %lld has wrong electron count", (long long)i);
        return -3;
      }
      for (int p = S.n; p < 128; ++p)
        if (bit(&d.w[2 * sp], p)) {
          snprintf(g_err, sizeof g_err, "det %lld uses orbital >= n", (long long)i);
          return -3;
        }
    }
    if (!seen.insert(d).second) {
      snprintf(g_err, sizeof g_err, "det %lld is a duplicate", (long long)i);
      return -4;
    }
    if (c && !std::isfinite(c[i])) {
      snprintf(g_err, sizeof g_err, "c[%lld] is not finite", (long long)i);
      return -5;
    }
  }
  return 0;
}

struct Unique {
  Det a;
  double A;      // sum of kept H_ai c_i
  double D;      // E0 - H_aa
  int64_t cnt;   // kept terms
  int64_t first; // index of its first term in the sorted term list
};

struct Result {
  std::vector<Term> terms;     // all kept terms (a in V included), sorted by (a, i)
  std::vector<uint8_t> in_v;   // per term
  std::vector<Unique> uniq;    // a not in V
  double e2 = 0.0, de2_de0 = 0.0;
  int64_t n_terms = 0, n_terms_gen = 0, n_intruder = 0, n_zero_denom = 0;
  double min_abs_denom = INFINITY;
  std::vector<double> grad;
};

// Batch of a determinant for the hash-batch decomposition of P (section IV):
// h mod n_batches, with h the 64-bit finaliser of MurmurHash3 (its published
// constants) chained over the ceil(2n/64) words of alpha | beta << n, starting
// from the first 64 bits of the fractional part of pi.  n_batches is a power
// of two, so h mod n_batches is h & (n_batches - 1).
static uint64_t murmur_fmix64(uint64_t k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdull;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ull;
  k ^= k >> 33;
  return k;
}

uint64_t batch_hash(const Det& d, int n) {
  // bits of alpha | beta << n, word by word
  uint64_t w[4] = {0, 0, 0, 0};
  for (int p = 0; p < n; ++p) {
    if (bit(&d.w[0], p)) w[p >> 6] |= 1ull << (p & 63);
    if (bit(&d.w[2], p)) w[(n + p) >> 6] |= 1ull << ((n + p) & 63);
  }
  uint64_t h = 0x243f6a8885a308d3ull;
  for (int j = 0; j < (2 * n + 63) / 64; ++j) h = murmur_fmix64(h ^ w[j]);
  return h;
}

void collect_terms(const System& S, const Det* dets, const double* c, int64_t nd, double eps2,
                   std::vector<Term>& out) {
  int nt = omp_get_max_threads();
  std::vector<std::vector<Term>> per(nt);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < nd; ++i) {
    auto& loc = per[omp_get_thread_num()];
    double ci = c[i];
    for_each_excitation(S, dets[i], [&](const Det& a, double hval) {
      if (kept(hval, ci, eps2)) loc.push_back(Term{a, (uint32_t)i, hval});
    });
  }
  size_t total = 0;
  for (auto& v : per) total += v.size();
  out.clear();
  out.reserve(total);
  for (auto& v : per) {
    out.insert(out.end(), v.begin(), v.end());
    std::vector<Term>().swap(v);
  }
  auto less = [](const Term& x, const Term& y) {
    if (x.a == y.a) return x.i < y.i;
    return x.a < y.a;
  };
  // sort by (a, i) (libstdc++ parallel mode: a multiway mergesort over threads)
  __gnu_parallel::sort(out.begin(), out.end(), less);
}

Result* run_det(const System& S, const Det* dets, const double* c, int64_t nd, double e0,
                double eps2, bool want_grad) {
  Result* R = new Result();
  std::unordered_set<Det, DetHash> V(dets, dets + nd);
  collect_terms(S, dets, c, nd, eps2, R->terms);
  R->n_terms_gen = (int64_t)R->terms.size();
  R->in_v.assign(R->terms.size(), 0);
  Neumaier e2, de0;
  size_t k = 0;
  while (k < R->terms.size()) {
    size_t j = k;
    while (j < R->terms.size() && R->terms[j].a == R->terms[k].a) ++j;
    const Det& a = R->terms[k].a;
    if (V.count(a)) {
      for (size_t m = k; m < j; ++m) R->in_v[m] = 1;
    } else {
      Neumaier A;
      for (size_t m = k; m < j; ++m) A.add(R->terms[m].h * c[R->terms[m].i]);
      double haa = diag_value(S, a);
      double D = e0 - haa;
      Unique u{a, A.value(), D, (int64_t)(j - k), (int64_t)k};
      if (D == 0.0) R->n_zero_denom++;
      if (D > 0.0) R->n_intruder++;
      R->min_abs_denom = std::min(R->min_abs_denom, std::fabs(D));
      e2.add(u.A * u.A / D);
      de0.add(-(u.A * u.A) / (D * D));
      R->n_terms += (int64_t)(j - k);
      R->uniq.push_back(u);
    }
    k = j;
  }
  R->e2 = e2.value();
  R->de2_de0 = de0.value();
  if (want_grad) {
    std::vector<Neumaier> g(nd);
    for (const Unique& u : R->uniq) {
      double ga = 2.0 * u.A / u.D;
      for (int64_t m = u.first; m < u.first + u.cnt; ++m) {
        const Term& t = R->terms[m];
        g[t.i].add(t.h * ga);
      }
    }
    R->grad.resize(nd);
    for (int64_t i = 0; i < nd; ++i) R->grad[i] = g[i].value();
  }
  return R;
}

}  // namespace

extern "C" {

const char* oracle_last_error() { return g_err; }

int oracle_max_threads() { return omp_get_max_threads(); }

double oracle_hij(int n, int na, int nb, const double* h1, const double* eri, const uint64_t* a,
                  const uint64_t* i) {
  System S{n, na, nb, h1, eri};
  Det da, di;
  std::memcpy(da.w, a, 32);
  std::memcpy(di.w, i, 32);
  return hij(S, da, di);
}

double oracle_diag(int n, int na, int nb, const double* h1, const double* eri, const uint64_t* d) {
  System S{n, na, nb, h1, eri};
  Det dd;
  std::memcpy(dd.w, d, 32);
  return diag_value(S, dd);
}

// Number of single+double excitations of one determinant, by enumeration.
int64_t oracle_count_excitations(int n, int na, int nb, const double* h1, const double* eri,
                                 const uint64_t* d) {
  System S{n, na, nb, h1, eri};
  Det dd;
  std::memcpy(dd.w, d, 32);
  int64_t cnt = 0;
  std::unordered_set<Det, DetHash> seen;
  bool unique = true;
  for_each_excitation(S, dd, [&](const Det& a, double) {
    ++cnt;
    if (!seen.insert(a).second) unique = false;
  });
  return unique ? cnt : -cnt;
}

// Deterministic screened PT2.  Returns a handle (NULL on error; see
// oracle_last_error).  `status` receives the error code.
void* oracle_pt2_det(int n, int na, int nb, const double* h1, const double* eri,
                     const uint64_t* dets, const double* c, int64_t nd, double e0, double eps2,
                     int want_grad, int* status) {
  System S{n, na, nb, h1, eri};
  const Det* D = reinterpret_cast<const Det*>(dets);
  int st = validate(S, D, c, nd);
  if (!st && !(eps2 >= 0.0)) {
    snprintf(g_err, sizeof g_err, "eps2 must be >= 0");
    st = -1;
  }
  *status = st;
  if (st) return nullptr;
  return run_det(S, D, c, nd, e0, eps2, want_grad != 0);
}

void oracle_result_free(void* h) { delete static_cast<Result*>(h); }

// scalars: e2, de2_de0, min_abs_denom ; counts: n_terms, n_terms_gen, n_unique, n_intruder, n_zero
void oracle_result_scalars(void* h, double* dbl3, int64_t* cnt5) {
  Result* R = static_cast<Result*>(h);
  dbl3[0] = R->e2;
  dbl3[1] = R->de2_de0;
  dbl3[2] = R->min_abs_denom;
  cnt5[0] = R->n_terms;
  cnt5[1] = R->n_terms_gen;
  cnt5[2] = (int64_t)R->uniq.size();
  cnt5[3] = R->n_intruder;
  cnt5[4] = R->n_zero_denom;
}

// unique a (not in V), in ascending key order: keys [n_unique][4], A, D, counts
void oracle_result_unique(void* h, uint64_t* keys, double* A, double* D, int64_t* cnt) {
  Result* R = static_cast<Result*>(h);
  for (size_t k = 0; k < R->uniq.size(); ++k) {
    std::memcpy(&keys[4 * k], R->uniq[k].a.w, 32);
    A[k] = R->uniq[k].A;
    D[k] = R->uniq[k].D;
    cnt[k] = R->uniq[k].cnt;
  }
}

// every kept term (a in V included), sorted by (a, i): keys, i, H_ai, in_v flag
void oracle_result_terms(void* h, uint64_t* keys, uint32_t* idx, double* hval, uint8_t* in_v) {
  Result* R = static_cast<Result*>(h);
  for (size_t k = 0; k < R->terms.size(); ++k) {
    std::memcpy(&keys[4 * k], R->terms[k].a.w, 32);
    idx[k] = R->terms[k].i;
    hval[k] = R->terms[k].h;
    in_v[k] = R->in_v[k];
  }
}

void oracle_result_grad(void* h, double* grad) {
  Result* R = static_cast<Result*>(h);
  std::copy(R->grad.begin(), R->grad.end(), grad);
}

// Quad-precision central finite differences of E2 with the screening mask of
// the base point frozen.  For each coordinate i the terms that do not involve
// c_i are identical at c_i +- h, so E2(c+h e_i) - E2(c-h e_i) is formed from
// the determinants a connected to i only, each A_a re-summed in binary128.
// fd[k] = (E2(+) - E2(-)) / (2 h_k), h_k = rel_step * |c_i| (or rel_step if c_i == 0).
void oracle_result_fd_grad(void* h, const double* c, const int64_t* coords, int64_t ncoord,
                           double rel_step, double* fd) {
  Result* R = static_cast<Result*>(h);
  // map term index -> unique index
  std::vector<int64_t> owner(R->terms.size(), -1);
  for (size_t u = 0; u < R->uniq.size(); ++u)
    for (int64_t m = R->uniq[u].first; m < R->uniq[u].first + R->uniq[u].cnt; ++m) owner[m] = (int64_t)u;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t k = 0; k < ncoord; ++k) {
    int64_t i = coords[k];
    __float128 ci = c[i];
    __float128 hq = rel_step * (c[i] != 0.0 ? std::fabs(c[i]) : 1.0);
    __float128 acc = 0;
    std::vector<int64_t> us;
    for (size_t m = 0; m < R->terms.size(); ++m)
      if (R->terms[m].i == (uint32_t)i && owner[m] >= 0) us.push_back(owner[m]);
    for (int64_t u : us) {
      const Unique& U = R->uniq[u];
      __float128 ap = 0, am = 0;
      for (int64_t m = U.first; m < U.first + U.cnt; ++m) {
        const Term& t = R->terms[m];
        __float128 cj = c[t.i];
        __float128 hv = t.h;
        if (t.i == (uint32_t)i) {
          ap += hv * (ci + hq);
          am += hv * (ci - hq);
        } else {
          ap += hv * cj;
          am += hv * cj;
        }
      }
      acc += (ap * ap - am * am) / (__float128)U.D;
    }
    fd[k] = (double)(acc / (2 * hq));
  }
}

// dE2/dE0 by central differences in binary128 with one Richardson step.
double oracle_result_fd_de0(void* h, double step) {
  Result* R = static_cast<Result*>(h);
  auto fd = [&](__float128 hq) {
    __float128 acc = 0;
    for (const Unique& U : R->uniq) {
      __float128 a2 = (__float128)U.A * (__float128)U.A;
      acc += a2 / ((__float128)U.D + hq) - a2 / ((__float128)U.D - hq);
    }
    return acc / (2 * hq);
  };
  __float128 f1 = fd(step), f2 = fd(step / 2);
  return (double)((4 * f2 - f1) / 3);
}

// A_a for given determinants a, computed from a's side: every single and
// double excitation j of a that lies in V contributes H_aj c_j if it passes
// the screen; terms are summed in ascending j.  in_v[k] = a is itself in V.
int oracle_pt2_at(int n, int na, int nb, const double* h1, const double* eri, const uint64_t* dets,
                  const double* c, int64_t nd, double e0, double eps2, const uint64_t* alist,
                  int64_t na_list, double* A, double* D, int64_t* cnt, uint8_t* in_v) {
  System S{n, na, nb, h1, eri};
  const Det* V = reinterpret_cast<const Det*>(dets);
  std::unordered_map<Det, int64_t, DetHash> index;
  index.reserve(nd * 2);
  for (int64_t i = 0; i < nd; ++i) index.emplace(V[i], i);
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t k = 0; k < na_list; ++k) {
    Det a;
    std::memcpy(a.w, &alist[4 * k], 32);
    in_v[k] = index.count(a) ? 1 : 0;
    std::vector<std::pair<int64_t, double>> hits;
    for_each_excitation(S, a, [&](const Det& j, double) {
      auto it = index.find(j);
      if (it == index.end()) return;
      double hval = hij(S, a, V[it->second]);  // evaluated from the source j
      if (kept(hval, c[it->second], eps2)) hits.emplace_back(it->second, hval);
    });
    std::sort(hits.begin(), hits.end());
    Neumaier s;
    for (auto& x : hits) s.add(x.second * c[x.first]);
    A[k] = s.value();
    cnt[k] = (int64_t)hits.size();
    D[k] = e0 - diag_value(S, a);
  }
  return 0;
}

// Kept terms (screened, a outside V) of the listed sources: for each source
// src[k], every single and double excitation a with fabs(H_ai)*fabs(c_i) >
// eps2 and a not in V, in enumeration order.  Writes up to cap entries
// (key of a, H_ai, k) and returns the total number found.
int64_t oracle_terms_of(int n, int na, int nb, const double* h1, const double* eri, const uint64_t* dets,
                        const double* c, int64_t nd, double eps2, const int64_t* src, int64_t nsrc,
                        uint64_t* keys, double* hv, int64_t* which, int64_t cap) {
  System S{n, na, nb, h1, eri};
  const Det* V = reinterpret_cast<const Det*>(dets);
  std::unordered_set<Det, DetHash> vset(V, V + nd);
  std::vector<std::vector<std::pair<Det, double>>> per(nsrc);
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t k = 0; k < nsrc; ++k) {
    const int64_t i = src[k];
    for_each_excitation(S, V[i], [&](const Det& a, double h) {
      if (kept(h, c[i], eps2) && !vset.count(a)) per[k].emplace_back(a, h);
    });
  }
  int64_t o = 0;
  for (int64_t k = 0; k < nsrc; ++k)
    for (auto& t : per[k]) {
      if (o < cap) {
        std::memcpy(&keys[4 * o], t.first.w, 32);
        hv[o] = t.second;
        which[o] = k;
      }
      ++o;
    }
  return o;
}

// Per-batch statistics of e_a = (A_a(eps2)^2 - A_a(eps2_hi)^2) / (E0 - H_aa)
// over the a outside V of batch `batch` (of n_batches), reached by a term
// with |H_ai c_i| > eps2; A_a(e) sums the terms above e (none when e is
// infinite).  out = {sum e_a, sum e_a^2}; counts = {number of a, kept terms}.
int oracle_det_batch(int n, int na, int nb, const double* h1, const double* eri, const uint64_t* dets,
                     const double* c, int64_t nd, double e0, double eps2, double eps2_hi, int32_t n_batches,
                     int32_t batch, double* out, int64_t* counts) {
  System S{n, na, nb, h1, eri};
  const Det* V = reinterpret_cast<const Det*>(dets);
  int st = validate(S, V, c, nd);
  if (st) return st;
  std::unordered_set<Det, DetHash> Vset(V, V + nd);
  std::vector<Term> terms;
  collect_terms(S, V, c, nd, eps2, terms);
  Neumaier sum, sq;
  int64_t nu = 0, nt = 0;
  size_t k = 0;
  while (k < terms.size()) {
    size_t j = k;
    while (j < terms.size() && terms[j].a == terms[k].a) ++j;
    const Det& a = terms[k].a;
    if (!Vset.count(a) && (int64_t)(batch_hash(a, n) & (uint64_t)(n_batches - 1)) == batch) {
      Neumaier A, Ah;
      for (size_t m = k; m < j; ++m) {
        const double t = terms[m].h * c[terms[m].i];
        A.add(t);
        if (kept(terms[m].h, c[terms[m].i], eps2_hi)) Ah.add(t);
      }
      const double Av = A.value(), Ahv = Ah.value();
      const double D = e0 - diag_value(S, a);
      const double e = (Av * Av - Ahv * Ahv) / D;
      sum.add(e);
      sq.add(e * e);
      ++nu;
      nt += (int64_t)(j - k);
    }
    k = j;
  }
  out[0] = sum.value();
  out[1] = sq.value();
  counts[0] = nu;
  counts[1] = nt;
  return 0;
}

// Stochastic estimator on explicit draws (stochastic PT2 equation).  draws is
// [ns][ndraw] indices into V; out[s] = S_s(eps2) - S_s(eps2_d), where
// S_s(e) = sum_{a not in V} [ (sum_i w_i c_i H_ai / p_i)^2
//            + sum_i (w_i (Nd-1)/p_i - w_i^2/p_i^2) c_i^2 H_ai^2 ] / ((E0 - H_aa) Nd (Nd-1)),
// the inner sums running over the distinct determinants of sample s whose
// term passes |H_ai c_i| > e.
//
// sample_core evaluates it with the sampling probabilities p_i and the
// screening taken from c_ref and the values from c (c_ref = c is the plain
// estimator; c != c_ref gives the frozen-mask function used for finite
// differences).  With grad != NULL it also accumulates the derivative of the
// mean over samples at frozen draws, p and masks,
//   d/dc_i = mean_s sum_{a: (i,a) kept} [ 2 X_a w_i H_ai / p_i
//            + 2 (w_i (Nd-1)/p_i - w_i^2/p_i^2) c_i H_ai^2 - (the same over the
//            eps2_d terms, with X_a^d) ] / ((E0 - H_aa) Nd (Nd-1)),
// and per sample de0[s] = dS_s/dE0 = -sum_a [...] / ((E0 - H_aa)^2 Nd (Nd-1)).
// sens[s] = sum_a |[...]| / ((E0 - H_aa)^2 Nd (Nd-1)) = sum_a |contribution_a| /
// |E0 - H_aa|: to first order, a change delta of every denominator moves S_s
// by at most delta * sens[s] (the conditioning of the estimate on H_aa).
static int sample_core(const System& S, const Det* V, int64_t nd, const double* c, const double* c_ref,
                       double e0, double eps2, double eps2_d, int32_t ns, int32_t ndraw,
                       const uint32_t* draws, double* out, double* grad, double* de0,
                       int32_t n_batches = 1, const int32_t* sbatch = nullptr, int64_t* nterm = nullptr,
                       double* sens = nullptr) {
  int st = validate(S, V, c_ref, nd);
  if (st) return st;
  if (ndraw < 2 || ns < 1 || !(eps2 >= 0.0) || !(eps2_d >= eps2)) {
    snprintf(g_err, sizeof g_err, "bad sample arguments");
    return -1;
  }
  for (int64_t k = 0; k < (int64_t)ns * ndraw; ++k)
    if ((int64_t)draws[k] >= nd) {
      snprintf(g_err, sizeof g_err, "draw out of range");
      return -1;
    }
  std::unordered_set<Det, DetHash> Vset(V, V + nd);
  Neumaier sa;
  for (int64_t i = 0; i < nd; ++i) sa.add(std::fabs(c_ref[i]));
  const double sum_abs = sa.value();
  const double Nd = (double)ndraw;
  if (grad)
    for (int64_t i = 0; i < nd; ++i) grad[i] = 0.0;
  std::vector<Neumaier> gacc(grad ? nd : 0);
  for (int32_t s = 0; s < ns; ++s) {
    std::vector<uint32_t> dr(draws + (int64_t)s * ndraw, draws + (int64_t)(s + 1) * ndraw);
    std::sort(dr.begin(), dr.end());
    struct Acc {
      Neumaier X, Y, Xd, Yd;
    };
    struct T {
      Det a;
      uint32_t i;
      double x, y;  // w c H / p and (w (Nd-1)/p - w^2/p^2) c^2 H^2
      double wh;    // w H / p
      double q;     // (w (Nd-1)/p - w^2/p^2) c H^2
      bool d;
    };
    std::vector<T> terms;
    size_t k = 0;
    std::vector<std::pair<uint32_t, int>> uw;
    while (k < dr.size()) {
      size_t j = k;
      while (j < dr.size() && dr[j] == dr[k]) ++j;
      uw.emplace_back(dr[k], (int)(j - k));
      k = j;
    }
    std::vector<std::vector<T>> per(uw.size());
#pragma omp parallel for schedule(dynamic, 1)
    for (size_t u = 0; u < uw.size(); ++u) {
      uint32_t i = uw[u].first;
      double w = uw[u].second;
      double ci = c[i], cr = c_ref[i];
      double p = std::fabs(cr) / sum_abs;
      // screening and H from the reference coefficients' determinant (H does
      // not depend on c); values with c
      for_each_excitation(S, V[i], [&](const Det& a, double hval) {
        if (!kept(hval, cr, eps2)) return;
        if (n_batches > 1 && (int64_t)(batch_hash(a, S.n) & (uint64_t)(n_batches - 1)) != sbatch[s]) return;
        double ch = ci * hval;
        double f = w * (Nd - 1.0) / p - w * w / (p * p);
        double x = w * ch / p;
        double y = f * ch * ch;
        per[u].push_back(T{a, i, x, y, w * hval / p, f * ci * hval * hval, kept(hval, cr, eps2_d)});
      });
    }
    size_t total = 0;
    for (auto& v : per) total += v.size();
    terms.reserve(total);
    for (auto& v : per) {
      terms.insert(terms.end(), v.begin(), v.end());
      std::vector<T>().swap(v);
    }
    __gnu_parallel::sort(terms.begin(), terms.end(), [](const T& x, const T& y) {
      if (x.a == y.a) return x.i < y.i;
      return x.a < y.a;
    });
    // one contribution per distinct a outside V, summed per thread
    // (Neumaier) and then across threads in thread order
    std::vector<size_t> heads;
    for (size_t m = 0; m < terms.size(); ++m)
      if (m == 0 || !(terms[m].a == terms[m - 1].a)) heads.push_back(m);
    heads.push_back(terms.size());
    const int64_t ngroups = (int64_t)heads.size() - 1;
    const int nthr = omp_get_max_threads();
    std::vector<Neumaier> part(nthr), dpart(nthr), spart(nthr);
    std::vector<int64_t> kept_terms(nthr, 0);  // terms of a outside V
    // per group: X, X^d and 1 / (D Nd (Nd-1)) (0 for members of V)
    std::vector<double> gX(grad ? ngroups : 0), gXd(grad ? ngroups : 0), gG(grad ? ngroups : 0);
#pragma omp parallel for schedule(static)
    for (int64_t g = 0; g < ngroups; ++g) {
      const size_t k0 = heads[g], j = heads[g + 1];
      if (Vset.count(terms[k0].a)) {
        if (grad) gG[g] = 0.0;
        continue;
      }
      Acc acc;
      kept_terms[omp_get_thread_num()] += (int64_t)(j - k0);
      for (size_t m = k0; m < j; ++m) {
        acc.X.add(terms[m].x);
        acc.Y.add(terms[m].y);
        if (terms[m].d) {
          acc.Xd.add(terms[m].x);
          acc.Yd.add(terms[m].y);
        }
      }
      double X = acc.X.value(), Y = acc.Y.value(), Xd = acc.Xd.value(), Yd = acc.Yd.value();
      double Dd = e0 - diag_value(S, terms[k0].a);
      double bracket = (X * X + Y) - (Xd * Xd + Yd);
      part[omp_get_thread_num()].add(bracket / (Dd * Nd * (Nd - 1.0)));
      dpart[omp_get_thread_num()].add(-bracket / (Dd * Dd * Nd * (Nd - 1.0)));
      spart[omp_get_thread_num()].add(std::fabs(bracket / (Dd * Dd * Nd * (Nd - 1.0))));
      if (grad) {
        gX[g] = X;
        gXd[g] = Xd;
        gG[g] = 1.0 / (Dd * Nd * (Nd - 1.0));
      }
    }
    Neumaier tot, dtot;
    for (int t = 0; t < nthr; ++t) {
      tot.add(part[t].s);
      tot.add(part[t].c);
      dtot.add(dpart[t].s);
      dtot.add(dpart[t].c);
    }
    // one batch of P per sample: the estimate is scaled by the number of batches
    out[s] = (double)n_batches * tot.value();
    if (nterm) {
      nterm[s] = 0;
      for (int t = 0; t < nthr; ++t) nterm[s] += kept_terms[t];
    }
    if (de0) de0[s] = (double)n_batches * dtot.value();
    if (sens) {
      Neumaier stot;
      for (int t = 0; t < nthr; ++t) {
        stot.add(spart[t].s);
        stot.add(spart[t].c);
      }
      sens[s] = (double)n_batches * stot.value();
    }
    if (grad) {
      // terms in (a, i) order; per source i the sum runs in that order
      for (int64_t g = 0; g < ngroups; ++g) {
        if (gG[g] == 0.0) continue;
        for (size_t m = heads[g]; m < heads[g + 1]; ++m) {
          const T& t = terms[m];
          double v = 2.0 * gX[g] * t.wh + 2.0 * t.q;
          if (t.d) v -= 2.0 * gXd[g] * t.wh + 2.0 * t.q;
          gacc[t.i].add(v * gG[g]);
        }
      }
    }
  }
  if (grad)
    for (int64_t i = 0; i < nd; ++i) grad[i] = gacc[i].value() / (double)ns;
  return 0;
}

// The per-sample estimates and, per sample, the number of kept terms whose a
// lies outside V and (sens, nullable) the conditioning on H_aa (sample_core).
int oracle_pt2_sample_counts(int n, int na, int nb, const double* h1, const double* eri, const uint64_t* dets,
                             const double* c, int64_t nd, double e0, double eps2, double eps2_d, int32_t ns,
                             int32_t ndraw, const uint32_t* draws, double* out, int64_t* nterm, double* sens) {
  System S{n, na, nb, h1, eri};
  return sample_core(S, reinterpret_cast<const Det*>(dets), nd, c, c, e0, eps2, eps2_d, ns, ndraw, draws, out,
                     nullptr, nullptr, 1, nullptr, nterm, sens);
}

int oracle_pt2_sample(int n, int na, int nb, const double* h1, const double* eri,
                      const uint64_t* dets, const double* c, int64_t nd, double e0, double eps2,
                      double eps2_d, int32_t ns, int32_t ndraw, const uint32_t* draws, double* out) {
  System S{n, na, nb, h1, eri};
  return sample_core(S, reinterpret_cast<const Det*>(dets), nd, c, c, e0, eps2, eps2_d, ns, ndraw, draws,
                     out, nullptr, nullptr);
}

// The estimator with one batch of P per sample: sample s keeps the a with
// batch_hash(a) mod n_batches == sbatch[s]; its estimate is multiplied by
// n_batches (stochastic step of the 3-step method, section IV).
int oracle_pt2_sample_batched(int n, int na, int nb, const double* h1, const double* eri,
                              const uint64_t* dets, const double* c, int64_t nd, double e0, double eps2,
                              double eps2_d, int32_t ns, int32_t ndraw, const uint32_t* draws,
                              int32_t n_batches, const int32_t* sbatch, double* out) {
  System S{n, na, nb, h1, eri};
  return sample_core(S, reinterpret_cast<const Det*>(dets), nd, c, c, e0, eps2, eps2_d, ns, ndraw, draws,
                     out, nullptr, nullptr, n_batches, sbatch);
}

// The estimator with p_i and the screening frozen at c_ref and values at c.
int oracle_pt2_sample_frozen(int n, int na, int nb, const double* h1, const double* eri,
                             const uint64_t* dets, const double* c, const double* c_ref, int64_t nd,
                             double e0, double eps2, double eps2_d, int32_t ns, int32_t ndraw,
                             const uint32_t* draws, double* out) {
  System S{n, na, nb, h1, eri};
  return sample_core(S, reinterpret_cast<const Det*>(dets), nd, c, c_ref, e0, eps2, eps2_d, ns, ndraw, draws,
                     out, nullptr, nullptr);
}

// Per-sample estimates, the gradient of their mean with respect to c (draws,
// p and masks frozen) and per-sample derivatives with respect to E0.
int oracle_pt2_sample_grad(int n, int na, int nb, const double* h1, const double* eri,
                           const uint64_t* dets, const double* c, int64_t nd, double e0, double eps2,
                           double eps2_d, int32_t ns, int32_t ndraw, const uint32_t* draws, double* out,
                           double* grad, double* de0) {
  System S{n, na, nb, h1, eri};
  return sample_core(S, reinterpret_cast<const Det*>(dets), nd, c, c, e0, eps2, eps2_d, ns, ndraw, draws,
                     out, grad, de0);
}

// <c|H|c> over all pairs of V (pairs more than two excitations apart are skipped).
double oracle_energy(int n, int na, int nb, const double* h1, const double* eri,
                     const uint64_t* dets, const double* c, int64_t nd) {
  System S{n, na, nb, h1, eri};
  const Det* V = reinterpret_cast<const Det*>(dets);
  std::vector<double> row(nd);
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t i = 0; i < nd; ++i) {
    Neumaier r;
    r.add(c[i] * c[i] * diag_value(S, V[i]));
    for (int64_t j = i + 1; j < nd; ++j) {
      int diff = 0;
      for (int w = 0; w < 4; ++w) diff += __builtin_popcountll(V[i].w[w] ^ V[j].w[w]);
      if (diff > 4) continue;
      double hv = hij(S, V[j], V[i]);
      if (hv != 0.0) r.add(2.0 * c[i] * c[j] * hv);
    }
    row[i] = r.value();
  }
  Neumaier e;
  for (int64_t i = 0; i < nd; ++i) e.add(row[i]);
  return e.value();
}

// H c on the variational space, row by row (the fast evaluation through alpha
// and beta string lists is the subject of section III and Algorithms 1-2; the
// oracle takes every pair): for each requested row i,
//   y_i = sum_j <i|H|j> c_j over all j of V in index order (Neumaier sum,
//         <i|H|j> evaluated from the source j),
// and the number of j != i that differ from i by one or two excitations.
int oracle_hc_rows(int n, int na, int nb, const double* h1, const double* eri, const uint64_t* dets,
                   const double* c, int64_t nd, const int64_t* rows, int64_t nrows, double* y,
                   int64_t* nconn) {
  System S{n, na, nb, h1, eri};
  const Det* V = reinterpret_cast<const Det*>(dets);
  if (int st = validate(S, V, c, nd)) return st;
  for (int64_t r = 0; r < nrows; ++r)
    if (rows[r] < 0 || rows[r] >= nd) {
      snprintf(g_err, sizeof g_err, "row %lld outside [0, %lld)", (long long)rows[r], (long long)nd);
      return -6;
    }
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t r = 0; r < nrows; ++r) {
    const int64_t i = rows[r];
    Neumaier acc;
    int64_t cnt = 0;
    for (int64_t j = 0; j < nd; ++j) {
      int diff = 0;
      for (int w = 0; w < 4; ++w) diff += __builtin_popcountll(V[i].w[w] ^ V[j].w[w]);
      if (diff > 4) continue;
      if (j != i) ++cnt;
      acc.add(hij(S, V[i], V[j]) * c[j]);
    }
    y[r] = acc.value();
    nconn[r] = cnt;
  }
  return 0;
}

// <c|H|c> for large V without visiting every pair.  Two distinct
// determinants that differ by a single or double excitation both contain some
// set of N-2 occupied spin orbitals (a "core"): for a double it is their common
// occupation, for a single their common occupation minus any one orbital.
// Every determinant is listed under each of its C(N,2) cores (the core's
// 64-bit hash, SplitMix64's finaliser chained over the four words), the list
// is sorted by hash, and within one hash group every pair is tested.  A pair
// is credited only in the group of its canonical core -- the common occupation
// with its lowest-addressed orbitals removed until N-2 remain -- so it is
// counted exactly once even when unrelated cores share a hash value.  The
// hash space is processed in 2^part_bits slices to bound memory.  hash_bits
// < 64 truncates the hash (tests use it to force collisions).  Pair terms are
// 2 c_i c_j H_ji for i < j, H_ji evaluated from the source i as in
// oracle_energy; diagonal terms c_i^2 H_ii.  Sums are Neumaier per thread
// (static schedules, so the result depends only on the thread count).
static uint64_t splitmix_fin(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}
static uint64_t core_hash(const uint64_t* w, int hash_bits) {
  uint64_t h = 0x6a09e667f3bcc909ull;
  for (int k = 0; k < 4; ++k) h = splitmix_fin(h ^ w[k]);
  return hash_bits >= 64 ? h : (h >> (64 - hash_bits));
}

double oracle_energy_cores(int n, int na, int nb, const double* h1, const double* eri,
                           const uint64_t* dets, const double* c, int64_t nd, int part_bits,
                           int hash_bits, int64_t* n_pairs_out) {
  System S{n, na, nb, h1, eri};
  const Det* V = reinterpret_cast<const Det*>(dets);
  const int ne = na + nb;
  const int nthr = omp_get_max_threads();
  if (hash_bits < part_bits) part_bits = hash_bits;
  std::vector<Neumaier> acc(nthr);
  std::vector<int64_t> npairs(nthr, 0);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < nd; ++i) acc[omp_get_thread_num()].add(c[i] * c[i] * diag_value(S, V[i]));
  const int64_t nparts = (int64_t)1 << part_bits;
  for (int64_t part = 0; part < nparts; ++part) {
    std::vector<std::vector<std::pair<uint64_t, uint32_t>>> buf(nthr);
#pragma omp parallel
    {
      auto& b = buf[omp_get_thread_num()];
      int pos[256];
#pragma omp for schedule(static)
      for (int64_t i = 0; i < nd; ++i) {
        int m = 0;
        for (int k = 0; k < 4; ++k)
          for (uint64_t x = V[i].w[k]; x; x &= x - 1) pos[m++] = 64 * k + __builtin_ctzll(x);
        for (int x = 0; x < m; ++x)
          for (int y = x + 1; y < m; ++y) {
            uint64_t w[4] = {V[i].w[0], V[i].w[1], V[i].w[2], V[i].w[3]};
            w[pos[x] >> 6] &= ~(1ull << (pos[x] & 63));
            w[pos[y] >> 6] &= ~(1ull << (pos[y] & 63));
            const uint64_t h = core_hash(w, hash_bits);
            const uint64_t slice = part_bits ? (h >> (hash_bits - part_bits)) : 0;
            if ((int64_t)slice == part) b.emplace_back(h, (uint32_t)i);
          }
      }
    }
    std::vector<std::pair<uint64_t, uint32_t>> all;
    size_t tot = 0;
    for (auto& b : buf) tot += b.size();
    all.reserve(tot);
    for (auto& b : buf) {
      all.insert(all.end(), b.begin(), b.end());
      std::vector<std::pair<uint64_t, uint32_t>>().swap(b);
    }
    __gnu_parallel::sort(all.begin(), all.end());
    std::vector<size_t> starts;
    for (size_t k = 0; k < all.size(); ++k)
      if (k == 0 || all[k].first != all[k - 1].first) starts.push_back(k);
    starts.push_back(all.size());
    const int64_t ng = (int64_t)starts.size() - 1;
#pragma omp parallel
    {
      const int t = omp_get_thread_num();
      std::vector<uint32_t> mem;
#pragma omp for schedule(static)
      for (int64_t g = 0; g < ng; ++g) {
        mem.clear();
        for (size_t k = starts[g]; k < starts[g + 1]; ++k)
          if (mem.empty() || mem.back() != all[k].second) mem.push_back(all[k].second);
        const uint64_t hg = all[starts[g]].first;
        for (size_t a = 0; a < mem.size(); ++a)
          for (size_t b = a + 1; b < mem.size(); ++b) {
            const Det& di = V[mem[a]];
            const Det& dj = V[mem[b]];
            int diff = 0;
            for (int k = 0; k < 4; ++k) diff += __builtin_popcountll(di.w[k] ^ dj.w[k]);
            if (diff > 4) continue;
            uint64_t w[4];
            int common = 0;
            for (int k = 0; k < 4; ++k) {
              w[k] = di.w[k] & dj.w[k];
              common += __builtin_popcountll(w[k]);
            }
            for (int k = 0; k < 4 && common > ne - 2; ++k)
              while (w[k] && common > ne - 2) {
                w[k] &= w[k] - 1;
                --common;
              }
            if (core_hash(w, hash_bits) != hg) continue;
            const double hv = hij(S, dj, di);
            ++npairs[t];
            if (hv != 0.0) acc[t].add(2.0 * c[mem[a]] * c[mem[b]] * hv);
          }
      }
    }
  }
  Neumaier e;
  int64_t np = 0;
  for (int t = 0; t < nthr; ++t) {
    e.add(acc[t].s);
    e.add(acc[t].c);
    np += npairs[t];
  }
  if (n_pairs_out) *n_pairs_out = np;
  return e.value();
}

// MP1-like amplitudes H_i0 / (E_HF - H_ii) for the determinants flagged in
// `mask` (doubles of the reference det `ref`), written in determinant order.
void oracle_mp1(int n, int na, int nb, const double* h1, const double* eri, const uint64_t* dets,
                const uint8_t* mask, int64_t nd, const uint64_t* ref, double* out) {
  System S{n, na, nb, h1, eri};
  const Det* V = reinterpret_cast<const Det*>(dets);
  Det r;
  std::memcpy(r.w, ref, 32);
  double ehf = diag_value(S, r);
  int64_t k = 0;
  for (int64_t i = 0; i < nd; ++i) {
    if (!mask[i]) continue;
    out[k++] = hij(S, V[i], r) / (ehf - diag_value(S, V[i]));
  }
}

}  // extern "C"
