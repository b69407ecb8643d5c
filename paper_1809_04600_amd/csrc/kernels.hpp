// Internal interfaces between the host API and the device kernels.
#pragma once
#include "common.hpp"

namespace shci {

// Integral-derived device tables owned by a context.
struct Tables {
  int n = 0, na = 0, nb = 0;
  int nss = 0;            // same-spin keys n(n-1)/2
  int64_t lss = 0, los = 0;  // entries per same-spin / opposite-spin key
  double* h1 = nullptr;      // [n][n]
  double* sD = nullptr;      // [k][p][r] (pr|kk) - (pk|kr)
  double* sJ = nullptr;      // [k][p][r] (pr|kk)
  double* ubound = nullptr;  // [p][r]
  double* fref = nullptr;    // [2][p][r] singles elements of the reference det (per call)
  double* diag = nullptr;    // packed diagonal table (diag.hpp layout)
  double* hpp = nullptr;     // = diag: h_pp
  double* jtri = nullptr;    // = diag + n: (pp|qq), p <= q, at q(q+1)/2 + p
  double* sstri = nullptr;   // (pp|qq) - (pq|qp), p < q, at q(q-1)/2 + p
  double* hb_val = nullptr;  // signed values, sorted per key
  uint16_t* hb_rs = nullptr; // r | s << 8
  double* hb_max = nullptr;  // per key, largest |value| (0 if empty)
  double* mag_cum = nullptr; // [2][72] entries with |value| >= 2^e, e = -64..7, per table kind
  double* g8 = nullptr;      // (pq|rs) folded by its 8-fold symmetry: pair indices P = pq, Q = rs
                             // (x(x+1)/2 + y, x >= y), entry max(P,Q)(max+1)/2 + min(P,Q)
};

int build_tables(Tables& T, const double* h1, const double* eri, hipStream_t st, uint32_t* dflag);
// T.fref for the reference determinant ref (device, 4 words)
void singles_ref(const Tables& T, const uint64_t* ref, hipStream_t st);

// Structure-of-arrays record buffer.
struct Recs {
  uint64_t* k[4] = {nullptr, nullptr, nullptr, nullptr};
  void* v = nullptr;      // double or float
  void* v2 = nullptr;     // second value (sample mode), same type
  uint32_t* pay = nullptr;  // optional source index
  uint32_t* bid = nullptr;  // bucket id (written by the generator, moved by the partition)
  double* haa = nullptr;    // H_aa of the term's determinant (written by the generator)
};

// Per-bucket partial results written by the reduce kernel.
struct Partials {
  double* e2 = nullptr;      // [nbucket] sum of contributions
  double* de0 = nullptr;     // [nbucket] sum of -A^2/D^2
  double* e2sq = nullptr;    // [nbucket] sum of squared contributions (per unique a)
  int64_t* nterm = nullptr;  // [nbucket] kept terms with a outside V
  int64_t* ngen = nullptr;   // [nbucket] all kept terms
  int32_t* nuniq = nullptr;  // [nbucket] unique a outside V
  int32_t* nintr = nullptr;  // [nbucket] intruders (D > 0)
  int32_t* nzero = nullptr;  // [nbucket] D == 0
  double* mind = nullptr;    // [nbucket] min |D|
  int32_t* nseg = nullptr;   // [nbucket] segments (unique keys incl. V members)
};

// Unique-key store (bucket-local, sorted by (h2, key)), used by the adjoint
// and by the export.
struct Uniq {
  uint64_t* k[4] = {nullptr, nullptr, nullptr, nullptr};
  uint32_t* h2 = nullptr;
  double* A = nullptr;   // A_a
  double* D = nullptr;   // E0 - H_aa
  double* g = nullptr;   // 2 A_a / D_a (0 for members of V)
  int32_t* cnt = nullptr;  // kept terms, negative for members of V
  uint64_t* start = nullptr;  // [nbucket] first record / unique slot of the bucket
};

struct GroupPlan {
  int bits_hash = 0;     // hash bits in the bucket id (per sample)
  int sbits = 0;         // sample-id bits in the key
  int nbits = 0;         // total bucket-id bits
  int64_t nbucket = 0;   // 2^nbits
};

}  // namespace shci
