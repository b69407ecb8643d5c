/*
 * shci_pt2.h -- screened Epstein-Nesbet PT2 energy on one AMD Instinct MI355X
 * (gfx950), C ABI.
 *
 * The library evaluates the second-order perturbative correction of selected
 * configuration interaction (paper, section II.B):
 *
 *   E2(eps2) = sum_{a in P} ( sum^{(eps2)}_{i in V} H_ai c_i )^2 / (E0 - H_aa)
 *
 * where V is the variational space, P the determinants outside V reached from
 * V by single and double excitations, and the inner sum keeps only the terms
 * with |H_ai c_i| > eps2 (screened PT2 equation; the strict inequality makes
 * eps2 = 0 keep exactly the non-zero elements, the definition of P in
 * section II).  H_aa is the Epstein-Nesbet zeroth-order energy of a
 * (partition equation).
 *
 * Inputs (the problem statement of section II.B):
 *   - determinants as bit strings: uint64 [n_det][4] =
 *     (alpha_lo, alpha_hi, beta_lo, beta_hi); orbital p of a spin sits at bit
 *     (p & 63) of word (p >> 6) of that spin (section V.A);
 *   - coefficients c [n_det], FP64;
 *   - one-electron integrals h1 [n][n] and two-electron integrals in
 *     chemists' notation (pq|rs) at eri[((p*n+q)*n+r)*n+s], FP64, real
 *     orbitals, symmetric under all eight index permutations;
 *   - E0 (used in every denominator) and the screening threshold(s).
 *
 * Conventions: spin orbitals are ordered alpha_0..alpha_{n-1},
 * beta_0..beta_{n-1}; a same-spin double p<q -> r<s is p->r then q->s.
 *
 * Memory: every pointer marked "device" must be device memory of the current
 * HIP device; "host" pointers are host memory.  All input and output buffers
 * are owned by the caller.  The context owns the integral-derived tables.
 * Device scratch memory: the PT2 calls take a workspace (ws, ws_bytes), a
 * device region owned by the caller (for instance from torch's caching
 * allocator), aligned to 256 bytes.  With a workspace the call allocates
 * nothing and frees nothing; when the screened terms do not fit it, the
 * deterministic calls split the perturbative space into hash batches and the
 * sampling calls evaluate fewer samples per chunk (shci_pt2_workspace_size
 * gives the bytes for a given number of records per pass).  With ws = NULL
 * the context's own grow-only buffers are used instead: they are allocated
 * (hipMalloc) when a call needs more than they hold, after a synchronisation
 * of the call's stream, and freed by shci_pt2_ctx_destroy.
 *
 * Streams: all work is enqueued on `stream` (a hipStream_t, NULL = default
 * stream).  Calls that return host scalars synchronise that stream before
 * returning.  Exception: the sampling calls with a workspace evaluate every
 * other chunk of samples on a second stream owned by the context, from a
 * second host thread, with half of the workspace left; that stream starts
 * after the work already queued on `stream`, and `stream` waits for it before
 * the call returns.  The chunk plan does not depend on this, so the results
 * are the same bits as with one stream.
 *
 * Errors: every entry point returns an shci_status; nothing is thrown across
 * the ABI.  shci_pt2_last_error() returns a thread-local message for the last
 * non-OK status of the calling thread.  Inputs are never modified.
 *
 * Concurrency: a context may be used by one call at a time (its grow-only
 * buffers, flags and timing events are shared by all calls on it); a
 * workspace may be used by one call at a time.
 */
#ifndef SHCI_PT2_H
#define SHCI_PT2_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct shci_pt2_ctx shci_pt2_ctx;

/* Arithmetic of the off-diagonal part.  SHCI_FP64: everything in binary64.
 * SHCI_FP32C: products H_ai c_i and the per-determinant sums A_a in binary32
 * with compensated (TwoSum) accumulation; H_aa, E0 - H_aa and the E2
 * reduction stay binary64.  Screening decisions are binary64 in both modes,
 * so both produce the same connection set. */
enum shci_precision { SHCI_FP64 = 0, SHCI_FP32C = 1 };

/* Operations sized by shci_pt2_workspace_size. */
enum shci_op {
  SHCI_OP_DET = 0,          /* shci_pt2_det, shci_pt2_det_batches */
  SHCI_OP_GRAD = 1,         /* shci_pt2_grad, recompute mode */
  SHCI_OP_GRAD_KEEP = 2,    /* shci_pt2_grad, keep mode */
  SHCI_OP_SAMPLE = 3,       /* shci_pt2_sample, shci_pt2_sample_batched (seed path included) */
  SHCI_OP_SAMPLE_GRAD = 4,  /* shci_pt2_sample_grad */
  SHCI_OP_DRAWS = 5         /* shci_pt2_draws */
};

/* Adjoint modes of shci_pt2_grad. */
enum shci_grad_mode {
  SHCI_GRAD_AUTO = 0,       /* keep when one pass holds every record, else recompute */
  SHCI_GRAD_KEEP = 1,       /* records carry their position; no second generation pass */
  SHCI_GRAD_RECOMPUTE = 2   /* the adjoint walks the connections again (hash batches allowed) */
};

enum shci_status {
  SHCI_OK = 0,
  SHCI_ERR_ARG = -1,        /* bad argument (NULL pointer, negative size, eps2 < 0, ...) */
  SHCI_ERR_NORB = -2,       /* n_orb / electron counts outside the supported range */
  SHCI_ERR_DET = -3,        /* a determinant has a wrong electron count or a bit >= n_orb */
  SHCI_ERR_DUP = -4,        /* two determinants of V are equal */
  SHCI_ERR_NONFINITE = -5,  /* NaN or Inf in c, E0 or the integrals */
  SHCI_ERR_WORKSPACE = -6,  /* device memory exhausted, or the problem exceeds a size limit */
  SHCI_ERR_SINGULAR = -7,   /* some kept a has E0 - H_aa == 0 exactly */
  SHCI_ERR_HIP = -8         /* a HIP runtime call failed */
};

/* Statistics of one call (host struct). */
typedef struct {
  int64_t n_terms;       /* screened terms (i, a) with a outside V */
  int64_t n_terms_gen;   /* screened terms including a inside V */
  int64_t n_unique;      /* |P(eps2)|, distinct a outside V with >= 1 kept term */
  int64_t n_intruder;    /* kept a with E0 - H_aa > 0 */
  double min_abs_denom;  /* min |E0 - H_aa| over kept a (+inf if none) */
  int32_t n_buckets;     /* hash buckets used by the grouping step */
  int32_t n_retries;     /* re-partitions after a bucket overflow */
  double ms_gen;         /* validation, hash set of V, excitation generation (count + write) */
  double ms_sort;        /* hash partition passes */
  double ms_reduce;      /* bucket sort, segmented reduce, diagonal, E2 reduction */
  double ms_total;       /* whole call, device time on `stream` */
  double ms_k_count;     /* generator kernel, count pass */
  double ms_k_write;     /* generator kernel, write pass */
  double ms_k_reduce;    /* bucket reduce kernel */
  int64_t n_records;     /* records materialised (screened terms, members of V included) */
  int32_t key_words;     /* 64-bit words per packed key */
  int32_t value_bytes;   /* bytes per record value (8 FP64, 4 FP32C; x2 in sample mode) */
  int32_t n_chunks;      /* hash batches (det, grad) or sample chunks (sample) evaluated */
  int32_t n_part_launches; /* partition scatter launches (passes summed over chunks) */
  double ms_k_part;      /* partition scatter kernels, summed over their launches */
  int64_t n_part_records; /* records moved by the scatter launches (records x passes, summed) */
  int64_t n_terms_all;   /* screened terms generated (records plus terms reduced in place) */
  int64_t n_hashes;      /* singleton split: grouping hashes listed and partitioned (fillers included) */
  int64_t n_singletons;  /* singleton split: terms reduced in place by the write walk (no record) */
  double ms_k_split;     /* singleton split: hash partition, repeat finder and marks */
} shci_pt2_stats;

/* Optional device outputs of shci_pt2_det (any pointer may be NULL).
 * Unique determinants a outside V, in an unspecified but deterministic order:
 *   u_keys [u_cap][4] uint64 (same layout as the input dets), u_A [u_cap]
 *   (A_a = sum of kept H_ai c_i), u_D [u_cap] (E0 - H_aa), u_cnt [u_cap]
 *   (kept terms of a).  u_n receives the number of unique a (host value); if
 *   it exceeds u_cap only u_cap entries are written.
 * Raw terms (a inside V included), in generation order:
 *   t_keys [t_cap][4], t_i [t_cap] (index of the source det), t_val [t_cap]
 *   (H_ai c_i, FP64, or the FP32 product widened in SHCI_FP32C).  t_n receives
 *   the number of terms (host value). */
typedef struct {
  uint64_t* u_keys;
  double* u_A;
  double* u_D;
  int32_t* u_cnt;
  int64_t u_cap;
  int64_t u_n;
  uint64_t* t_keys;
  uint32_t* t_i;
  double* t_val;
  int64_t t_cap;
  int64_t t_n;
} shci_pt2_export;

/* Creates a context for n_orb spatial orbitals (1 <= n_orb <= 127) and
 * n_alpha, n_beta electrons (each in [1, n_orb - 1]).  h1 and eri are device
 * pointers (FP64, layout above); they are read during this call only.  Builds
 * on the device:
 *   - the heat-bath tables: for every occupied spatial pair, the matrix
 *     elements of all double excitations from it, sorted by decreasing
 *     magnitude with their target pair (section II.A, heat-bath screening,
 *     used again for eps2 in section II.B):
 *       same spin, pair p<q: all r<s outside {p,q}, value (pr|qs) - (ps|qr);
 *       opposite spin, pair (p_alpha, q_beta): all r != p, s != q, value (pr|qs);
 *     ties are ordered by ascending (r, s);
 *   - single-excitation tables (pr|kk) - (pk|kr), (pr|kk) and an upper bound
 *     of |H_ai| per (p, r);
 *   - diagonal tables (pp|qq), (pq|qp).
 * Returns SHCI_ERR_NONFINITE if an integral is not finite. */
int shci_pt2_ctx_create(int n_orb, int n_alpha, int n_beta, const double* h1, const double* eri,
                        void* stream, shci_pt2_ctx** out);

/* Frees the context, its tables and its grow-only buffers.  NULL is ignored. */
void shci_pt2_ctx_destroy(shci_pt2_ctx* ctx);

/* Caps the context's own grow-only buffers (bytes; 0 = no cap; calls with
 * ws = NULL).  A region that would exceed the cap fails with
 * SHCI_ERR_WORKSPACE. */
int shci_pt2_ctx_set_workspace_limit(shci_pt2_ctx* ctx, size_t bytes);

/* Workspace bytes for `op` (enum shci_op) on n_det variational determinants
 * when one pass materialises up to n_records screened terms (values below
 * 1024 count as 1024; the records of a previous call are in
 * shci_pt2_stats.n_records).  Sampling ops also take n_samples and n_draws
 * (the seed path's draws and alias table are included).  A workspace of this
 * size holds one pass of that many records; a smaller one makes the call use
 * more hash batches or smaller sample chunks.  The figure assumes at most
 * 2 n_det work items (heavy determinants split over their occupied pairs);
 * more items take their room from the records.
 *   bytes  host, out.  Errors: SHCI_ERR_ARG. */
int shci_pt2_workspace_size(const shci_pt2_ctx* ctx, int op, int64_t n_det, int64_t n_records, int32_t n_samples,
                            int32_t n_draws, int precision, size_t* bytes);

/* Caps the screened-term records one generation pass materialises
 * (0 = automatic: what free device memory, or the workspace cap, holds).
 * Above the cap, shci_pt2_det and shci_pt2_grad split the perturbative
 * determinants into 2^k hash batches (at most 256) and regenerate the terms
 * once per batch, keeping in batch b only the a whose determinant hash has
 * low bits b; every a is reduced whole in one batch, so E2 and the gradient
 * are sums over batches (the paper's hash-batch decomposition of P,
 * section IV).  shci_pt2_sample instead evaluates its samples in chunks of
 * consecutive samples.  st->n_chunks reports the batches or chunks used. */
int shci_pt2_ctx_set_record_limit(shci_pt2_ctx* ctx, int64_t max_records);

/* How the screened terms are grouped by perturbative determinant a (the sums
 * A_a = sum_i H_ai c_i of the screened PT2 equation, section II.B; the paper
 * accumulates them in a hash table, section V.C).
 *   SHCI_GROUP_SPLIT: singleton split.  The count pass lists a
 *     64-bit grouping hash per term (determinant hash, sample id mixed in);
 *     the list is partitioned and hashes that occur more than once are set in
 *     a presence filter.  The write pass makes records only of terms whose
 *     hash passes the filter (every a with two or more terms, plus false
 *     positives) and adds the contribution of every other term, alone in its
 *     group, in place.  Same terms, groups and counts as SHCI_GROUP_RECORDS;
 *     E2 differs by summation order only.  Calls that export or keep
 *     per-term or per-a data (unique export, term export, adjoints) group
 *     every term as a record.
 *   SHCI_GROUP_RECORDS: every term becomes a record (key, value, H_aa).
 *   SHCI_GROUP_AUTO (default): the singleton split for the passes of the
 *     sampling calls, and for deterministic passes of 1e8 kept terms or
 *     more; a smaller deterministic pass groups every term as a record (its
 *     count pass still lists the hashes; the choice follows the exact count,
 *     so a repeat makes the same one).
 * The limit of shci_pt2_ctx_set_record_limit applies to the terms of a pass
 * in every mode. */
enum { SHCI_GROUP_AUTO = 0, SHCI_GROUP_RECORDS = 1, SHCI_GROUP_SPLIT = 2 };
int shci_pt2_ctx_set_grouping(shci_pt2_ctx* ctx, int mode);

/* Sample chunks in flight at once in the sampling calls with a workspace: 2
 * (default; a second stream and host thread take every other chunk, see
 * Streams above) or 1 (every chunk on `stream`, in order).  The results are
 * the same bits either way; 1 gives each kernel the whole GPU (profiling). */
int shci_pt2_ctx_set_lanes(shci_pt2_ctx* ctx, int lanes);

/* Hashes per bucket of the singleton split's repeat finder, in [64, 2^24]
 * (default 12500: one workgroup's shared-memory table of 36,864 tags takes
 * a bucket in one fill and holds its hashes in registers).  Larger buckets
 * are taken from memory, in slices by hash bits when their distinct tags
 * overflow the table; the results are the same up to the order of the sums
 * (the terms, groups and counts are exact in every case).  A tuning and
 * testing knob: the default is the fast one. */
int shci_pt2_ctx_set_split_bucket(shci_pt2_ctx* ctx, int64_t hashes);

/* Deterministic screened PT2 (screened PT2 equation).
 *   dets  device uint64 [n_det][4], unique, with n_alpha / n_beta electrons;
 *   c     device FP64 [n_det];
 *   e0    E0 of every denominator; eps2 >= 0 the screening threshold;
 *   precision  SHCI_FP64 or SHCI_FP32C;
 *   ws, ws_bytes  device workspace or NULL (see Memory above);
 *   e2    host, receives E2; st host, nullable; ex host struct, nullable.
 * The result is deterministic: repeated calls give identical bits.
 * SHCI_ERR_SINGULAR is returned (with e2 = +-inf or nan) if a kept a has
 * E0 - H_aa == 0 exactly; intruders with E0 - H_aa > 0 are counted, not
 * rejected. */
int shci_pt2_det(shci_pt2_ctx* ctx, const uint64_t* dets, const double* c, int64_t n_det,
                 double e0, double eps2, int precision, void* ws, size_t ws_bytes, void* stream, double* e2,
                 shci_pt2_stats* st, shci_pt2_export* ex);

/* shci_pt2_det for callers that cannot allocate device memory (code under
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).  The
 * call allocates and frees nothing: its workspace is a fixed 128 MiB device
 * array in the library (one per GPU, held until the process ends, its address
 * taken once per device when a context is created there).  Terms that do not
 * fit it are split into hash batches as in shci_pt2_det (at most 256).
 * n_det <= 500000, else SHCI_ERR_WORKSPACE; SHCI_ERR_WORKSPACE also when one
 * batch does not fit.  Every call on a GPU shares that GPU's array: calls that
 * overlap on one GPU (other streams, other threads) race and must not be
 * issued.  Arguments and results as shci_pt2_det (no export). */
int shci_pt2_det_static(shci_pt2_ctx* ctx, const uint64_t* dets, const double* c, int64_t n_det, double e0,
                        double eps2, int precision, void* stream, double* e2, shci_pt2_stats* st);

/* Stochastic part of the semistochastic PT2 (semistochastic and stochastic
 * PT2 equations).  For each sample s of n_draws draws (indices into V, drawn
 * with replacement with p_i = |c_i| / sum_j |c_j|, the sampling-probability
 * equation), with w_i the multiplicity of det i in the sample:
 *   S_s(e) = sum_{a not in V} [ (sum_i w_i c_i H_ai / p_i)^2
 *            + sum_i (w_i (N_d - 1)/p_i - w_i^2/p_i^2) c_i^2 H_ai^2 ]
 *            / ((E0 - H_aa) N_d (N_d - 1)),
 * the inner sums over the distinct dets of the sample whose term passes
 * |H_ai c_i| > e, and per_sample[s] = S_s(eps2) - S_s(eps2_d), both
 * thresholds evaluated on the same samples in one pass.  The semistochastic
 * estimate is E2 = E2_det(eps2_d) + mean_s per_sample[s].
 *   draws   device uint32 [n_samples][n_draws], each < n_det, or NULL: the
 *           seed path draws them on the device with p_i = |c_i| / sum_j |c_j|
 *           by the alias method (sampling-probability equation; the paper
 *           cites Walker and Kronmal-Peterson): an alias table built by
 *           Vose's method on exact 128-bit integer masses (weights
 *           floor(|c_i| 2^(K-E)), 2^(E-1) <= max|c| < 2^E, K = 127 -
 *           2 ceil(log2 n_det)), and draw k of sample s taken from SplitMix64
 *           outputs 2(s n_draws + k) + 1 (bucket, multiply-shift) and + 2
 *           (64-bit threshold); shci_pt2_draws returns the same draws;
 *   seed    the SplitMix64 seed of the seed path (ignored with draws);
 *   eps2 <= eps2_d; n_draws in [2, 4096]; n_samples >= 1;
 *   n_samples * n_draws < 2^31;
 *   ws, ws_bytes  device workspace or NULL;
 *   per_sample  device FP64 [n_samples];
 *   mean, sem   host, nullable: mean and standard error (sd / sqrt(n_samples))
 *               of per_sample (sem = 0 when n_samples == 1). */
int shci_pt2_sample(shci_pt2_ctx* ctx, const uint64_t* dets, const double* c, int64_t n_det,
                    double e0, double eps2, double eps2_d, int32_t n_samples, int32_t n_draws,
                    const uint32_t* draws, uint64_t seed, int precision, void* ws, size_t ws_bytes,
                    void* stream, double* per_sample, double* mean, double* sem, shci_pt2_stats* st);

/* The seed path's draws alone: draws [n_samples][n_draws] (device, out) as
 * shci_pt2_sample makes them from c and seed.  ws, ws_bytes: workspace or
 * NULL.  Errors: SHCI_ERR_ARG, SHCI_ERR_NONFINITE (c not finite or all
 * zero). */
int shci_pt2_draws(shci_pt2_ctx* ctx, const double* c, int64_t n_det, uint64_t seed, int32_t n_samples,
                   int32_t n_draws, void* ws, size_t ws_bytes, void* stream, uint32_t* draws);

/* The alias table of p_i = |c_i| / sum_j |c_j| that the seed path draws
 * from: bucket k keeps k when a uniform 64-bit value is below threshold[k],
 * else it gives alias[k].  threshold device uint64 [n_det], alias device
 * uint32 [n_det] (out).  Errors as shci_pt2_draws. */
int shci_pt2_alias_table(shci_pt2_ctx* ctx, const double* c, int64_t n_det, void* ws, size_t ws_bytes,
                         void* stream, uint64_t* threshold, uint32_t* alias);

/* Stochastic part with one batch of P per sample (the stochastic step of the
 * paper's 3-step method, section IV): sample s keeps only the a whose
 * determinant hash h has h mod n_batches == sample_batch[s], and its estimate
 * is multiplied by n_batches (unbiased over a uniform choice of batch).
 *   n_batches     power of two in [1, 65536];
 *   sample_batch  device int32 [n_samples], each in [0, n_batches) (random
 *                 numbers of the method, passed in like the draws), or NULL:
 *                 sample s takes the top log2(n_batches) bits of SplitMix64
 *                 output 2 n_samples n_draws + s + 1 of `seed`.
 * Other arguments as shci_pt2_sample. */
int shci_pt2_sample_batched(shci_pt2_ctx* ctx, const uint64_t* dets, const double* c, int64_t n_det,
                            double e0, double eps2, double eps2_d, int32_t n_samples, int32_t n_draws,
                            const uint32_t* draws, int32_t n_batches, const int32_t* sample_batch,
                            uint64_t seed, int precision, void* ws, size_t ws_bytes, void* stream,
                            double* per_sample, double* mean, double* sem, shci_pt2_stats* st);

/* Per-batch statistics of the deterministic corrections (section IV): for
 * each listed batch b (h mod n_batches == b, h the determinant hash), over
 * the a outside V reached by a term with |H_ai c_i| > eps2,
 *   e_a = (A_a(eps2)^2 - A_a(eps2_hi)^2) / (E0 - H_aa),
 * A_a(e) the screened sum at threshold e (A_a(INFINITY) = 0, so eps2_hi =
 * INFINITY gives the plain contributions).  out[k] = {sum e_a, sum e_a^2,
 * number of a, number of kept terms}.  A batch whose records exceed the
 * record budget (or the workspace) fails with SHCI_ERR_WORKSPACE. */
typedef struct {
  double sum, sumsq;
  int64_t n_unique, n_terms;
} shci_pt2_batch;
int shci_pt2_det_batches(shci_pt2_ctx* ctx, const uint64_t* dets, const double* c, int64_t n_det,
                         double e0, double eps2, double eps2_hi, int32_t n_batches, const int32_t* batches,
                         int32_t n_list, int precision, void* ws, size_t ws_bytes, void* stream,
                         shci_pt2_batch* out, shci_pt2_stats* st);

/* The paper's 3-step perturbative correction (3-step equation, section IV):
 *   E2 = E2_dtm(eps2_dtm)
 *      + [E2_psto(eps2_psto) - E2_psto(eps2_dtm)]   pseudo-stochastic: batches of
 *        P (nb_psto) evaluated in order until the standard error of the sum
 *        over the unevaluated determinants is below 40% of target_error
 *      + mean_s [S_s(eps2) - S_s(eps2_psto)]        stochastic: one batch of P
 *        (of nb_sto) per sample, as shci_pt2_sample_batched.
 * err combines the pseudo-stochastic and stochastic standard errors.
 * draws and sample_batch may be NULL (seed path, as shci_pt2_sample and
 * shci_pt2_sample_batched).  The paper asks for at least 16
 * pseudo-stochastic batches and at least 10 samples; the call accepts
 * smaller values (small tests) and leaves that choice to the caller. */
typedef struct {
  double e2, err;
  double e2_dtm;
  double e2_psto, err_psto;
  int32_t psto_batches_used;
  double e2_sto, err_sto;
} shci_pt2_3step_result;
int shci_pt2_three_step(shci_pt2_ctx* ctx, const uint64_t* dets, const double* c, int64_t n_det,
                        double e0, double eps2_dtm, double eps2_psto, double eps2, double target_error,
                        int32_t nb_psto, int32_t nb_sto, int32_t n_samples, int32_t n_draws,
                        const uint32_t* draws, const int32_t* sample_batch, uint64_t seed, int precision,
                        void* ws, size_t ws_bytes, void* stream, double* per_sample, shci_pt2_3step_result* res);

/* Selection of new variational determinants from the same pass (variational
 * stage, section II.A): one deterministic pass with generation threshold
 * eps_gen, then among its perturbative determinants a outside V
 *   SHCI_SELECT_HCI:   every a, i.e. max_i |H_ai c_i| > eps_gen (the
 *                      heat-bath criterion with eps1 = eps_gen); value = A_a;
 *   SHCI_SELECT_CIPSI: |A_a^2 / (E0 - H_aa)| > threshold (the CIPSI energy
 *                      criterion, preselected at eps_gen); value = A_a^2 / D_a.
 *   out_keys  device uint64 [cap][4] (input layout), out_val device FP64 [cap];
 *   n_out     host: number selected.  SHCI_ERR_WORKSPACE if the pass has more
 *             than cap perturbative determinants.  Order unspecified but
 *             deterministic.  Scratch memory comes from the context's
 *             grow-only buffers. */
enum { SHCI_SELECT_HCI = 0, SHCI_SELECT_CIPSI = 1 };
int shci_pt2_select(shci_pt2_ctx* ctx, const uint64_t* dets, const double* c, int64_t n_det, double e0,
                double eps_gen, int mode, double threshold, int precision, void* stream, uint64_t* out_keys,
                double* out_val, int64_t cap, int64_t* n_out, shci_pt2_stats* st);

/* Adjoint of the stochastic part: the per-sample estimates of
 * shci_pt2_sample and the derivatives of their mean with respect to c and
 * E0, with the draws, p_i and the screening masks held at the forward point
 * (derivative of the stochastic PT2 equation):
 *   de2_dc[i] = mean_s sum_{a: (i,a) kept} [ 2 X_a w_i H_ai / p_i
 *       + 2 (w_i (N_d - 1)/p_i - w_i^2/p_i^2) c_i H_ai^2 - (the same over the
 *       eps2_d terms, with X_a^d) ] / ((E0 - H_aa) N_d (N_d - 1)),
 *   X_a = sum_i w_i c_i H_ai / p_i over the sample's kept terms of a.
 *   de2_dc    device FP64 [n_det], overwritten;
 *   de2_de0   host, nullable: mean over samples of dS_s/dE0.
 * The adjoint recomputes each sample's terms (a second generation pass)
 * and looks its per-a factors up in the sample's unique store.  Other
 * arguments as shci_pt2_sample; per_sample must be non-NULL. */
int shci_pt2_sample_grad(shci_pt2_ctx* ctx, const uint64_t* dets, const double* c, int64_t n_det,
                         double e0, double eps2, double eps2_d, int32_t n_samples, int32_t n_draws,
                         const uint32_t* draws, uint64_t seed, int precision, void* ws, size_t ws_bytes,
                         void* stream, double* per_sample, double* mean, double* sem, double* de2_dc,
                         double* de2_de0, shci_pt2_stats* st);

/* Gradient of the deterministic screened E2 with the screening mask held at
 * the given c:
 *   dE2/dc_i = sum_{a: (i,a) kept, a not in V} 2 H_ai A_a / (E0 - H_aa)
 *   dE2/dE0  = -sum_a A_a^2 / (E0 - H_aa)^2.
 * The forward pass runs first (precision as in shci_pt2_det).  mode
 * (enum shci_grad_mode):
 *   SHCI_GRAD_KEEP: every record carries its position; the reduce writes
 *     t * 2 A_a / D_a per record (t = H_ai c_i, 0 for a in V) and the sums
 *     over each source's records, divided by c_i, give dE2/dc_i (fixed
 *     order, deterministic); 12 more bytes per record;
 *   SHCI_GRAD_RECOMPUTE: the unique a are kept with 2 A_a / D_a and the
 *     adjoint regenerates the connections of every i and looks them up, so
 *     no per-term storage is kept (hash batches allowed);
 *   SHCI_GRAD_AUTO: keep when one pass holds every record, else recompute.
 * de2_dc: device FP64 [n_det]; e2, de2_de0: host, nullable; ws, ws_bytes:
 * workspace or NULL. */
int shci_pt2_grad(shci_pt2_ctx* ctx, const uint64_t* dets, const double* c, int64_t n_det,
                  double e0, double eps2, int precision, int mode, void* ws, size_t ws_bytes, void* stream,
                  double* e2, double* de2_dc, double* de2_de0, shci_pt2_stats* st);

/* y = H c on the variational space (section III: the alpha/beta string lists
 * of Table I and the connection loops of Algorithms 1-2), and the
 * variational energy <c|H|c>/<c|c>.  Determinants are grouped by their alpha
 * and by their beta string; row i visits its beta group (alpha singles and
 * doubles), its alpha group (beta singles and doubles) and, through the
 * alpha-singles lists, the determinants one alpha and one beta single away.
 *   dets   device uint64 [n_det][4] (input layout), unique; c device FP64 [n_det]
 *   y      device FP64 [n_det], out: sum_j H_ij c_j (H_ii c_i included)
 *   n_conn device uint32 [n_det] or NULL, out: the j != i one or two
 *          excitations from i
 *   e_var  host or NULL, out: <c|H|c> / <c|c>
 *   st     host or NULL: n_terms = sum of n_conn, n_records = length of the
 *          alpha-singles lists, ms_gen (lists), ms_reduce (rows), ms_total
 * FP64 throughout; rows are summed in a fixed order, so y is deterministic.
 * Errors: SHCI_ERR_ARG (NULL, n_det outside [1, 2^31 - 1)), SHCI_ERR_DET,
 * SHCI_ERR_DUP, SHCI_ERR_NONFINITE (c), SHCI_ERR_WORKSPACE, SHCI_ERR_HIP.
 * Scratch memory comes from the context's grow-only buffers. */
int shci_pt2_hc(shci_pt2_ctx* ctx, const uint64_t* dets, const double* c, int64_t n_det, void* stream,
                double* y, uint32_t* n_conn, double* e_var, shci_pt2_stats* st);

/* Message for the last non-OK status returned to the calling thread. */
const char* shci_pt2_last_error(void);

/* Library version string. */
const char* shci_pt2_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SHCI_PT2_H */
