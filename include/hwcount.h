/*
 * hwcount.h -- C ABI of libhwcount.so: Hasse-Weil point counts of
 * hyperelliptic curves over small finite fields on MI355X (gfx950).
 *
 * For a curve C_f : y^2 = f(X) = sum_{i<=2g+2} a_i X^i over F_q (q odd,
 * f square-free of degree 2g+1 or 2g+2; Sec. 1.1 of Raum, "Hyperelliptic
 * Curves over Small Finite Fields and GPU Accelerators") the library returns
 * N_k = #C_f(F_{q^k}) for k = 1..g, counted on the model in the weighted
 * projective plane P(1, g+1, 1):
 *
 *   N_k = r^0 + 2 r^square + (1 + chi(a_{2g+2}))        (decomposition of Sec. 1.1)
 *
 * with r^0 the roots of f in F_{q^k}, r^square the x with f(x) a nonzero
 * square, and the last term the points at infinity (one when deg f = 2g+1,
 * two or none when deg f = 2g+2).  The Hasse-Weil invariant of eq. (1.1) is
 * a_k = q^k + 1 - N_k.  It also returns the histogram of the tuples
 * (N_1..N_g), i.e. the a-tuple part of the map N_{g,q} of eq. (1.2), with
 * every input row counted once.
 *
 * Evaluation (default) uses Zech-logarithm arithmetic in HIP kernels:
 * elements as discrete logarithms to a primitive element with a zero
 * sentinel, additions through a Zech table (Sec. 2.3, eq. (2.1), encoding
 * (3.1), table (3.2)), the quadratic character read from the parity of the
 * logarithm (eq. (3.3)).  As an opt-in (HWC_OPT_MFMA) prime q <= 31 can be
 * counted instead by int8 matrix products of the coefficients with the
 * coordinates of the powers x^i over F_q, which gives the same sums.  Every
 * N_k is an exact integer either way.
 *
 * Coefficient codes.  A coefficient is an integer code c in [0, q).  For
 * q = p^e with e > 1, c = sum_i d_i p^i (0 <= d_i < p) stands for
 * sum_i d_i t^i in F_p[t]/(P_q) with P_q the lexicographically first
 * primitive monic polynomial of degree e over F_p (monic polynomials
 * t^e + b_{e-1} t^{e-1} + ... + b_0 ranked by the integer sum_i b_i p^i).
 * Rows are a_0 .. a_{2g+2}, constant term first, row-major [n][2g+3].
 *
 * Ownership.  The caller owns every input and output buffer; the library
 * owns its tables and scratch memory.  Functions return HWC_OK (0) or a
 * negative HWC_ERR_* code; hwc_last_error() gives a message.  Calls on one
 * context are serialised internally.  Supported: 1 <= g <= 4, odd prime
 * powers q with q^g <= 2^24 and q <= 32768.  Level tables of up to 131070
 * nonzero elements are staged in the 160 KiB LDS of a CU (e.g. q = 13 at
 * g = 4, q = 49 at g = 3, q = 293 at g = 2; the largest as half tables, the
 * rest following from the symmetry of the Zech logarithm); larger levels
 * keep their Zech tables in device memory, served by L2 and the MALL.
 * Histogram keys must fit 63 bits.
 */
#ifndef HWCOUNT_H
#define HWCOUNT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HWC_OK 0
#define HWC_ERR_NOT_ODD_PRIME_POWER (-1) /* q (or p) is not an odd prime power (prime) */
#define HWC_ERR_BAD_G (-2)               /* g outside 1..4 */
#define HWC_ERR_FIELD_TOO_LARGE (-3)     /* tables of F_{q^g} exceed what the kernels hold */
#define HWC_ERR_COEFF_RANGE (-4)         /* a code outside [0, q) */
#define HWC_ERR_DEGREE (-5)              /* a_{2g+2} = a_{2g+1} = 0 */
#define HWC_ERR_HIST_CAPACITY (-6)       /* histogram longer than its capacity; len holds the need */
#define HWC_ERR_OOM_BUDGET (-7)          /* table cache would exceed the context's HBM budget */
#define HWC_ERR_DEVICE (-8)              /* HIP error (message in hwc_last_error) */
#define HWC_ERR_SINGULAR (-9)            /* HWC_VALIDATE found a row that is not square-free */
#define HWC_ERR_ARG (-10)                /* null pointer, bad size or bad flag */
#define HWC_ERR_NO_DEVICE (-11)          /* counting asked of a host-only context */

/* flags */
#define HWC_FULL_SWEEP 1u /* level k sweeps every x of F_{q^k}; default: one x per Frobenius orbit */
#define HWC_PLAIN 2u      /* one kernel launch per (q, g, k) and a separate assembly; no graph */
#define HWC_VALIDATE 4u   /* host checks that every row is square-free (host-pointer call only) */
#define HWC_NO_GRAPH 8u   /* launch kernels directly instead of replaying a captured HIP graph */

typedef struct hwc_ctx hwc_ctx;
typedef struct hwc_field hwc_field;

typedef struct {
  uint32_t p, e, k, n;     /* F_Q = F_p[t]/(P), n = e*k, contains F_q, q = p^e */
  uint64_t q, Q;
  uint32_t modulus[41];    /* P, lex-first primitive, constant term first, modulus[n] = 1 */
  uint32_t qmodulus[41];   /* P_q, the same for degree e */
  uint32_t root_log;       /* log to t of the root of P_q used to embed F_q */
  uint64_t nprim_orbits;   /* Frobenius orbits of F_Q^x of size exactly k */
  uint64_t table_bytes;    /* host bytes of exp, log, Zech and embedding tables */
} hwc_field_desc;

/* Histogram of tuples, sorted ascending lexicographically.  The caller
 * allocates keys (capacity*g int32) and counts (capacity uint64). */
typedef struct {
  uint32_t g;
  uint64_t capacity;
  uint64_t len;            /* out: number of distinct tuples */
  int32_t* keys;
  uint64_t* counts;
} hwc_hist;

/* One request of a batch: device pointers, asynchronous. */
typedef struct {
  uint32_t q, g;
  const void* d_coeffs;    /* [n][2g+3] codes, int8 (coeff_bytes 1, q <= 127) or int16 (2) */
  int coeff_bytes;
  uint64_t n;
  int32_t* d_out_N;        /* [n][g]; required */
  int32_t* d_hist_keys;    /* [hist_capacity][g] or NULL (no histogram) */
  uint64_t* d_hist_counts; /* [hist_capacity] */
  uint64_t hist_capacity;
  uint64_t* d_hist_len;    /* device uint64: number of distinct tuples */
} hwc_job;

/* Context on HIP device `device` (-1: host-only context, which builds fields
 * but cannot count).  hbm_budget_bytes bounds the device table cache (0: no
 * bound).  Creates its own HIP stream.  Ownership of *out passes to the
 * caller; release it with hwc_ctx_destroy. */
int hwc_ctx_create(int device, uint64_t hbm_budget_bytes, hwc_ctx** out);
void hwc_ctx_destroy(hwc_ctx* ctx);

/* Message for the last error on ctx ("" if none).  Valid until the next call.
 * With ctx = NULL: why the calling thread's last hwc_ctx_create failed. */
const char* hwc_last_error(const hwc_ctx* ctx);

/* Builds F_{p^(e k)} with F_{p^e} embedded (Sec. 2.3, Sec. 3.1-3.2): the
 * lex-first primitive modulus, exp/log tables with the zero sentinel Q-1,
 * the Zech table with the sentinel where 1 + t^L = 0, the embedding of the
 * F_q codes and the Frobenius orbit representatives.  p must be an odd prime.
 * Idempotent: a second call with the same (p, e, k) returns a handle to the
 * same cached tables.  Release the handle with hwc_field_release. */
int hwc_build_field(hwc_ctx* ctx, uint32_t p, uint32_t e, uint32_t k, hwc_field** out);
int hwc_field_info(const hwc_field* f, hwc_field_desc* out);

/* Host copies of the tables of a field (any pointer may be NULL):
 * exp[Q-1] (packed sum_i b_i p^i of t^L), log[Q] (log[0] = Q-1),
 * zech[Q-1] (Q-1 where 1 + t^L = 0), emb[q] (log of each F_q code, emb[0] = Q-1),
 * prim_reps[nprim_orbits] (least log of each Frobenius orbit of size k). */
int hwc_field_tables(const hwc_field* f, uint32_t* exp, uint32_t* log, uint32_t* zech, uint32_t* emb,
                     uint32_t* prim_reps);
void hwc_field_release(hwc_field* f);

/* Counts n curves from host memory and waits for the result: N_k by the
 * decomposition of Sec. 1.1 for k = 1..g, and the histogram of the tuples,
 * the a-tuple part of eq. (1.2) (Algorithm 1's count of curves per tuple).
 * coeffs: [n][2g+3] int16 codes.  out_N: [n][g] int32 or NULL.  out_hist:
 * histogram or NULL (out_hist->g must equal g).  Returns HWC_ERR_COEFF_RANGE
 * / HWC_ERR_DEGREE for a bad row, HWC_ERR_HIST_CAPACITY when out_hist is too
 * short (out_hist->len is then the needed length; out_N is complete). */
int hwc_count_curves(hwc_ctx* ctx, uint32_t q, uint32_t g, const int16_t* coeffs, uint64_t n, int32_t* out_N,
                     hwc_hist* out_hist, uint32_t flags);

/* Device-pointer form of hwc_count_curves (the same N_k of Sec. 1.1 and
 * histogram of eq. (1.2)): enqueues the whole count on `stream` (a hipStream_t;
 * NULL = the context's stream) and returns without waiting.  Row errors are
 * found on the device and reported by hwc_ctx_status.  The histogram is
 * written when d_hist_keys is not NULL (d_hist_len receives its length; at
 * most hist_capacity entries are written).  Buffers must stay valid until
 * the stream reaches this work.  Where the top level sweeps at least 8192
 * points by Frobenius orbits, every tile's top-level sweep is shared out over
 * 8 waves whose counts are summed before N is assembled (not in the plain
 * form, which keeps one launch per level over whole tiles). */
int hwc_count_curves_dev(hwc_ctx* ctx, uint32_t q, uint32_t g, const void* d_coeffs, int coeff_bytes, uint64_t n,
                         int32_t* d_out_N, int32_t* d_hist_keys, uint64_t* d_hist_counts, uint64_t hist_capacity,
                         uint64_t* d_hist_len, uint32_t flags, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * count as hwc_count_curves_dev, with the same arguments, results, errors and
 * ownership of the caller's buffers, but this call allocates and frees
 * nothing.  Its scratch is a static device array of HWC_NOALLOC_SCRATCH_BYTES
 * per GPU (held from the library's load until the process ends), so:
 *  - the plan of (q, g) and the sweep of `flags` must already be resident,
 *    made by an earlier call such as hwc_plan_info or a count on this
 *    context (HWC_ERR_ARG otherwise; a plan can leave the cache under an HBM
 *    budget);
 *  - a request whose scratch exceeds the array fails with HWC_ERR_ARG before
 *    anything is enqueued (the need is about 31 bytes per row with the
 *    histogram, 6 without, plus (2g+3) * coeff_bytes on the Zech path, which
 *    counts rows with zero coefficients as dense translates, plus 4g with
 *    HWC_PLAIN: up to about 1.6 million rows at g = 3 with int8 codes and the
 *    histogram, about a million at g = 4 with int16 codes and every part);
 *  - kernels are launched directly on `stream`, never from a graph;
 *  - every call on one GPU, from any context, uses that GPU's one array and
 *    leaves its contents behind: calls that overlap on one GPU race, and the
 *    caller must order them (one stream, or events).
 * HWC_VALIDATE is rejected (it needs host rows). */
#define HWC_NOALLOC_SCRATCH_BYTES (64ull << 20)
int hwc_count_curves_dev_noalloc(hwc_ctx* ctx, uint32_t q, uint32_t g, const void* d_coeffs, int coeff_bytes,
                                 uint64_t n, int32_t* d_out_N, int32_t* d_hist_keys, uint64_t* d_hist_counts,
                                 uint64_t hist_capacity, uint64_t* d_hist_len, uint32_t flags, void* stream);

/* As hwc_count_curves_dev, plus the factorization partition lambda(f) of
 * every row (Sec. 1.1: the partition of 2g+2 by the degrees of the
 * irreducible factors of f over F_q, with an extra part 1 when deg f = 2g+1),
 * the second argument of the map N_{g,q} of eq. (1.2) -- Algorithm 1 takes
 * it from the root counts r^0 where they decide it, else by factoring.
 * d_out_lambda: [n] uint32 codes; the multiplicity of part j (1 <= j <= 10)
 * sits in bits [s_j, s_j + w_j) with s = 0, 4, 7, 9, 11, 13, 14, 15, 16, 17
 * and w = 4, 3, 2, 2, 2, 1, 1, 1, 1, 1; 0xFFFFFFFF marks a row whose root
 * counts are inconsistent with a square-free f.  The histogram (when
 * d_hist_keys is not NULL) has g+1 columns: N_1..N_g and the code, sorted
 * lexicographically.  Needs q <= 10923 (HWC_ERR_FIELD_TOO_LARGE otherwise);
 * other errors and ownership as hwc_count_curves_dev. */
int hwc_count_lambda_dev(hwc_ctx* ctx, uint32_t q, uint32_t g, const void* d_coeffs, int coeff_bytes, uint64_t n,
                         int32_t* d_out_N, uint32_t* d_out_lambda, int32_t* d_hist_keys, uint64_t* d_hist_counts,
                         uint64_t hist_capacity, uint64_t* d_hist_len, uint32_t flags, void* stream);

/* The rows the counting entry points evaluate in place of the caller's.  A
 * translate f(x + t), t in F_q, has the same N_k, factorization pattern and
 * discriminant as f (x -> x + t permutes every F_{q^k} and keeps the degree
 * and leading coefficient; Algorithm 1 divides out the same equivalence).
 * When the plan of (q, g) translates (q <= 32 and HWC_OPT_SHIFT on, the
 * default), a row with a zero coefficient below its leading one becomes
 * f(x + t) for the first code t = 1, 2, .., 8 that leaves no such zero, since
 * such dense rows are cheaper to count; every other row is copied.  d_coeffs
 * as in hwc_count_curves_dev; d_out: [n][2g+3] of the same coeff_bytes, device
 * memory, owned by the caller, not overlapping d_coeffs.  Enqueued on
 * `stream`; errors as hwc_count_curves_dev (rows are not validated here). */
int hwc_translate_dev(hwc_ctx* ctx, uint32_t q, uint32_t g, const void* d_coeffs, int coeff_bytes, uint64_t n,
                      void* d_out, void* stream);

/* The map N_{g,q} of eq. (1.2) over every square-free f of degree 2g+1 and
 * 2g+2, by Algorithm 1: the reduced, twist-reduced representatives of
 * Sec. 1.2-1.3 are generated and counted on the device (with lambda), each
 * weighted by its multiplicity mult(f) and entered twice, for f and for its
 * quadratic twist (Algorithm 1 adds both; the twist's invariants follow from
 * the corrected relation a_k(nf) = (-1)^k a_k(f)).  Output (host memory, in
 * lexicographic order): keys[len][g+1] = a_1..a_g, lambda code (a_k = q^k + 1
 * - N_k, eq. 1.1; code as in hwc_count_lambda_dev) and counts[len]; *len is
 * the number of entries (HWC_ERR_HIST_CAPACITY when it exceeds capacity),
 * *reps (may be NULL) the number of representatives evaluated.  The counts
 * add up to (q-1)(q^{2g+2} - q^{2g+1}) + (q-1)(q^{2g+1} - q^{2g}), the number
 * of square-free polynomials of those degrees.  Synchronous; needs
 * q <= 10923. */
int hwc_count_map(hwc_ctx* ctx, uint32_t q, uint32_t g, int32_t* keys, uint64_t* counts, uint64_t capacity,
                  uint64_t* len, uint64_t* reps, uint32_t flags);

/* One curve over large fields -- the single-curve experiment of Table 1
 * (Sec. 4), with the paper's lane-per-x layout: every device lane evaluates
 * f at its own x.  coeffs: [2g+3] int16 codes (host).  Counts N_1..N_kmax
 * into out_N[kmax] (int64, host) for q^kmax <= 2^24; level j sweeps the
 * primitive Frobenius orbits of F_{q^j} (HWC_FULL_SWEEP: every nonzero x).
 * The Zech tables (one period, u32, built on the host and kept on the device
 * per field) serve from L2/MALL.  timings (may be NULL): [3] milliseconds of
 * table construction on the host, table upload, and the kernels (HIP
 * events).  Synchronous; the row must be square-free for N to be a point
 * count (not checked). */
int hwc_count_single(hwc_ctx* ctx, uint32_t q, uint32_t g, const int16_t* coeffs, uint32_t kmax, int64_t* out_N,
                     double* timings, uint32_t flags);

/* Diagnostic: the rate of dependent random u16 gathers from an LDS table of
 * table_entries entries (the count kernel's bound, Sec. 3.2 tables read at
 * random), measured with `chains` (1, 2 or 4) independent chains per lane on
 * a grid of 32 workgroups of 256 lanes per CU.  *lookups_per_s receives the
 * best of two timed runs.  Synchronous. */
int hwc_lds_gather_rate(hwc_ctx* ctx, uint32_t table_entries, uint32_t chains, double* lookups_per_s);

/* Diagnostic: the issue rate of plain 32-bit vector instructions (chains of
 * add, subtract and min, eight independent chains per lane, eight waves per
 * SIMD), in wave64 instructions per second over the whole device -- the
 * other resource the count kernels' table walks (Sec. 3.3) saturate.  Best of
 * two timed runs; synchronous. */
int hwc_valu_issue_rate(hwc_ctx* ctx, double* insts_per_s);

/* Diagnostic: the rate of dependent random u32 gathers from a table of
 * table_entries entries (64 .. 2^26) in device memory -- the placement of
 * Zech tables too large for LDS (Sec. 3.2 tables read at random, served by
 * L2 and the MALL) -- with `chains` (1, 2 or 4) independent chains per lane
 * on a grid of 32 workgroups of 256 lanes per CU.  *lookups_per_s receives
 * the best of two timed runs.  Uses the context's synchronous scratch for
 * the table; synchronous. */
int hwc_device_gather_rate(hwc_ctx* ctx, uint64_t table_entries, uint32_t chains, double* lookups_per_s);

/* Several requests (each as hwc_count_curves_dev: N_k of Sec. 1.1 and the
 * histogram of eq. (1.2)) in the persistent batched form, enqueued on
 * `stream`: the rows of every Zech-path job are bucketed, then a persistent
 * multi-plan launch takes the jobs one after another, most expensive tiles
 * first, every wave popping tiles from the current job's queue (the LDS
 * image restaged only when a workgroup moves to a job of another plan; a
 * job whose top level sweeps at least 8192 points by orbits has each tile's
 * top-level sweep shared out over 8 waves, whose counts are summed before N
 * is assembled) -- the loops over the curves and fields of Algorithm 1 in one
 * launch, where
 * the paper launches once per curve and field (Sec. 3.3); jobs on the
 * opt-in matrix-product path follow as their own launches on the same
 * stream.
 * Without HWC_NO_GRAPH the whole batch is captured once into a HIP graph
 * (keyed by the jobs' shapes and pointers) and replayed.  Errors as
 * hwc_count_curves_dev; a plan that cannot fit the HBM budget fails the
 * call (HWC_ERR_OOM_BUDGET) before anything is enqueued. */
int hwc_count_batch(hwc_ctx* ctx, const hwc_job* jobs, size_t njobs, uint32_t flags, void* stream);

/* Waits for `stream` (NULL = context stream) and returns the first row error
 * that device-side validation found since the last call (HWC_OK if none). */
int hwc_ctx_status(hwc_ctx* ctx, void* stream);

/* Profiling.  While enabled, every call is launched directly (no graph) and
 * HIP events are recorded on its launch stream around three phases: curve
 * bucketing, the count kernel(s) (with assembly in the plain form), and the
 * histogram.  hwc_ctx_profile_read waits for the recorded events, returns the
 * summed milliseconds of each phase and the number of calls, and resets. */
int hwc_ctx_profile(hwc_ctx* ctx, int enable);
int hwc_ctx_profile_read(hwc_ctx* ctx, double* prep_ms, double* count_ms, double* hist_ms, uint64_t* calls);

/* Launch and layout options of a context (the autotuner's search space).
 * Setting one drops the cached plans and graphs. */
#define HWC_OPT_SPLIT 1         /* 1 (default): split evaluation over the m-th roots of unity of F_q on
                                   every level with at least HWC_OPT_SPLIT_MIN_M elements: m = 4 when
                                   4 | q-1, else 3 on byte-unit levels when 3 | q-1, else 2; 0: plain
                                   Horner at every x */
#define HWC_OPT_BLOCK 2         /* threads per workgroup of the count kernel: 0 (auto), 256, 512, 1024 */
#define HWC_OPT_WG_PER_CU 3     /* cap on workgroups per CU of the persistent grid; 0: occupancy limit */
#define HWC_OPT_DEVICE_TABLES 4 /* bit mask over levels: bit j-1 set puts level j's Zech table in device
                                    memory (served by L2/MALL) instead of LDS; 0..15 */
#define HWC_OPT_WAVES_PER_SIMD 5 /* count-kernel build that leaves registers for at least 6 or 8 waves per SIMD
                                    (0 or 1: no constraint) */
#define HWC_OPT_SPLIT_MIN_M 6     /* split only levels with at least this many nonzero elements (default 64):
                                    on small fields a wave meets vanishing bases too often */
#define HWC_OPT_MFMA 8            /* 0 (default): Zech logarithms for every plan.  1 (opt-in): for prime
                                    q <= 31, when the level images fit LDS (the top level may be split over
                                    several passes), f(x) is evaluated as an int8 matrix product of the
                                    coefficients with the coordinates of the powers x^i over F_q (Sec. 1.1's
                                    sums, exact in int32), the character read from a table */
#define HWC_OPT_SHIFT 7           /* 1 (default): for q <= 32, a row with a zero coefficient below its leading
                                    one is counted as f(x + t), t in F_q, when some t (of the first 8 tried)
                                    leaves no such zero -- same N_k, factorization pattern and discriminant
                                    (x -> x + t permutes F_{q^k}); the caller's rows are not modified.
                                    0: rows are counted as given */
int hwc_ctx_set_option(hwc_ctx* ctx, int opt, int64_t value);
/* The same option for the plan of (q, g) and the sweep of `flags` only
 * (overrides the context default; used to apply autotuned settings). */
int hwc_ctx_set_plan_option(hwc_ctx* ctx, uint32_t q, uint32_t g, uint32_t flags, int opt, int64_t value);

/* Geometry of the counting plan for (q, g) and the sweep of `flags` (built
 * and cached if needed): per level j = 1..g, levels[j-1] receives the order
 * M of F_{q^j}^x, the table form (0: u16 in LDS, byte units; 1: u16 in LDS,
 * folded index over two periods; 2: u32 in device memory; 3: u16 in LDS, one
 * period, for M up to 65534; 4: half a period of 17-bit entries in LDS, for M
 * up to 131070; 5: the same half period as u32 entries in LDS, where it fits
 * the LDS image, if need be with the levels below it in device memory),
 * the number nx of swept x, the
 * weight of each, the split factor m (0: plain Horner; else the sweep runs nt
 * tuples of m points x w^s, w^m = 1, sharing the sub-polynomial values at
 * x^m, plus ns single points), the LDS bytes of the plan, and mfma = 1 when
 * the plan counts by int8 matrix products (HWC_OPT_MFMA) instead of Zech
 * logarithms, 2 when it does so in the balanced form (p = 11, 13: one
 * 24-bit multiply-high per coordinate for the quotients). */
typedef struct {
  uint32_t M, form, nx, weight, msplit, nt, ns, lds_bytes, mfma;
} hwc_level_desc;
int hwc_plan_info(hwc_ctx* ctx, uint32_t q, uint32_t g, uint32_t flags, hwc_level_desc* levels);

/* Table-cache statistics: plans resident, device bytes of their tables, hits
 * and misses of the cache, plans evicted (least recently used first) to stay
 * within the HBM budget, and bytes released but not yet freed (memory that
 * work still in flight may read; it is freed once that work is complete and
 * counts against the budget until then).  Any pointer may be NULL. */
int hwc_ctx_stats(const hwc_ctx* ctx, uint64_t* plans_resident, uint64_t* table_bytes, uint64_t* cache_hits,
                  uint64_t* cache_misses, uint64_t* evictions, uint64_t* pending_free_bytes);

/* Preallocates the scratch of the calls enqueued on `stream` (NULL = the
 * context's stream) for requests and batches of up to max_curves rows in
 * total over at most max_jobs jobs (any g, int8 or int16 codes), so that
 * such calls never grow a buffer while earlier work is in flight -- a
 * serving loop calls it once per stream before it starts.  Calls on
 * different streams use different scratch (up to four streams; more share),
 * so their kernels overlap on the device.  Synchronous; HWC_ERR_ARG for
 * max_curves >= 2^31 or max_jobs outside 1..65535. */
int hwc_ctx_reserve(hwc_ctx* ctx, uint64_t max_curves, uint32_t max_jobs, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* HWCOUNT_H */
