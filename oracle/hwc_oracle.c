/*
 * hwc_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow CPU point counter for hyperelliptic curves y^2 = f(x) over
 * F_q (q odd).  Only tests/, the package smoke check and the benchmark's CPU
 * baseline may load it; the product path never calls it.
 *
 * What it computes.  For a square-free f of degree 2g+1 or 2g+2 with
 * coefficients in F_q and k >= 1, N_k(f) = #C_f(F_{q^k}), the number of
 * points of the model of C_f in the weighted projective plane P(1, g+1, 1)
 * (Sec. 1.1):
 *   * affine points: pairs (x, y) in F_{q^k}^2 with y^2 = f(x).  For each x
 *     this is 1 when f(x) = 0, 2 when f(x) is a nonzero square and 0
 *     otherwise -- the decomposition r^0 + 2 r^square of Sec. 1.1 and the
 *     loop body of Algorithm 1;
 *   * points at infinity: 1 + chi(f(infinity)) with f(infinity) = c_{2g+2}
 *     (Sec. 1.1): one point when deg f = 2g+1, two or none when deg f = 2g+2
 *     according to whether c_{2g+2} is a square in F_{q^k}.
 * Everything is done with the definition: elements of F_{p^n} are
 * polynomials in t over F_p reduced modulo a primitive polynomial (the
 * representation of Sec. 2.2), products are schoolbook products reduced
 * modulo the polynomial and modulo p, and "is a nonzero square" is read
 * from a table made by squaring every nonzero element.  There are no
 * discrete logarithms, no Zech tables and no lookup of sums.
 *
 * Conventions (the paper leaves them open; these are the readings adopted):
 *   * a primitive monic polynomial of degree n over F_p is written
 *     t^n + a_{n-1} t^{n-1} + ... + a_0; candidates are ordered by the
 *     integer sum_i a_i p^i and the first primitive one is used
 *     ("lex-first").  A variant takes the last one ("lex-last") to show
 *     that counts do not depend on the model of F_{q^k};
 *   * an F_q coefficient is an integer code c = sum_i d_i p^i, standing for
 *     sum_i d_i t^i in F_p[t]/(P_q) with P_q the lex-first primitive
 *     polynomial of degree e (q = p^e);
 *   * F_q sits in F_{q^k} = F_p[t]/(P_Q) through a root z of P_q in F_Q;
 *     the default root is the one with the smallest packed value
 *     sum_i b_i p^i, a variant takes the largest.  Any root gives the same
 *     counts, since two roots differ by a Frobenius automorphism.
 * Coefficient rows are a_0 .. a_{2g+2}, constant term first.
 *
 * It also returns the factorization partition lambda(f) of eq. (1.2) by
 * distinct-degree factorization (see orc_factor_degrees below).
 *
 * Parity pins (tests/test_oracle_pins.py): brute-force pair counting on
 * tiny fields, the Weil bound, the quadratic twist in its corrected form,
 * the L-polynomial prediction of N_{g+1}, L(1) > 0, a closed form for
 * x^{2g+1} + c, invariance under X -> aX + b, f -> s^2 f and coefficient
 * reversal, and independence of the modulus and of the root.  Pins of
 * lambda (tests/test_oracle_lambda_pins.py): trial division by every monic
 * polynomial of small degree in table-built field models, and Gauss's count
 * of irreducible polynomials over full enumerations.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

#define ORC_MAXN 24        /* max extension degree over F_p */
#define ORC_MAXCOEF 32     /* max 2g+3 */

typedef struct {
  int p, n;                /* F_{p^n} = F_p[t]/(P) */
  int P[ORC_MAXN + 1];     /* monic: P[n] = 1 */
  int64_t Q;               /* p^n */
} orc_field;

/* ---------- integer helpers ---------- */

static int orc_factor(int64_t q, int *p, int *e) {
  if (q < 3 || (q % 2) == 0) return -1;
  int64_t f = 0;
  for (int64_t d = 3; d * d <= q; d += 2)
    if (q % d == 0) { f = d; break; }
  if (!f) f = q;
  int n = 0;
  int64_t r = q;
  while (r % f == 0) { r /= f; ++n; }
  if (r != 1) return -1;
  *p = (int)f;
  *e = n;
  return 0;
}

/* ---------- element arithmetic on digit vectors ---------- */

static void orc_unpack(const orc_field *F, int64_t v, int *a) {
  for (int i = 0; i < F->n; ++i) { a[i] = (int)(v % F->p); v /= F->p; }
}

static int64_t orc_pack(const orc_field *F, const int *a) {
  int64_t v = 0;
  for (int i = F->n - 1; i >= 0; --i) v = v * F->p + a[i];
  return v;
}

static void orc_add(const orc_field *F, const int *a, const int *b, int *out) {
  for (int i = 0; i < F->n; ++i) {
    int s = a[i] + b[i];
    out[i] = s >= F->p ? s - F->p : s;
  }
}

/* schoolbook product, then reduction modulo P and p */
static void orc_mul(const orc_field *F, const int *a, const int *b, int *out) {
  int n = F->n, p = F->p;
  int64_t c[2 * ORC_MAXN];
  for (int i = 0; i < 2 * n - 1; ++i) c[i] = 0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) c[i + j] += (int64_t)a[i] * b[j];
  for (int i = 0; i < 2 * n - 1; ++i) c[i] %= p;
  /* t^n = -(P[0] + ... + P[n-1] t^{n-1}) */
  for (int d = 2 * n - 2; d >= n; --d) {
    int64_t top = c[d] % p;
    c[d] = 0;
    if (top == 0) continue;
    for (int i = 0; i < n; ++i) c[d - n + i] = (c[d - n + i] - top * F->P[i]) % p;
  }
  for (int i = 0; i < n; ++i) {
    int64_t v = c[i] % p;
    out[i] = (int)(v < 0 ? v + p : v);
  }
}

static int orc_is_zero(const orc_field *F, const int *a) {
  for (int i = 0; i < F->n; ++i) if (a[i]) return 0;
  return 1;
}

static int orc_is_one(const orc_field *F, const int *a) {
  if (a[0] != 1) return 0;
  for (int i = 1; i < F->n; ++i) if (a[i]) return 0;
  return 1;
}

/* Is t primitive in F_p[t]/(P)?  Walk its powers: it must first return to 1
 * after exactly p^n - 1 steps. */
static int orc_t_is_primitive(const orc_field *F) {
  int x[ORC_MAXN], t[ORC_MAXN], y[ORC_MAXN];
  memset(t, 0, sizeof(t));
  if (F->n == 1) t[0] = (F->p - F->P[0]) % F->p; /* t = -P[0] */
  else t[1] = 1;
  memset(x, 0, sizeof(x));
  x[0] = 1;
  int64_t M = F->Q - 1;
  for (int64_t k = 1; k <= M; ++k) {
    orc_mul(F, x, t, y);
    memcpy(x, y, sizeof(int) * F->n);
    if (orc_is_one(F, x)) return k == M;
    if (orc_is_zero(F, x)) return 0;
  }
  return 0;
}

/* Lex-first (last = 0) or lex-last (last = 1) primitive monic polynomial of
 * degree n over F_p.  Fills F; returns 0 on success. */
static int orc_primitive(int p, int n, int last, orc_field *F) {
  if (n < 1 || n > ORC_MAXN) return -1;
  memset(F, 0, sizeof(*F));
  F->p = p;
  F->n = n;
  int64_t Q = 1;
  for (int i = 0; i < n; ++i) Q *= p;
  F->Q = Q;
  for (int64_t s = 0; s < Q; ++s) {
    int64_t v = last ? (Q - 1 - s) : s;
    int64_t w = v;
    for (int i = 0; i < n; ++i) { F->P[i] = (int)(w % p); w /= p; }
    F->P[n] = 1;
    if (F->P[0] == 0) continue;
    if (orc_t_is_primitive(F)) return 0;
  }
  return -1;
}

/* ---------- the count ---------- */

typedef struct {
  int q, p, e, g, k;
  orc_field FQ;                 /* F_{q^k} */
  int emb[4096][ORC_MAXN];      /* code -> element of F_{q^k} (digits) */
  uint8_t *sq;                  /* sq[packed y] = 1 iff y is a nonzero square */
} orc_level;

/* Builds F_{q^k}, the embedding of the coefficient codes and the square table. */
static int orc_level_init(orc_level *L, int q, int g, int k, int modulus_last, int root_last) {
  memset(L, 0, sizeof(*L));
  if (orc_factor(q, &L->p, &L->e)) return -1;
  if (q > 4096) return -1;
  L->q = q; L->g = g; L->k = k;
  if (orc_primitive(L->p, L->e * k, modulus_last, &L->FQ)) return -1;
  orc_field Fq;
  if (orc_primitive(L->p, L->e, 0, &Fq)) return -1;   /* coefficient convention: always lex-first */
  const orc_field *F = &L->FQ;
  int n = F->n;
  /* a root z of P_q in F_Q: scan all elements, keep the smallest (or largest) */
  int64_t zpack = -1;
  int z[ORC_MAXN], acc[ORC_MAXN], tmp[ORC_MAXN], cz[ORC_MAXN];
  for (int64_t v = 0; v < F->Q; ++v) {
    orc_unpack(F, v, z);
    /* Horner: P_q(z) with P_q[i] in F_p embedded as constants */
    memset(acc, 0, sizeof(acc));
    acc[0] = 1; /* leading coefficient 1 */
    for (int i = Fq.n - 1; i >= 0; --i) {
      orc_mul(F, acc, z, tmp);
      memset(cz, 0, sizeof(cz));
      cz[0] = Fq.P[i];
      orc_add(F, tmp, cz, acc);
    }
    if (orc_is_zero(F, acc)) {
      zpack = v;
      if (!root_last) break;
    }
  }
  if (zpack < 0) return -1;
  orc_unpack(F, zpack, z);
  /* emb[c] = sum_i d_i z^i */
  for (int c = 0; c < q; ++c) {
    int zp[ORC_MAXN], out[ORC_MAXN], term[ORC_MAXN];
    memset(zp, 0, sizeof(zp));
    zp[0] = 1;
    memset(out, 0, sizeof(out));
    int w = c;
    for (int i = 0; i < Fq.n; ++i) {
      int d = w % L->p;
      w /= L->p;
      memset(term, 0, sizeof(term));
      for (int j = 0; j < n; ++j) term[j] = (int)(((int64_t)zp[j] * d) % L->p);
      orc_add(F, out, term, tmp);
      memcpy(out, tmp, sizeof(int) * n);
      orc_mul(F, zp, z, tmp);
      memcpy(zp, tmp, sizeof(int) * n);
    }
    memcpy(L->emb[c], out, sizeof(int) * n);
  }
  /* squares: square every nonzero element */
  L->sq = (uint8_t *)calloc((size_t)F->Q, 1);
  if (!L->sq) return -1;
  int x[ORC_MAXN], y[ORC_MAXN];
  for (int64_t v = 1; v < F->Q; ++v) {
    orc_unpack(F, v, x);
    orc_mul(F, x, x, y);
    L->sq[orc_pack(F, y)] = 1;
  }
  return 0;
}

static void orc_level_free(orc_level *L) { free(L->sq); L->sq = NULL; }

/* N_k for one curve (codes a_0..a_{2g+2}) */
static int64_t orc_count_one(const orc_level *L, const int16_t *codes) {
  const orc_field *F = &L->FQ;
  int g = L->g, ncoef = 2 * g + 3;
  int d = ncoef - 1;
  while (d > 0 && codes[d] == 0) --d;
  int x[ORC_MAXN], y[ORC_MAXN], tmp[ORC_MAXN];
  int64_t pts = 0;
  for (int64_t v = 0; v < F->Q; ++v) {
    orc_unpack(F, v, x);
    memcpy(y, L->emb[codes[d]], sizeof(int) * F->n);
    for (int i = d - 1; i >= 0; --i) {
      orc_mul(F, y, x, tmp);
      orc_add(F, tmp, L->emb[codes[i]], y);
    }
    if (orc_is_zero(F, y)) pts += 1;
    else if (L->sq[orc_pack(F, y)]) pts += 2;
  }
  /* points at infinity of the model in P(1, g+1, 1) */
  int lead = codes[2 * g + 2];
  if (lead == 0) pts += 1;
  else pts += L->sq[orc_pack(F, L->emb[lead])] ? 2 : 0;
  return pts;
}

typedef struct {
  const orc_level *L;
  const int16_t *codes;
  int ncoef, kidx, kcount;
  int64_t start, count;
  int32_t *out;
} orc_job;

static void *orc_worker(void *arg) {
  orc_job *J = (orc_job *)arg;
  for (int64_t i = J->start; i < J->start + J->count; ++i)
    J->out[i * J->kcount + J->kidx] = (int32_t)orc_count_one(J->L, J->codes + i * J->ncoef);
  return NULL;
}

/* ---------------------------- public API ------------------------------ */

/* Coefficients of the lex-first (last = 0) or lex-last (last = 1) primitive
 * monic polynomial of degree n over F_p: out[0..n] with out[n] = 1. */
int orc_primitive_poly(int p, int n, int last, int *out) {
  orc_field F;
  if (orc_primitive(p, n, last, &F)) return -1;
  memcpy(out, F.P, sizeof(int) * (n + 1));
  return 0;
}

/* Validate one row: codes in [0, q), degree 2g+1 or 2g+2. */
static int orc_check_rows(int q, int g, const int16_t *codes, int64_t ncurves) {
  int ncoef = 2 * g + 3;
  for (int64_t i = 0; i < ncurves; ++i) {
    const int16_t *c = codes + i * ncoef;
    for (int j = 0; j < ncoef; ++j) if (c[j] < 0 || c[j] >= q) return -4;
    if (c[ncoef - 1] == 0 && c[ncoef - 2] == 0) return -5;
  }
  return 0;
}

/* N_k for k = 1..kmax, for every curve: out[i*kmax + (k-1)].
 * variant bit 0: lex-last modulus for F_{q^k}; bit 1: largest root for the
 * embedding.  Returns 0, or a negative code (-1 bad q, -2 bad g, -4 code out
 * of range, -5 degree below 2g+1, -3 field too large). */
int orc_count_curves(int q, int g, int kmax, const int16_t *codes, int64_t ncurves,
                     int32_t *out, int threads, int variant) {
  int p, e;
  if (orc_factor(q, &p, &e) || q > 4096) return -1;
  if (g < 1 || 2 * g + 3 > ORC_MAXCOEF || kmax < 1) return -2;
  if (e * kmax > ORC_MAXN) return -3;
  int rc = orc_check_rows(q, g, codes, ncurves);
  if (rc) return rc;
  if (threads < 1) threads = 1;
  if (threads > 256) threads = 256;
  for (int k = 1; k <= kmax; ++k) {
    orc_level *L = (orc_level *)malloc(sizeof(orc_level));
    if (!L) return -3;
    if (orc_level_init(L, q, g, k, variant & 1, (variant >> 1) & 1)) { orc_level_free(L); free(L); return -3; }
    pthread_t th[256];
    orc_job jobs[256];
    int64_t per = (ncurves + threads - 1) / threads;
    int used = 0;
    for (int t = 0; t < threads; ++t) {
      int64_t s = (int64_t)t * per;
      if (s >= ncurves) break;
      jobs[t].L = L; jobs[t].codes = codes; jobs[t].ncoef = 2 * g + 3;
      jobs[t].kidx = k - 1; jobs[t].kcount = kmax; jobs[t].out = out;
      jobs[t].start = s; jobs[t].count = (ncurves - s < per) ? ncurves - s : per;
      used++;
    }
    int started = 0;
    for (int t = 0; t < used; ++t) {
      if (pthread_create(&th[t], NULL, orc_worker, &jobs[t])) break;
      started++;
    }
    for (int t = started; t < used; ++t) orc_worker(&jobs[t]);
    for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
    orc_level_free(L);
    free(L);
  }
  return 0;
}

/* Square table of F_{p^n} (lex-first modulus): out[v] = 1 iff the element
 * with packed value v is a nonzero square.  out has p^n bytes. */
int orc_square_table(int p, int n, uint8_t *out) {
  orc_field F;
  if (orc_primitive(p, n, 0, &F)) return -1;
  memset(out, 0, (size_t)F.Q);
  int x[ORC_MAXN], y[ORC_MAXN];
  for (int64_t v = 1; v < F.Q; ++v) {
    orc_unpack(&F, v, x);
    orc_mul(&F, x, x, y);
    out[orc_pack(&F, y)] = 1;
  }
  return 0;
}

/* Product of two packed elements of F_{p^n} = F_p[t]/(lex-first primitive). */
int64_t orc_field_mul(int p, int n, int64_t a, int64_t b) {
  orc_field F;
  if (orc_primitive(p, n, 0, &F)) return -1;
  int x[ORC_MAXN], y[ORC_MAXN], z[ORC_MAXN];
  memset(x, 0, sizeof(x));
  memset(y, 0, sizeof(y));
  orc_unpack(&F, a, x);
  orc_unpack(&F, b, y);
  orc_mul(&F, x, y, z);
  return orc_pack(&F, z);
}

/* Histogram of tuples: rows of N (ncurves x width, int32) sorted
 * lexicographically, equal rows merged.  Writes up to cap distinct rows to
 * keys (cap x width) and their multiplicities to counts; returns the number
 * of distinct rows. */
static int orc_hist_width;
static const int32_t *orc_hist_base;
static int orc_row_cmp(const void *a, const void *b) {
  const int32_t *x = orc_hist_base + (*(const int64_t *)a) * orc_hist_width;
  const int32_t *y = orc_hist_base + (*(const int64_t *)b) * orc_hist_width;
  for (int i = 0; i < orc_hist_width; ++i) {
    if (x[i] < y[i]) return -1;
    if (x[i] > y[i]) return 1;
  }
  return 0;
}

int64_t orc_histogram(const int32_t *N, int64_t ncurves, int width, int32_t *keys, uint64_t *counts, int64_t cap) {
  int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ncurves > 0 ? ncurves : 1));
  if (!idx) return -1;
  for (int64_t i = 0; i < ncurves; ++i) idx[i] = i;
  orc_hist_width = width;
  orc_hist_base = N;
  qsort(idx, (size_t)ncurves, sizeof(int64_t), orc_row_cmp);
  int64_t distinct = 0;
  for (int64_t i = 0; i < ncurves;) {
    int64_t j = i + 1;
    while (j < ncurves && orc_row_cmp(&idx[i], &idx[j]) == 0) ++j;
    if (distinct < cap) {
      memcpy(keys + distinct * width, N + idx[i] * width, sizeof(int32_t) * width);
      counts[distinct] = (uint64_t)(j - i);
    }
    distinct++;
    i = j;
  }
  free(idx);
  return distinct;
}

/* ---------- factorization partition lambda(f) (Sec. 1.1, eq. 1.2) ----------
 *
 * lambda(f) is the partition of 2g+2 given by the degrees of the irreducible
 * factors of f over F_q, with an extra part 1 when deg f = 2g+1.  The oracle
 * finds it by distinct-degree factorization (the textbook algorithm: the
 * product of the monic irreducible factors of degree k of a square-free
 * monic h is gcd(h, X^{q^k} - X) once all factors of smaller degree have
 * been divided out), with plain polynomial arithmetic over F_q: coefficients
 * are digit vectors of F_p[t]/(P_q) (the code convention above), products
 * are schoolbook, inverses are a^{q-2}.
 */

#define ORC_MAXDEG 40                     /* > 2 * (2g+2) for g <= 8 */

typedef struct {
  orc_field F;                            /* F_q */
  int64_t q;
} orc_fq;

typedef struct {
  int deg;                                /* -1 for the zero polynomial */
  int c[ORC_MAXDEG + 1][ORC_MAXN];
} orc_poly;

static void fq_set(const orc_fq *K, int *a, int64_t code) {
  memset(a, 0, sizeof(int) * ORC_MAXN);
  orc_unpack(&K->F, code, a);
}

static void fq_sub(const orc_fq *K, const int *a, const int *b, int *out) {
  for (int i = 0; i < K->F.n; ++i) {
    int s = a[i] - b[i];
    out[i] = s < 0 ? s + K->F.p : s;
  }
}

static void fq_pow(const orc_fq *K, const int *a, int64_t e, int *out) {
  int base[ORC_MAXN], acc[ORC_MAXN], tmp[ORC_MAXN];
  memcpy(base, a, sizeof(base));
  memset(acc, 0, sizeof(acc));
  acc[0] = 1;
  while (e > 0) {
    if (e & 1) { orc_mul(&K->F, acc, base, tmp); memcpy(acc, tmp, sizeof(acc)); }
    orc_mul(&K->F, base, base, tmp);
    memcpy(base, tmp, sizeof(base));
    e >>= 1;
  }
  memcpy(out, acc, sizeof(acc));
}

static void fq_inv(const orc_fq *K, const int *a, int *out) { fq_pow(K, a, K->q - 2, out); }

static void poly_trim(const orc_fq *K, orc_poly *a) {
  while (a->deg >= 0 && orc_is_zero(&K->F, a->c[a->deg])) --a->deg;
}

static void poly_zero(orc_poly *a) { memset(a, 0, sizeof(*a)); a->deg = -1; }

/* a <- a mod b (b != 0) */
static void poly_mod(const orc_fq *K, orc_poly *a, const orc_poly *b) {
  int inv[ORC_MAXN], f[ORC_MAXN], t[ORC_MAXN];
  fq_inv(K, b->c[b->deg], inv);
  poly_trim(K, a);
  while (a->deg >= b->deg) {
    int s = a->deg - b->deg;
    orc_mul(&K->F, a->c[a->deg], inv, f);
    for (int i = 0; i <= b->deg; ++i) {
      orc_mul(&K->F, f, b->c[i], t);
      fq_sub(K, a->c[s + i], t, a->c[s + i]);
    }
    poly_trim(K, a);
  }
}

/* out <- a * b mod m */
static void poly_mulmod(const orc_fq *K, const orc_poly *a, const orc_poly *b, const orc_poly *m, orc_poly *out) {
  orc_poly r;
  poly_zero(&r);
  int t[ORC_MAXN];
  if (a->deg >= 0 && b->deg >= 0) {
    r.deg = a->deg + b->deg;
    for (int i = 0; i <= a->deg; ++i)
      for (int j = 0; j <= b->deg; ++j) {
        orc_mul(&K->F, a->c[i], b->c[j], t);
        orc_add(&K->F, r.c[i + j], t, r.c[i + j]);
      }
  }
  poly_mod(K, &r, m);
  *out = r;
}

static void poly_gcd(const orc_fq *K, const orc_poly *a0, const orc_poly *b0, orc_poly *out) {
  orc_poly a = *a0, b = *b0;
  poly_trim(K, &a);
  poly_trim(K, &b);
  while (b.deg >= 0) {
    poly_mod(K, &a, &b);
    orc_poly t = a; a = b; b = t;
  }
  *out = a;
}

/* a <- a / b exactly (b divides a) */
static void poly_divexact(const orc_fq *K, orc_poly *a, const orc_poly *b) {
  orc_poly qt;
  poly_zero(&qt);
  int inv[ORC_MAXN], f[ORC_MAXN], t[ORC_MAXN];
  fq_inv(K, b->c[b->deg], inv);
  poly_trim(K, a);
  qt.deg = a->deg - b->deg;
  while (a->deg >= b->deg && a->deg >= 0) {
    int s = a->deg - b->deg;
    orc_mul(&K->F, a->c[a->deg], inv, f);
    memcpy(qt.c[s], f, sizeof(f));
    for (int i = 0; i <= b->deg; ++i) {
      orc_mul(&K->F, f, b->c[i], t);
      fq_sub(K, a->c[s + i], t, a->c[s + i]);
    }
    poly_trim(K, a);
  }
  poly_trim(K, &qt);
  *a = qt;
}

/* multiplicities of the factor degrees of one row: out[j-1] = number of
 * irreducible factors of degree j, j = 1..2g+2 (plus the part 1 at infinity
 * for odd degree) */
static void orc_lambda_one(const orc_fq *K, int g, const int16_t *codes, uint8_t *out) {
  int ncoef = 2 * g + 3;
  memset(out, 0, (size_t)(ncoef - 1));
  orc_poly f;
  poly_zero(&f);
  for (int i = 0; i < ncoef; ++i) fq_set(K, f.c[i], codes[i]);
  f.deg = ncoef - 1;
  poly_trim(K, &f);
  int d = f.deg;
  if (d == 2 * g + 1) out[0] += 1;
  /* h = X mod f, then the distinct-degree loop */
  orc_poly rest = f, h, xq, x;
  poly_zero(&x);
  x.deg = 1;
  x.c[1][0] = 1;
  h = x;
  for (int k = 1; 2 * k <= rest.deg; ++k) {
    /* h <- h^q mod rest */
    orc_poly acc, base = h;
    poly_zero(&acc);
    acc.deg = 0;
    acc.c[0][0] = 1;
    for (int64_t e = K->q; e > 0; e >>= 1) {
      if (e & 1) poly_mulmod(K, &acc, &base, &rest, &acc);
      poly_mulmod(K, &base, &base, &rest, &base);
    }
    h = acc;
    /* gcd(rest, h - X) */
    xq = h;
    if (xq.deg < 1) xq.deg = 1;
    fq_sub(K, xq.c[1], x.c[1], xq.c[1]);
    poly_trim(K, &xq);
    orc_poly gk;
    if (xq.deg < 0) gk = rest;            /* h = X: every remaining factor has degree dividing k */
    else poly_gcd(K, &rest, &xq, &gk);
    if (gk.deg > 0) {
      out[k - 1] += (uint8_t)(gk.deg / k);
      poly_divexact(K, &rest, &gk);
      poly_mod(K, &h, &rest);
    }
  }
  if (rest.deg > 0) out[rest.deg - 1] += 1;
}

typedef struct {
  const orc_fq *K;
  int g;
  const int16_t *codes;
  uint8_t *out;
  int64_t start, count;
} orc_lam_job;

static void *orc_lam_worker(void *arg) {
  orc_lam_job *J = (orc_lam_job *)arg;
  int w = 2 * J->g + 2, nc = 2 * J->g + 3;
  for (int64_t i = J->start; i < J->start + J->count; ++i)
    orc_lambda_one(J->K, J->g, J->codes + i * nc, J->out + i * w);
  return NULL;
}

/* Factor-degree multiplicities for every row: out[i*(2g+2) + j-1].  Returns 0
 * or a negative code as orc_count_curves. */
int orc_factor_degrees(int q, int g, const int16_t *codes, int64_t ncurves, uint8_t *out, int threads) {
  int p, e;
  if (orc_factor(q, &p, &e) || q > 4096) return -1;
  if (g < 1 || 4 * g + 4 > ORC_MAXDEG) return -2;
  int rc = orc_check_rows(q, g, codes, ncurves);
  if (rc) return rc;
  orc_fq K;
  if (orc_primitive(p, e, 0, &K.F)) return -3;
  K.q = q;
  if (threads < 1) threads = 1;
  if (threads > 256) threads = 256;
  pthread_t th[256];
  orc_lam_job jobs[256];
  int64_t per = (ncurves + threads - 1) / threads;
  int used = 0;
  for (int t = 0; t < threads; ++t) {
    int64_t s = (int64_t)t * per;
    if (s >= ncurves) break;
    jobs[t].K = &K; jobs[t].g = g; jobs[t].codes = codes; jobs[t].out = out;
    jobs[t].start = s; jobs[t].count = (ncurves - s < per) ? ncurves - s : per;
    used++;
  }
  int started = 0;
  for (int t = 0; t < used; ++t) {
    if (pthread_create(&th[t], NULL, orc_lam_worker, &jobs[t])) break;
    started++;
  }
  for (int t = started; t < used; ++t) orc_lam_worker(&jobs[t]);
  for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
  return 0;
}
