/*
 * curvegen.c -- seeded synthetic curve sets y^2 = f(x) over F_q, q odd.
 *
 * This module only produces inputs.  It holds none of the point-counting
 * arithmetic; both the device path and the CPU reference take their curve
 * sets from here.  Its only field arithmetic is what the input filter
 * needs: f is kept when it has degree 2g+1 or 2g+2 and is square-free
 * (gcd(f, f') = 1 over F_q), which is the curve family Pg_g of Sec. 1.1.
 *
 * Coefficient codes.  A coefficient is an integer code c in [0, q).  For
 * q = p^e with e > 1 the code c = sum_i d_i p^i (0 <= d_i < p) stands for
 * the element sum_i d_i t^i of F_p[t]/(P_q), where P_q is the
 * lexicographically first primitive monic polynomial of degree e over F_p
 * (polynomials t^e + a_{e-1} t^{e-1} + ... + a_0 ordered by the integer
 * sum_i a_i p^i).  Rows are a_0 .. a_{2g+2} (constant term first).
 *
 * Random sets.  Curve i of a stream (seed, q, g) draws its coefficients
 * from a SplitMix64 sequence whose start is a hash of (seed, q, g, i), so
 * every curve is reproducible on its own and the set can be built in
 * parallel.  Bounded draws use Lemire's multiply-shift with rejection.
 * A draw of 2g+3 codes is repeated until it passes the filter.
 *
 * Full enumeration.  Coefficient vectors are visited in increasing order
 * of sum_i a_i q^i and kept when they pass the same filter.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

#define CG_MAXQ 4096
#define CG_MAXDEG 32

typedef struct {
  int q, p, e;
  int *log_;   /* log_[c] for c != 0, code -> discrete log */
  int *exp_;   /* exp_[k] code of generator^k, k in [0, q-1) */
  int *add_;   /* add_[a*q+b] code of a+b (digitwise mod p) */
} cg_field;

static uint64_t cg_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

typedef struct { uint64_t s; uint32_t spare; int have_spare; } cg_rng;

static uint32_t cg_next32(cg_rng *r) {
  if (r->have_spare) { r->have_spare = 0; return r->spare; }
  r->s += 0x9e3779b97f4a7c15ULL;
  uint64_t v = cg_mix(r->s);
  r->spare = (uint32_t)(v >> 32);
  r->have_spare = 1;
  return (uint32_t)v;
}

/* Lemire: uniform integer in [0, n) */
static uint32_t cg_bounded(cg_rng *r, uint32_t n) {
  uint32_t x = cg_next32(r);
  uint64_t m = (uint64_t)x * n;
  uint32_t l = (uint32_t)m;
  if (l < n) {
    uint32_t t = (uint32_t)(-n) % n;
    while (l < t) {
      x = cg_next32(r);
      m = (uint64_t)x * n;
      l = (uint32_t)m;
    }
  }
  return (uint32_t)(m >> 32);
}

static uint64_t cg_stream_key(uint64_t seed, int q, int g) {
  uint64_t k = cg_mix(seed + 0x9e3779b97f4a7c15ULL);
  k = cg_mix(k ^ (uint64_t)(uint32_t)q);
  k = cg_mix(k ^ ((uint64_t)(uint32_t)g << 20));
  return k;
}

/* ---- F_q by log/exp tables built from the lex-first primitive P_q ---- */

static int cg_factor(int q, int *p, int *e) {
  if (q < 3 || (q % 2) == 0) return -1;
  int f = 0;
  for (int d = 3; d * d <= q; d += 2)
    if (q % d == 0) { f = d; break; }
  if (!f) f = q;
  int n = 0, r = q;
  while (r % f == 0) { r /= f; ++n; }
  if (r != 1) return -1;
  *p = f; *e = n;
  return 0;
}

/* multiply packed element v (digits base p, length e) by t modulo P (monic, coeffs a[0..e-1]) */
static int cg_mul_t(int v, int p, int e, const int *a) {
  int d[CG_MAXDEG];
  for (int i = 0; i < e; ++i) { d[i] = v % p; v /= p; }
  int top = d[e - 1];
  for (int i = e - 1; i > 0; --i) d[i] = d[i - 1];
  d[0] = 0;
  for (int i = 0; i < e; ++i) d[i] = ((d[i] - top * a[i]) % p + p) % p;
  int out = 0;
  for (int i = e - 1; i >= 0; --i) out = out * p + d[i];
  return out;
}

static int cg_build_field(cg_field *F, int q) {
  memset(F, 0, sizeof(*F));
  if (q > CG_MAXQ) return -1;
  if (cg_factor(q, &F->p, &F->e)) return -1;
  F->q = q;
  int p = F->p, e = F->e;
  F->log_ = (int *)malloc(sizeof(int) * q);
  F->exp_ = (int *)malloc(sizeof(int) * q);
  F->add_ = (int *)malloc(sizeof(int) * q * q);
  if (!F->log_ || !F->exp_ || !F->add_) return -1;
  /* addition table on codes */
  for (int a = 0; a < q; ++a)
    for (int b = 0; b < q; ++b) {
      int x = a, y = b, out = 0, pw = 1;
      for (int i = 0; i < e; ++i) { out += ((x % p + y % p) % p) * pw; x /= p; y /= p; pw *= p; }
      F->add_[a * q + b] = out;
    }
  /* search the lex-first primitive monic polynomial of degree e */
  int a[CG_MAXDEG];
  for (int v = 0; v < q; ++v) {
    int w = v;
    for (int i = 0; i < e; ++i) { a[i] = w % p; w /= p; }
    if (a[0] == 0) continue;
    /* element t: for e == 1 the residue of t is -a0 */
    int t = (e == 1) ? ((p - a[0]) % p) : p; /* packed t = 0 + 1*p^1 */
    int cur = 1, ok = 1;
    for (int k = 0; k < q - 1; ++k) {
      F->exp_[k] = cur;
      if (k > 0 && cur == 1) { ok = 0; break; }
      if (e == 1) cur = (int)(((long)cur * t) % p);
      else cur = cg_mul_t(cur, p, e, a);
    }
    if (ok && cur == 1) {
      for (int k = 0; k < q - 1; ++k) F->log_[F->exp_[k]] = k;
      F->log_[0] = -1;
      return 0;
    }
  }
  return -1;
}

static void cg_free_field(cg_field *F) {
  free(F->log_); free(F->exp_); free(F->add_);
  memset(F, 0, sizeof(*F));
}

static inline int cg_mul(const cg_field *F, int a, int b) {
  if (a == 0 || b == 0) return 0;
  int k = F->log_[a] + F->log_[b];
  if (k >= F->q - 1) k -= F->q - 1;
  return F->exp_[k];
}
static inline int cg_add(const cg_field *F, int a, int b) { return F->add_[a * F->q + b]; }
static inline int cg_neg(const cg_field *F, int a) {
  /* -a digitwise */
  int p = F->p, out = 0, pw = 1;
  for (int i = 0; i < F->e; ++i) { int d = a % p; out += ((p - d) % p) * pw; a /= p; pw *= p; }
  return out;
}
static inline int cg_inv(const cg_field *F, int a) {
  int k = F->log_[a];
  return F->exp_[k == 0 ? 0 : (F->q - 1 - k)];
}

/* degree of polynomial with coeffs c[0..n-1] (codes), -1 for zero */
static int cg_deg(const int *c, int n) {
  for (int i = n - 1; i >= 0; --i) if (c[i]) return i;
  return -1;
}

/* r = a mod b over F_q (in place on a copy); returns deg of remainder */
static int cg_polyrem(const cg_field *F, int *a, int da, const int *b, int db) {
  int ilc = cg_inv(F, b[db]);
  while (da >= db && da >= 0) {
    int coef = cg_mul(F, a[da], ilc);
    int nc = cg_neg(F, coef);
    for (int i = 0; i <= db; ++i)
      a[da - db + i] = cg_add(F, a[da - db + i], cg_mul(F, nc, b[i]));
    /* a[da] is now 0 */
    da = cg_deg(a, da);
  }
  return da;
}

/* 1 if f (codes c[0..n-1]) is square-free over F_q */
static int cg_squarefree(const cg_field *F, const int *c, int n) {
  int d = cg_deg(c, n);
  if (d < 1) return 0;
  int A[CG_MAXDEG], B[CG_MAXDEG], T[CG_MAXDEG];
  memcpy(A, c, sizeof(int) * (d + 1));
  int dd = -1;
  for (int i = 1; i <= d; ++i) {
    /* i * c_i : add c_i to itself i times (i mod p times) */
    int v = 0, m = i % F->p;
    for (int j = 0; j < m; ++j) v = cg_add(F, v, c[i]);
    B[i - 1] = v;
  }
  dd = cg_deg(B, d);
  if (dd < 0) return 0; /* f' = 0: f is a p-th power */
  int da = d, db = dd;
  while (db >= 0) {
    da = cg_polyrem(F, A, da, B, db);
    memcpy(T, A, sizeof(int) * (da + 1 > 0 ? da + 1 : 1));
    /* swap: A <- B, B <- remainder */
    memcpy(A, B, sizeof(int) * (db + 1));
    int tda = db;
    if (da >= 0) memcpy(B, T, sizeof(int) * (da + 1));
    db = da;
    da = tda;
  }
  return da == 0; /* gcd is a nonzero constant */
}

/* filter: degree 2g+1 or 2g+2 and square-free */
static int cg_accept(const cg_field *F, const int *c, int g) {
  int n = 2 * g + 3;
  if (c[n - 1] == 0 && c[n - 2] == 0) return 0;
  return cg_squarefree(F, c, n);
}

/* ---------------------------- public API ------------------------------ */

typedef struct {
  const cg_field *F;
  int g, q, width;   /* width: 1 (int8) or 2 (int16) */
  uint64_t key;
  uint64_t id0;      /* absolute curve id of row 0 of out */
  uint64_t row0, rows;
  void *out;
} cg_job;

static void *cg_sample_worker(void *arg) {
  cg_job *J = (cg_job *)arg;
  int n = 2 * J->g + 3;
  int c[CG_MAXDEG];
  for (uint64_t row = J->row0; row < J->row0 + J->rows; ++row) {
    cg_rng r;
    r.s = cg_mix(J->key ^ cg_mix(J->id0 + row + 1));
    r.have_spare = 0;
    for (;;) {
      for (int j = 0; j < n; ++j) c[j] = (int)cg_bounded(&r, (uint32_t)J->q);
      if (cg_accept(J->F, c, J->g)) break;
    }
    for (int j = 0; j < n; ++j) {
      if (J->width == 1) ((int8_t *)J->out)[row * n + j] = (int8_t)c[j];
      else ((int16_t *)J->out)[row * n + j] = (int16_t)c[j];
    }
  }
  return NULL;
}

/* Fill out[count][2g+3] with curves start .. start+count-1 of stream (seed, q, g).
 * width = 1 writes int8 codes (needs q <= 127), width = 2 writes int16.
 * Returns 0, or -1 for bad arguments (q not an odd prime power <= 4096, g < 1). */
int cg_sample(uint64_t seed, int q, int g, uint64_t start, uint64_t count, int width, void *out, int threads) {
  if (g < 1 || 2 * g + 3 > CG_MAXDEG || (width != 1 && width != 2) || (width == 1 && q > 127)) return -1;
  cg_field F;
  if (cg_build_field(&F, q)) { cg_free_field(&F); return -1; }
  if (threads < 1) threads = 1;
  if (threads > 256) threads = 256;
  uint64_t key = cg_stream_key(seed, q, g);
  pthread_t th[256];
  cg_job jobs[256];
  uint64_t per = (count + (uint64_t)threads - 1) / (uint64_t)threads;
  int used = 0;
  for (int t = 0; t < threads; ++t) {
    uint64_t s = (uint64_t)t * per;
    if (s >= count) break;
    jobs[t].F = &F; jobs[t].g = g; jobs[t].q = q; jobs[t].width = width;
    jobs[t].key = key; jobs[t].id0 = start; jobs[t].out = out;
    jobs[t].row0 = s; jobs[t].rows = (count - s < per) ? count - s : per;
    used++;
  }
  int started = 0;
  for (int t = 0; t < used; ++t) {
    if (pthread_create(&th[t], NULL, cg_sample_worker, &jobs[t])) break;
    started++;
  }
  for (int t = started; t < used; ++t) cg_sample_worker(&jobs[t]);
  for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
  cg_free_field(&F);
  return 0;
}

/* Every f of degree 2g+1 or 2g+2 over F_q that is square-free, in increasing
 * order of sum_i a_i q^i.  Writes at most max_out rows when out != NULL and
 * returns the total number of such f (or -1 for bad arguments). */
int64_t cg_enumerate(int q, int g, int width, void *out, int64_t max_out) {
  if (g < 1 || 2 * g + 3 > CG_MAXDEG || (width != 1 && width != 2) || (width == 1 && q > 127)) return -1;
  cg_field F;
  if (cg_build_field(&F, q)) { cg_free_field(&F); return -1; }
  int n = 2 * g + 3;
  double total = 1.0;
  for (int i = 0; i < n; ++i) total *= q;
  if (total > 4.0e9) { cg_free_field(&F); return -1; }
  int c[CG_MAXDEG];
  memset(c, 0, sizeof(c));
  int64_t found = 0;
  for (;;) {
    if (cg_accept(&F, c, g)) {
      if (out && found < max_out)
        for (int j = 0; j < n; ++j) {
          if (width == 1) ((int8_t *)out)[found * n + j] = (int8_t)c[j];
          else ((int16_t *)out)[found * n + j] = (int16_t)c[j];
        }
      found++;
    }
    int j = 0;
    while (j < n && ++c[j] == q) { c[j] = 0; ++j; }
    if (j == n) break;
  }
  cg_free_field(&F);
  return found;
}

/* Square-free test of one coefficient row (codes, constant term first). */
int cg_is_squarefree(int q, const int *codes, int ncoef) {
  if (ncoef < 1 || ncoef > CG_MAXDEG) return -1;
  cg_field F;
  if (cg_build_field(&F, q)) { cg_free_field(&F); return -1; }
  int r = cg_squarefree(&F, codes, ncoef);
  cg_free_field(&F);
  return r;
}
