// Host construction of the Zech tables (see field.h).
#include "field.h"

#include <algorithm>
#include <numeric>

namespace hwc {

bool factor_odd_prime_power(uint64_t q, uint32_t* p, uint32_t* e) {
  if (q < 3 || (q & 1) == 0) return false;
  uint64_t f = 0;
  for (uint64_t d = 3; d * d <= q; d += 2)
    if (q % d == 0) { f = d; break; }
  if (!f) f = q;
  uint32_t cnt = 0;
  while (q % f == 0) { q /= f; ++cnt; }
  if (q != 1) return false;
  *p = (uint32_t)f;
  *e = cnt;
  return true;
}

namespace {

// Packed element v = sum_i d_i p^i; digits in d[0..n).
struct Packer {
  uint32_t p, n;
  std::vector<uint64_t> pw;  // p^i
  Packer(uint32_t p_, uint32_t n_) : p(p_), n(n_), pw(n_ + 1, 1) {
    for (uint32_t i = 1; i <= n; ++i) pw[i] = pw[i - 1] * p;
  }
  void unpack(uint64_t v, uint32_t* d) const {
    for (uint32_t i = 0; i < n; ++i) { d[i] = (uint32_t)(v % p); v /= p; }
  }
  uint64_t pack(const uint32_t* d) const {
    uint64_t v = 0;
    for (uint32_t i = n; i-- > 0;) v = v * p + d[i];
    return v;
  }
};

// v * t mod P, on packed values
inline uint64_t times_t(const Packer& P, const std::vector<uint32_t>& poly, uint64_t v) {
  const uint32_t n = P.n, p = P.p;
  if (n == 1) return (v * ((p - poly[0]) % p)) % p;
  uint64_t top = v / P.pw[n - 1];              // coefficient of t^{n-1}
  uint64_t shifted = (v % P.pw[n - 1]) * p;    // other coefficients move up
  if (top == 0) return shifted;
  // subtract top * (a_0 + a_1 t + ... + a_{n-1} t^{n-1}) digitwise
  uint32_t d[64];
  P.unpack(shifted, d);
  for (uint32_t i = 0; i < n; ++i) d[i] = (uint32_t)((d[i] + p - (top * poly[i]) % p) % p);
  return P.pack(d);
}

}  // namespace

bool lex_first_primitive(uint32_t p, uint32_t n, std::vector<uint32_t>* poly,
                         std::vector<uint32_t>* exp_out) {
  if (n < 1 || n > 40) return false;
  Packer P(p, n);
  const uint64_t Q = P.pw[n], M = Q - 1;
  if (Q > (1ull << 31)) return false;
  std::vector<uint32_t> a(n + 1, 0);
  std::vector<uint32_t> ex;
  if (exp_out) ex.resize(M);
  for (uint64_t cand = 0; cand < Q; ++cand) {
    uint64_t w = cand;
    for (uint32_t i = 0; i < n; ++i) { a[i] = (uint32_t)(w % p); w /= p; }
    a[n] = 1;
    if (a[0] == 0) continue;                    // t divides P
    // walk the powers of t; t is primitive iff the walk first returns to 1 at M
    uint64_t cur = 1;
    bool ok = true;
    for (uint64_t L = 0; L < M; ++L) {
      if (L > 0 && cur == 1) { ok = false; break; }
      if (exp_out) ex[L] = (uint32_t)cur;
      cur = times_t(P, a, cur);
    }
    if (ok && cur == 1) {
      *poly = a;
      if (exp_out) exp_out->swap(ex);
      return true;
    }
  }
  return false;
}

std::string build_field(uint32_t p, uint32_t e, uint32_t k, Field* F) {
  if (e < 1 || k < 1) return "e and k must be positive";
  uint32_t pp, ee;
  if (!factor_odd_prime_power(p, &pp, &ee) || ee != 1) return "p must be an odd prime";
  const uint32_t n = e * k;
  double Qd = 1;
  for (uint32_t i = 0; i < n; ++i) Qd *= p;
  if (Qd > 16777216.0) return "field too large";
  F->p = p; F->e = e; F->k = k; F->n = n;
  Packer P(p, n);
  F->Q = P.pw[n];
  F->M = F->Q - 1;
  F->q = 1;
  for (uint32_t i = 0; i < e; ++i) F->q *= p;
  const uint64_t Q = F->Q, M = F->M;
  if (!lex_first_primitive(p, n, &F->modulus, &F->exp)) return "no primitive polynomial";
  // log table with the zero sentinel M (encoding (3.1))
  F->log.assign(Q, (uint32_t)M);
  for (uint64_t L = 0; L < M; ++L) F->log[F->exp[L]] = (uint32_t)L;
  // Zech table: 1 + gamma^L adds one to the constant digit
  F->zech.resize(M);
  for (uint64_t L = 0; L < M; ++L) {
    uint64_t v = F->exp[L];
    uint64_t d0 = v % p;
    uint64_t w = v - d0 + (d0 + 1) % p;
    F->zech[L] = F->log[w];                     // w = 0 gives the sentinel M
  }
  // F_q inside F_Q: a root of P_q (lex-first primitive of degree e over F_p).
  // The roots lie in the subgroup of order q-1, i.e. logs divisible by
  // r = M/(q-1); the root with the smallest such log is used.  Any root gives
  // the same point counts (roots differ by a Frobenius automorphism).
  if (!lex_first_primitive(p, e, &F->qmodulus, nullptr)) return "no primitive polynomial for F_q";
  const uint64_t r = M / (F->q - 1);
  // evaluate P_q at gamma^L with Zech arithmetic on logs
  auto add_logs = [&](uint64_t a, uint64_t b) -> uint64_t {  // log(gamma^a + gamma^b), M = zero
    if (a == M) return b;
    if (b == M) return a;
    uint64_t d = (b + M - a) % M;
    uint64_t z = F->zech[d];
    return z == M ? M : (a + z) % M;
  };
  auto const_log = [&](uint32_t c) -> uint64_t {  // log of the F_p constant c
    return F->log[c % p];
  };
  bool found = false;
  for (uint64_t j = 0; j < F->q - 1 && !found; ++j) {
    uint64_t L = j * r;
    // Horner over P_q with leading 1
    uint64_t acc = 0;  // log 1
    for (uint32_t i = e; i-- > 0;) {
      acc = (acc == M) ? M : (acc + L) % M;
      acc = add_logs(acc, const_log(F->qmodulus[i]));
    }
    if (acc == M) { F->root_log = (uint32_t)L; found = true; }
  }
  if (!found) return "no root of P_q in F_Q";
  // emb[c]: code c = sum_i d_i p^i  ->  log(sum_i d_i z^i)
  F->emb.resize(F->q);
  for (uint64_t c = 0; c < F->q; ++c) {
    uint64_t acc = M;  // zero
    uint64_t w = c;
    for (uint32_t i = 0; i < e; ++i) {
      uint32_t d = (uint32_t)(w % p);
      w /= p;
      if (d == 0) continue;
      uint64_t term = (const_log(d) + (uint64_t)i * F->root_log) % M;
      acc = add_logs(acc, term);
    }
    F->emb[c] = (uint32_t)acc;
  }
  // primitive Frobenius orbits: L -> qL mod M with orbit size exactly k
  F->prim_reps.clear();
  std::vector<uint8_t> seen(M, 0);
  for (uint64_t L = 0; L < M; ++L) {
    if (seen[L]) continue;
    uint64_t x = L;
    uint32_t size = 0;
    do {
      seen[x] = 1;
      x = (x * F->q) % M;
      ++size;
    } while (x != L);
    if (size == k) F->prim_reps.push_back((uint32_t)L);
  }
  return "";
}

void split_orbits(const Field& F, uint32_t m, std::vector<uint32_t>* tuples, std::vector<uint32_t>* singles) {
  tuples->clear();
  singles->clear();
  const uint64_t M = F.M;
  // least element of the Frobenius orbit of every primitive element
  std::vector<uint32_t> rep(M, UINT32_MAX);
  for (uint32_t r : F.prim_reps) {
    uint64_t x = r;
    do {
      rep[x] = r;
      x = (x * F.q) % M;
    } while (x != r);
  }
  std::vector<uint8_t> done(M, 0);
  const uint64_t step = M / m;
  // x -> w x permutes the primitive orbits (w lies in F_q, so it commutes
  // with Frobenius); the orbits met by x, wx, .., w^(m-1) x share one
  // stabiliser.  Trivial stabiliser: m distinct orbits, one tuple.  Else every
  // orbit met is swept on its own.
  std::vector<uint32_t> met(m);
  for (uint32_t r : F.prim_reps) {
    if (done[r]) continue;
    bool distinct = true;
    for (uint32_t s = 0; s < m; ++s) {
      met[s] = rep[(r + s * step) % M];
      for (uint32_t t = 0; t < s; ++t) distinct &= met[t] != met[s];
    }
    if (distinct) {
      tuples->push_back(r);
    } else {
      for (uint32_t s = 0; s < m; ++s)
        if (!done[met[s]]) {
          singles->push_back(met[s]);
          done[met[s]] = 1;
        }
    }
    for (uint32_t s = 0; s < m; ++s) done[met[s]] = 1;
  }
}

}  // namespace hwc
