// Host-side construction of finite-field tables in Zech-logarithm form.
//
// F_Q = F_p[t]/(P), Q = p^n, with P the lexicographically first primitive
// monic polynomial of degree n over F_p (coefficients a_0..a_{n-1} ranked by
// the integer sum_i a_i p^i), so gamma = t generates F_Q^x.  Elements are
// encoded by their discrete logarithm to gamma with a zero sentinel
// (encoding (3.1) of Sec. 3.1); addition goes through the Zech logarithm
// Z(k) = log(1 + gamma^k) (eq. 2.1 and the table (3.2) of Sec. 3.2).
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace hwc {

struct Field {
  uint32_t p = 0, e = 0, k = 0;   // F_Q with Q = (p^e)^k; F_q, q = p^e, is embedded
  uint32_t n = 0;                 // e*k, degree over F_p
  uint64_t q = 0, Q = 0, M = 0;   // M = Q - 1 (order of gamma)
  std::vector<uint32_t> modulus;  // P: n+1 coefficients, constant term first, modulus[n] = 1
  std::vector<uint32_t> exp;      // exp[L] = packed gamma^L (sum_i b_i p^i), L in [0, M)
  std::vector<uint32_t> log;      // log[packed v] for v != 0; log[0] = M (sentinel)
  std::vector<uint32_t> zech;     // zech[L] = log(1 + gamma^L), or M when 1 + gamma^L = 0
  std::vector<uint32_t> emb;      // emb[c] = log of the F_q code c in F_Q; emb[0] = M
  uint32_t root_log = 0;          // log of the root of P_q used for the embedding
  std::vector<uint32_t> qmodulus; // P_q (degree e), constant term first
  // Frobenius x -> x^q acts on logs as L -> qL mod M.  Orbit representatives
  // (least element of each orbit) of the elements whose smallest field of
  // definition containing F_q is F_Q itself, i.e. orbits of size exactly k.
  std::vector<uint32_t> prim_reps;
};

// Factor q as p^e with p an odd prime; false otherwise.
bool factor_odd_prime_power(uint64_t q, uint32_t* p, uint32_t* e);

// Lex-first primitive monic polynomial of degree n over F_p.  Also returns
// the power table of t when exp_out != nullptr.  False if none (n too big).
bool lex_first_primitive(uint32_t p, uint32_t n, std::vector<uint32_t>* poly,
                         std::vector<uint32_t>* exp_out);

// Groups the primitive Frobenius orbits into cosets of mu_m (m | q - 1, so the
// m-th roots of unity lie in F_q and multiplying by them keeps an element's
// field of definition).  For a representative x of each group whose points
// x, wx, .., w^(m-1)x (w = gamma^(M/m)) lie in m distinct Frobenius orbits,
// the representative's log goes to *tuples; the orbits of a group with fewer
// distinct orbits (some w^s x, 0 < s < m, in the orbit of x) go to *singles.
// Every primitive orbit is covered exactly once:
// m * tuples.size() + singles.size() == prim_reps.size().
void split_orbits(const Field& F, uint32_t m, std::vector<uint32_t>* tuples, std::vector<uint32_t>* singles);

// Build every table of F_{p^(e k)} with F_{p^e} embedded.  Returns an empty
// string on success, else a message.
std::string build_field(uint32_t p, uint32_t e, uint32_t k, Field* out);

}  // namespace hwc
