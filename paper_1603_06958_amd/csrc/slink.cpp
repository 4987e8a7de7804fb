// Single-linkage consumer of LCS row tiles (paper, Methods, "Determination
// of the guide tree": single linkage computed incrementally with SLINK in
// O(k^2) time and O(k) memory, run while the similarities are produced).
//
// Similarity of a pair (Methods, "Pairwise similarities calculation"):
//   indel = |A| + |B| - 2 LCS,   similarity = LCS / indel^2,
// kept as the exact rational (LCS, indel^2); indel = 0 (identical sequences,
// including two empty ones) is +infinity.  Two similarities are compared by
// cross-multiplying in int64, exact for lengths up to FAMSA_LCS_MAX_LEN
// (numerators <= 65535, denominators <= 131070^2).
//
// SLINK (Sibson 1973) inserts points one by one and keeps the pointer
// representation: for each inserted point, pi = the later-inserted point it
// first joins and lambda = the similarity of that join.  With similarities
// the roles of <= and min in the distance form are mirrored: "lambda(i) >=
// M(i)" becomes "lambda(i) is no more similar than M(i)" and min becomes max.
// Points are inserted from index k-1 down to 0, so inserting point i needs
// LCS(i, j) for all j > i: row i of the upper triangle.
#include <stdint.h>
#include <string.h>

#include <new>
#include <vector>

#include "runtime.h"

namespace {

struct Sim {
  int64_t num, den;  // den == 0: +infinity; the "never joins" value is (-1, 1)
};

inline bool sim_less(const Sim& a, const Sim& b) {  // a strictly less similar than b
  if (a.den == 0) return false;
  if (b.den == 0) return true;
  return a.num * b.den < b.num * a.den;
}

inline Sim sim_of(int64_t L, int64_t la, int64_t lb) {
  const int64_t d = la + lb - 2 * L;
  return Sim{L, d * d};
}

}  // namespace

struct famsa_slink_s {
  uint32_t k = 0;
  std::vector<uint32_t> len;   // by original index
  std::vector<uint32_t> pi;    // by insertion order p (point p is original index k-1-p)
  std::vector<Sim> lambda, M;
  uint32_t n = 0;              // points inserted
  void insert_row(const int32_t* row);  // row: LCS(i, j) for j = i+1..k-1, i = k-1-n
};

void famsa_slink_s::insert_row(const int32_t* row) {
  const uint32_t i_new = k - 1 - n;
  // distances to the inserted points p = 0..n-1 (original j = k-1-p)
  for (uint32_t p = 0; p < n; ++p) {
    const uint32_t j = k - 1 - p;
    M[p] = sim_of(row[j - i_new - 1], len[i_new], len[j]);
  }
  pi[n] = n;
  lambda[n] = Sim{-1, 1};
  for (uint32_t p = 0; p < n; ++p) {
    const uint32_t q = pi[p];
    if (!sim_less(M[p], lambda[p])) {  // lambda(p) no more similar than M(p)
      if (sim_less(M[q], lambda[p])) M[q] = lambda[p];
      lambda[p] = M[p];
      pi[p] = n;
    } else {
      if (sim_less(M[q], M[p])) M[q] = M[p];
    }
  }
  for (uint32_t p = 0; p < n; ++p)
    if (!sim_less(lambda[pi[p]], lambda[p])) pi[p] = n;
  ++n;
}

extern "C" {

int famsa_slink_create(const uint32_t* lengths, uint32_t k, famsa_slink_t** out) {
  famsa::clear_error();
  if (!out) return famsa::set_error(FAMSA_LCS_EINVAL, "out is NULL");
  *out = nullptr;
  if (k && !lengths) return famsa::set_error(FAMSA_LCS_EINVAL, "lengths is NULL");
  for (uint32_t i = 0; i < k; ++i)
    if (lengths[i] > FAMSA_LCS_MAX_LEN)
      return famsa::set_error(FAMSA_LCS_EINVAL, "length %u of sequence %u exceeds %u", lengths[i], i,
                              FAMSA_LCS_MAX_LEN);
  famsa_slink_s* s = new (std::nothrow) famsa_slink_s();
  if (!s) return famsa::set_error(FAMSA_LCS_ENOMEM, "out of host memory");
  try {
    s->k = k;
    s->len.assign(lengths, lengths + k);
    s->pi.assign(k, 0);
    s->lambda.assign(k, Sim{-1, 1});
    s->M.assign(k, Sim{-1, 1});
  } catch (...) {
    delete s;
    return famsa::set_error(FAMSA_LCS_ENOMEM, "out of host memory");
  }
  *out = s;
  return 0;
}

int famsa_slink_consume(void* user, const famsa_lcs_tile* t) {
  famsa_slink_s* s = static_cast<famsa_slink_s*>(user);
  if (!s || !t || t->k != s->k || t->row_end > s->k || t->row_begin > t->row_end) return 1;
  // rows must arrive from the last one down: this tile must end where the
  // previous one began
  if (t->row_end != s->k - s->n) return 1;
  if (t->count && !t->lcs) return 1;
  if (t->values != FAMSA_LCS_VALUES_LCS) return 1;  // SLINK needs the LCS values
  const uint64_t k = s->k;
  for (uint32_t i = t->row_end; i-- > t->row_begin;) {
    const uint64_t off = famsa::tri_rows(k, t->row_begin, i);
    s->insert_row(t->lcs + off);
  }
  return 0;
}

int famsa_slink_result(const famsa_slink_t* s, uint32_t* pi, int64_t* num, int64_t* den) {
  famsa::clear_error();
  if (!s) return famsa::set_error(FAMSA_LCS_EINVAL, "slink is NULL");
  if (s->n != s->k) return famsa::set_error(FAMSA_LCS_EINVAL, "only %u of %u rows inserted", s->n, s->k);
  for (uint32_t p = 0; p < s->k; ++p) {
    const uint32_t i = s->k - 1 - p;
    if (pi) pi[i] = s->k - 1 - s->pi[p];
    const bool root = s->pi[p] == p;
    if (num) num[i] = root ? -1 : s->lambda[p].num;
    if (den) den[i] = root ? 0 : s->lambda[p].den;
  }
  return 0;
}

int famsa_slink_guide_tree(const famsa_slink_t* s, uint32_t* left, uint32_t* right, int64_t* num, int64_t* den,
                           uint32_t* nmerges) {
  famsa::clear_error();
  if (!s || !nmerges) return famsa::set_error(FAMSA_LCS_EINVAL, "NULL argument");
  const uint32_t k = s->k;
  std::vector<uint32_t> pi(k), eu, ev;
  std::vector<int64_t> ln(k), ld(k), en, ed;
  int rc = famsa_slink_result(s, pi.data(), ln.data(), ld.data());
  if (rc) return rc;
  // every point but the root joins the cluster of pi(i) at height lambda(i)
  for (uint32_t i = 0; i < k; ++i) {
    if (pi[i] == i) continue;
    eu.push_back(i);
    ev.push_back(pi[i]);
    en.push_back(ln[i]);
    ed.push_back(ld[i]);
  }
  return famsa::guide_tree(k, eu.data(), ev.data(), en.data(), ed.data(), (uint32_t)eu.size(), left, right, num, den,
                           nmerges);
}

uint32_t famsa_slink_rows_done(const famsa_slink_t* s) { return s ? s->n : 0; }

void famsa_slink_destroy(famsa_slink_t* s) { delete s; }

}  // extern "C"
