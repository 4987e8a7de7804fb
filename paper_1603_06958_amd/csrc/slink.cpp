// Single-linkage consumer of LCS row tiles (paper, Methods, "Determination
// of the guide tree": single linkage computed incrementally with SLINK in
// O(k^2) time and O(k) memory, run while the similarities are produced).
//
// Similarity of a pair (Methods, "Pairwise similarities calculation"):
//   indel = |A| + |B| - 2 LCS,   similarity = LCS / indel^2,
// kept exactly as (LCS, indel); indel = 0 (identical sequences, including
// two empty ones) is +infinity.  Two similarities are compared by an integer
// key that orders them exactly (below).
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

// Similarities are ordered by a 64-bit key: the bits of the correctly rounded
// double LCS / indel^2, plus one (+infinity for indel 0); 0 is the "never
// joins" value below every similarity.  For lengths up to FAMSA_LCS_MAX_LEN
// two different ratios differ by a relative 2^-50 or more, so their doubles
// differ and keep the exact order; equal ratios give equal keys.  The exact
// rational is kept beside each key (LCS in the low and indel in the high 32
// bits) for the result.
inline uint64_t sim_key(int64_t L, int64_t d) {
  const double s = d == 0 ? __builtin_inf() : (double)L / ((double)d * (double)d);
  uint64_t bits;
  memcpy(&bits, &s, 8);
  return bits + 1;
}

inline uint64_t pack_ld(int64_t L, int64_t d) { return ((uint64_t)d << 32) | (uint64_t)L; }

}  // namespace

struct famsa_slink_s {
  uint32_t k = 0;
  std::vector<uint32_t> len;   // by original index
  std::vector<uint32_t> pi;    // by insertion order p (point p is original index k-1-p)
  std::vector<uint64_t> lk, mk;  // keys of lambda and M
  std::vector<uint64_t> lv, mv;  // their (LCS, indel) values
  uint32_t n = 0;              // points inserted
  void insert_row(const int32_t* row);  // row: LCS(i, j) for j = i+1..k-1, i = k-1-n
};

void famsa_slink_s::insert_row(const int32_t* row) {
  const uint32_t i_new = k - 1 - n;
  const int64_t li = len[i_new];
  uint64_t* __restrict__ Mk = mk.data();
  uint64_t* __restrict__ Mv = mv.data();
  uint64_t* __restrict__ Lk = lk.data();
  uint64_t* __restrict__ Lv = lv.data();
  uint32_t* __restrict__ P = pi.data();
  // similarities to the inserted points p = 0..n-1 (original j = k-1-p)
  for (uint32_t p = 0; p < n; ++p) {
    const uint32_t j = k - 1 - p;
    const int64_t L = row[j - i_new - 1];
    const int64_t d = li + (int64_t)len[j] - 2 * L;
    Mk[p] = sim_key(L, d);
    Mv[p] = pack_ld(L, d);
  }
  P[n] = n;
  Lk[n] = 0;
  Lv[n] = 0;
  // with similarities "lambda(p) >= M(p)" of the distance form reads "lambda(p)
  // is no more similar than M(p)"; the updates are written as selects, since
  // which way each point goes is data dependent
  for (uint32_t p = 0; p < n; ++p) {
    const uint32_t q = P[p];  // q > p: a later point
    const bool c = Mk[p] >= Lk[p];
    const uint64_t ck = c ? Lk[p] : Mk[p], cv = c ? Lv[p] : Mv[p];
    const bool up = Mk[q] < ck;
    Mk[q] = up ? ck : Mk[q];
    Mv[q] = up ? cv : Mv[q];
    Lk[p] = c ? Mk[p] : Lk[p];
    Lv[p] = c ? Mv[p] : Lv[p];
    P[p] = c ? n : q;
  }
  for (uint32_t p = 0; p < n; ++p) P[p] = Lk[P[p]] >= Lk[p] ? n : P[p];
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
    s->lk.assign(k, 0);
    s->mk.assign(k, 0);
    s->lv.assign(k, 0);
    s->mv.assign(k, 0);
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
    const int64_t L = (int64_t)(s->lv[p] & 0xFFFFFFFFu), d = (int64_t)(s->lv[p] >> 32);
    if (num) num[i] = root ? -1 : L;
    if (den) den[i] = root ? 0 : d * d;
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
