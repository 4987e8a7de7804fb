/*
 * CPU oracle for the all-pairs LCS similarity stage -- TEST INFRASTRUCTURE.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load this file's library.  It shares no source with the GPU path.
 *
 * What it computes (FAMSA paper, Methods, "Pairwise similarities
 * calculation"): the length of a longest common subsequence of two sequences,
 * i.e. the largest number of columns in which the two sequences can be
 * aligned with identical symbols.  The paper refers this quantity to the
 * textbook dynamic-programming rule (its citation of Gusfield, 1997):
 *
 *   L[i][0] = L[0][j] = 0
 *   L[i][j] = L[i-1][j-1] + 1                 if a[i] == b[j]
 *           = max(L[i-1][j], L[i][j-1])       otherwise
 *   LCS_len(A, B) = L[|A|][|B|]
 *
 * computed here row by row with two int32 rows, single threaded, symbols
 * compared as plain byte codes.  Nothing is blocked, vectorised or reordered.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* LCS length of a[0..m) and b[0..n) by the DP rule above.  Returns -1 if the
 * row buffers cannot be allocated. */
int32_t oracle_lcs(const uint8_t* a, uint64_t m, const uint8_t* b, uint64_t n) {
  int32_t* prev = (int32_t*)calloc(n + 1, sizeof(int32_t));
  int32_t* cur = (int32_t*)calloc(n + 1, sizeof(int32_t));
  if (!prev || !cur) { free(prev); free(cur); return -1; }
  for (uint64_t i = 1; i <= m; ++i) {
    cur[0] = 0;
    for (uint64_t j = 1; j <= n; ++j) {
      if (a[i - 1] == b[j - 1]) {
        cur[j] = prev[j - 1] + 1;
      } else {
        cur[j] = prev[j] > cur[j - 1] ? prev[j] : cur[j - 1];
      }
    }
    int32_t* t = prev; prev = cur; cur = t;
  }
  int32_t r = prev[n];
  free(prev);
  free(cur);
  return r;
}

/* LCS for a list of pairs (ia[p], ib[p]) of sequences given as concatenated
 * codes with offsets seq_off (nseq + 1 entries).  out[p] receives the value.
 * Returns 0, or -1 on a bad index or an allocation failure. */
int oracle_lcs_pairs(const uint8_t* codes, const uint64_t* seq_off, uint64_t nseq,
                     const uint64_t* ia, const uint64_t* ib, uint64_t npairs, int32_t* out) {
  for (uint64_t p = 0; p < npairs; ++p) {
    uint64_t i = ia[p], j = ib[p];
    if (i >= nseq || j >= nseq) return -1;
    int32_t v = oracle_lcs(codes + seq_off[i], seq_off[i + 1] - seq_off[i],
                           codes + seq_off[j], seq_off[j + 1] - seq_off[j]);
    if (v < 0) return -1;
    out[p] = v;
  }
  return 0;
}

/* Rows [r0, r1) of the upper triangle of one family of k sequences whose
 * first sequence is global index fam_base: row i holds LCS(i, j) for
 * j = i+1 .. k-1, rows back to back (this is the tile layout the library
 * promises).  out must hold sum_{i=r0}^{r1-1} (k-1-i) values. */
int oracle_lcs_rows(const uint8_t* codes, const uint64_t* seq_off, uint64_t fam_base, uint64_t k,
                    uint64_t r0, uint64_t r1, int32_t* out) {
  uint64_t p = 0;
  for (uint64_t i = r0; i < r1 && i < k; ++i) {
    uint64_t gi = fam_base + i;
    for (uint64_t j = i + 1; j < k; ++j) {
      uint64_t gj = fam_base + j;
      int32_t v = oracle_lcs(codes + seq_off[gi], seq_off[gi + 1] - seq_off[gi],
                             codes + seq_off[gj], seq_off[gj + 1] - seq_off[gj]);
      if (v < 0) return -1;
      out[p++] = v;
    }
  }
  return 0;
}
