/*
 * CPU oracle for aligning one sequence to a profile -- TEST INFRASTRUCTURE.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load this file's library.  It shares no source with the GPU path.
 *
 * FAMSA, Methods, "Progressive construction of the alignment": most profile
 * alignments of the progressive stage are of a single sequence against a
 * profile, and the DP is then simpler: the cost of aligning a residue to a
 * profile column is read from the profile's table of column-to-symbol costs.
 * Gap costs are affine with terminal and non-terminal open and extension
 * costs (same section, "Gap types and costs determination").  The caller
 * (oracle/profile.py) derives from the profile, by definition:
 *   cost[(j-1)*sigma + a]  score of aligning symbol a to column j (1..n)
 *   w[j-1]                 profile rows with a residue in column j
 *   ifirst[p], iext[p]     cost of the first and of each further gap column
 *                          inserted into the profile at boundary p (0..n),
 *                          summed over its rows
 * This file runs the three-state dynamic programming (Gotoh's affine-gap
 * scheme) over those numbers and traces one optimal alignment back:
 *
 *   M(i,j) = best(i-1,j-1) + cost(j, a_i)                       i, j >= 1
 *   D(i,j) = max(M(i,j-1) - w_j*o, I(i,j-1) - w_j*o, D(i,j-1) - w_j*e)
 *            with (o, e) = (To, Te) on rows 0 and m (leading and trailing
 *            gaps of the sequence), (Go, Ge) otherwise               j >= 1
 *   I(i,j) = max(M(i-1,j) - ifirst_j, D(i-1,j) - ifirst_j,
 *                I(i-1,j) - iext_j)                                  i >= 1
 *   best = max(M, D, I); the empty prefix is M(0,0) = 0; every state not
 *   listed is unreachable.  D follows I and I follows D directly: the paper
 *   checks consecutive gap columns in both profiles rather than forbidding
 *   them.
 *
 * Ties take the first maximum in the order written above (M, D, I for best;
 * the candidates of D and of I left to right), a documented rule both the
 * oracle and the GPU follow so that the alignment, not only its score, is
 * unique.  Arithmetic is int64; nothing is blocked or reordered.
 */
#include <stdint.h>
#include <stdlib.h>

#define NEG (INT64_MIN / 4)

enum { ST_M = 0, ST_D = 1, ST_I = 2 };

static int argmax3(int64_t x0, int64_t x1, int64_t x2, int64_t* best) {
  int k = 0;
  int64_t b = x0;
  if (x1 > b) { b = x1; k = 1; }
  if (x2 > b) { b = x2; k = 2; }
  *best = b;
  return k;
}

/* Returns 0, or -1 if memory runs out.  ops receives the alignment from its
 * first column to its last: 0 = residue to column (M), 1 = column against a
 * gap in the sequence (D), 2 = residue against a new gap column in the
 * profile (I); it must hold m + n entries. */
int oracle_profile_dp(uint32_t m, const uint8_t* a, uint32_t n, uint32_t sigma, const int64_t* cost,
                      const int64_t* w, const int64_t* ifirst, const int64_t* iext, int64_t To, int64_t Te,
                      int64_t Go, int64_t Ge, int64_t* score, uint8_t* ops, uint32_t* nops) {
  const uint64_t cols = (uint64_t)n + 1, cells = ((uint64_t)m + 1) * cols;
  int64_t* M = (int64_t*)malloc(cells * sizeof(int64_t));
  int64_t* D = (int64_t*)malloc(cells * sizeof(int64_t));
  int64_t* I = (int64_t*)malloc(cells * sizeof(int64_t));
  uint8_t* bestk = (uint8_t*)malloc(cells);
  uint8_t* dsrc = (uint8_t*)malloc(cells);
  uint8_t* isrc = (uint8_t*)malloc(cells);
  if (!M || !D || !I || !bestk || !dsrc || !isrc) {
    free(M); free(D); free(I); free(bestk); free(dsrc); free(isrc);
    return -1;
  }
  for (uint32_t i = 0; i <= m; ++i) {
    for (uint32_t j = 0; j <= n; ++j) {
      const uint64_t c = (uint64_t)i * cols + j;
      int64_t vm = NEG, vd = NEG, vi = NEG;
      uint8_t ds = 0, is = 0;
      if (i == 0 && j == 0) {
        vm = 0;
      }
      if (i >= 1 && j >= 1) {
        const uint64_t dg = (uint64_t)(i - 1) * cols + (j - 1);
        int64_t b;
        argmax3(M[dg], D[dg], I[dg], &b);
        vm = b + cost[(uint64_t)(j - 1) * sigma + a[i - 1]];
      }
      if (j >= 1) {
        const int terminal = (i == 0 || i == m);
        const int64_t o = (terminal ? To : Go) * w[j - 1];
        const int64_t e = (terminal ? Te : Ge) * w[j - 1];
        const uint64_t l = c - 1;
        ds = (uint8_t)argmax3(M[l] - o, I[l] - o, D[l] - e, &vd);
      }
      if (i >= 1) {
        const uint64_t u = c - cols;
        is = (uint8_t)argmax3(M[u] - ifirst[j], D[u] - ifirst[j], I[u] - iext[j], &vi);
      }
      M[c] = vm;
      D[c] = vd;
      I[c] = vi;
      dsrc[c] = ds;
      isrc[c] = is;
      int64_t b;
      bestk[c] = (uint8_t)argmax3(vm, vd, vi, &b);
    }
  }
  const uint64_t end = (uint64_t)m * cols + n;
  int64_t b;
  int st = argmax3(M[end], D[end], I[end], &b);
  *score = b;
  /* trace back from (m, n) to the empty prefix */
  uint32_t i = m, j = n, k = 0;
  while (i > 0 || j > 0) {
    const uint64_t c = (uint64_t)i * cols + j;
    ops[k++] = (uint8_t)st;
    if (st == ST_M) {
      --i; --j;
      st = bestk[(uint64_t)i * cols + j];
    } else if (st == ST_D) {
      const int s = dsrc[c];
      --j;
      st = s == 0 ? ST_M : s == 1 ? ST_I : ST_D;
    } else {
      const int s = isrc[c];
      --i;
      st = s == 0 ? ST_M : s == 1 ? ST_D : ST_I;
    }
  }
  for (uint32_t x = 0; x < k / 2; ++x) {
    const uint8_t t = ops[x];
    ops[x] = ops[k - 1 - x];
    ops[k - 1 - x] = t;
  }
  *nops = k;
  free(M); free(D); free(I); free(bestk); free(dsrc); free(isrc);
  return 0;
}
