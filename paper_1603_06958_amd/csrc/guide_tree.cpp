// The single-linkage guide tree as a merge list (paper, Methods,
// "Determination of the guide tree": FAMSA builds its guide tree by single
// linkage; the progressive stage merges profiles in the tree's bottom-up
// order).
//
// Input: the k-1 edges of a maximum spanning tree of the similarities (or any
// edge set whose single-linkage merges they are, such as SLINK's pointer
// pairs), each with its similarity as the exact rational num/den.  Single
// linkage joins clusters in the order of decreasing similarity, and at each
// join the two clusters are the ones holding the edge's ends (Kruskal).  So:
// sort the edges by similarity, most similar first, equal similarities by the
// pair (u, v), u < v, lexicographically; then union-find over the sorted
// edges gives merge t joining clusters left[t] (holding u) and right[t]
// (holding v) into cluster k + t.  Clusters 0..k-1 are the sequences.
#include <stdint.h>

#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <numeric>
#include <string>
#include <vector>

#include "runtime.h"

namespace famsa {

namespace {

// a strictly more similar than b; den == 0 is +infinity
inline bool more_similar(int64_t an, int64_t ad, int64_t bn, int64_t bd) {
  if (ad == 0) return bd != 0;
  if (bd == 0) return false;
  return (__int128)an * bd > (__int128)bn * ad;
}

}  // namespace

int guide_tree(uint32_t k, const uint32_t* u, const uint32_t* v, const int64_t* num, const int64_t* den,
               uint32_t nedges, uint32_t* left, uint32_t* right, int64_t* mnum, int64_t* mden, uint32_t* nmerges) {
  if (!nmerges) return set_error(FAMSA_LCS_EINVAL, "nmerges is NULL");
  *nmerges = 0;
  if (k == 0) return nedges ? set_error(FAMSA_LCS_EINVAL, "edges given for k = 0") : 0;
  if (nedges > k - 1) return set_error(FAMSA_LCS_EINVAL, "%u edges for %u sequences (at most k-1)", nedges, k);
  if (nedges && (!u || !v || !num || !den)) return set_error(FAMSA_LCS_EINVAL, "NULL edge array");
  std::vector<uint32_t> eu(nedges), ev(nedges), order(nedges);
  for (uint32_t e = 0; e < nedges; ++e) {
    if (u[e] >= k || v[e] >= k || u[e] == v[e])
      return set_error(FAMSA_LCS_EINVAL, "edge %u (%u, %u) is not a pair of distinct sequences < %u", e, u[e], v[e], k);
    if (den[e] < 0 || (den[e] > 0 && num[e] < 0))
      return set_error(FAMSA_LCS_EINVAL, "edge %u: similarity %lld/%lld is not >= 0", e, (long long)num[e],
                       (long long)den[e]);
    eu[e] = std::min(u[e], v[e]);
    ev[e] = std::max(u[e], v[e]);
  }
  std::iota(order.begin(), order.end(), 0u);
  std::sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) {
    if (more_similar(num[a], den[a], num[b], den[b])) return true;
    if (more_similar(num[b], den[b], num[a], den[a])) return false;
    return eu[a] != eu[b] ? eu[a] < eu[b] : ev[a] < ev[b];
  });
  std::vector<uint32_t> parent(k), cluster(k);
  std::iota(parent.begin(), parent.end(), 0u);
  std::iota(cluster.begin(), cluster.end(), 0u);
  auto find = [&](uint32_t x) {
    while (parent[x] != x) {
      parent[x] = parent[parent[x]];
      x = parent[x];
    }
    return x;
  };
  for (uint32_t t = 0; t < nedges; ++t) {
    const uint32_t e = order[t];
    const uint32_t a = find(eu[e]), b = find(ev[e]);
    if (a == b) return set_error(FAMSA_LCS_EINVAL, "edge (%u, %u) closes a cycle: the edges are not a forest", eu[e], ev[e]);
    if (left) left[t] = cluster[a];
    if (right) right[t] = cluster[b];
    if (mnum) mnum[t] = num[e];
    if (mden) mden[t] = den[e];
    parent[a] = b;
    cluster[b] = k + t;
  }
  *nmerges = nedges;
  return 0;
}

// Maximum spanning forest of any edge set under the same total order
// (Kruskal: most similar first, equal similarities by the pair).  The
// forest of a union of edge sets is the forest of the union of their
// forests, so forests of disjoint shards of the tiles merge into the forest
// of all the tiles.
int spanning_forest(uint32_t k, const uint32_t* u, const uint32_t* v, const int64_t* num, const int64_t* den,
                    uint64_t nedges, uint32_t* ou, uint32_t* ov, int64_t* onum, int64_t* oden, uint32_t* nout) {
  if (!nout) return set_error(FAMSA_LCS_EINVAL, "nout is NULL");
  *nout = 0;
  if (nedges && (!u || !v || !num || !den)) return set_error(FAMSA_LCS_EINVAL, "NULL edge array");
  std::vector<uint32_t> eu(nedges), ev(nedges);
  std::vector<uint64_t> order(nedges);
  for (uint64_t e = 0; e < nedges; ++e) {
    if (u[e] >= k || v[e] >= k || u[e] == v[e])
      return set_error(FAMSA_LCS_EINVAL, "edge %llu (%u, %u) is not a pair of distinct sequences < %u",
                       (unsigned long long)e, u[e], v[e], k);
    if (den[e] < 0 || (den[e] > 0 && num[e] < 0))
      return set_error(FAMSA_LCS_EINVAL, "edge %llu: similarity %lld/%lld is not >= 0", (unsigned long long)e,
                       (long long)num[e], (long long)den[e]);
    eu[e] = std::min(u[e], v[e]);
    ev[e] = std::max(u[e], v[e]);
    order[e] = e;
  }
  std::sort(order.begin(), order.end(), [&](uint64_t a, uint64_t b) {
    if (more_similar(num[a], den[a], num[b], den[b])) return true;
    if (more_similar(num[b], den[b], num[a], den[a])) return false;
    return eu[a] != eu[b] ? eu[a] < eu[b] : ev[a] < ev[b];
  });
  std::vector<uint32_t> parent(k);
  std::iota(parent.begin(), parent.end(), 0u);
  auto find = [&](uint32_t x) {
    while (parent[x] != x) {
      parent[x] = parent[parent[x]];
      x = parent[x];
    }
    return x;
  };
  uint32_t n = 0;
  for (uint64_t t = 0; t < nedges; ++t) {
    const uint64_t e = order[t];
    const uint32_t a = find(eu[e]), b = find(ev[e]);
    if (a == b) continue;  // closes a cycle: not in the forest
    parent[a] = b;
    if (ou) ou[n] = eu[e];
    if (ov) ov[n] = ev[e];
    if (onum) onum[n] = num[e];
    if (oden) oden[n] = den[e];
    ++n;
  }
  *nout = n;
  return 0;
}

}  // namespace famsa

extern "C" int famsa_spanning_forest(uint32_t k, const uint32_t* u, const uint32_t* v, const int64_t* num,
                                     const int64_t* den, uint64_t nedges, uint32_t* out_u, uint32_t* out_v,
                                     int64_t* out_num, int64_t* out_den, uint32_t* nout) {
  famsa::clear_error();
  return famsa::spanning_forest(k, u, v, num, den, nedges, out_u, out_v, out_num, out_den, nout);
}

extern "C" int famsa_guide_tree(uint32_t k, const uint32_t* u, const uint32_t* v, const int64_t* num,
                                const int64_t* den, uint32_t nedges, uint32_t* left, uint32_t* right,
                                int64_t* merge_num, int64_t* merge_den, uint32_t* nmerges) {
  famsa::clear_error();
  return famsa::guide_tree(k, u, v, num, den, nedges, left, right, merge_num, merge_den, nmerges);
}

namespace {

// Children of every cluster and the roots (clusters no merge consumed), after
// checking that the merge list is well formed.
int tree_children(uint32_t k, const uint32_t* left, const uint32_t* right, uint32_t nmerges,
                  std::vector<uint32_t>* roots) {
  if (nmerges > (k ? k - 1 : 0)) return famsa::set_error(FAMSA_LCS_EINVAL, "%u merges for %u leaves", nmerges, k);
  if (nmerges && (!left || !right)) return famsa::set_error(FAMSA_LCS_EINVAL, "NULL merge array");
  std::vector<uint8_t> used(k + nmerges, 0);
  for (uint32_t t = 0; t < nmerges; ++t) {
    const uint32_t a = left[t], b = right[t];
    if (a >= k + t || b >= k + t || a == b || used[a] || used[b])
      return famsa::set_error(FAMSA_LCS_EINVAL, "merge %u (%u, %u) is not a merge of two current clusters", t, a, b);
    used[a] = used[b] = 1;
  }
  roots->clear();
  for (uint32_t c = 0; c < k + nmerges; ++c)
    if (!used[c]) roots->push_back(c);
  return 0;
}

}  // namespace

extern "C" int famsa_guide_tree_leaf_order(uint32_t k, const uint32_t* left, const uint32_t* right, uint32_t nmerges,
                                           uint32_t* order, uint32_t* first, uint32_t* size) {
  famsa::clear_error();
  std::vector<uint32_t> roots;
  int rc = tree_children(k, left, right, nmerges, &roots);
  if (rc) return rc;
  // leaves in depth-first order, left subtree first; a cluster's leaves are
  // then one contiguous range
  const uint32_t nc = k + nmerges;
  std::vector<uint32_t> f(nc, 0), n(nc, 0);
  for (uint32_t c = 0; c < k; ++c) n[c] = 1;
  for (uint32_t t = 0; t < nmerges; ++t) n[k + t] = n[left[t]] + n[right[t]];
  uint32_t next = 0;
  for (uint32_t r : roots) {
    f[r] = next;
    next += n[r];
  }
  for (uint32_t t = nmerges; t-- > 0;) {  // parents before children
    const uint32_t c = k + t;
    f[left[t]] = f[c];
    f[right[t]] = f[c] + n[left[t]];
  }
  for (uint32_t c = 0; c < k; ++c)
    if (order) order[f[c]] = c;
  for (uint32_t c = 0; c < nc; ++c) {
    if (first) first[c] = f[c];
    if (size) size[c] = n[c];
  }
  return 0;
}

extern "C" int famsa_guide_tree_newick(uint32_t k, const uint32_t* left, const uint32_t* right, uint32_t nmerges,
                                       char* buf, uint64_t buf_size, uint64_t* needed) {
  famsa::clear_error();
  if (!needed) return famsa::set_error(FAMSA_LCS_EINVAL, "needed is NULL");
  std::vector<uint32_t> roots;
  int rc = tree_children(k, left, right, nmerges, &roots);
  if (rc) return rc;
  // iterative walk: emit "(" on entering a merge, "," between its children,
  // ")" on leaving; leaves by index; several roots are wrapped together
  std::string out;
  std::vector<std::pair<uint32_t, int>> st;  // (cluster, children done)
  char num[16];
  if (roots.size() != 1) out += '(';
  for (size_t ri = 0; ri < roots.size(); ++ri) {
    if (ri) out += ',';
    st.push_back({roots[ri], 0});
    while (!st.empty()) {
      auto& top = st.back();
      const uint32_t c = top.first;
      if (c < k) {
        snprintf(num, sizeof num, "%u", c);
        out += num;
        st.pop_back();
        continue;
      }
      const uint32_t t = c - k;
      if (top.second == 0) {
        out += '(';
        top.second = 1;
        st.push_back({left[t], 0});
      } else if (top.second == 1) {
        out += ',';
        top.second = 2;
        st.push_back({right[t], 0});
      } else {
        out += ')';
        st.pop_back();
      }
    }
  }
  if (roots.size() != 1) out += ')';
  out += ';';
  *needed = out.size() + 1;
  if (buf && buf_size >= out.size() + 1) memcpy(buf, out.c_str(), out.size() + 1);
  else if (buf) return famsa::set_error(FAMSA_LCS_EINVAL, "buffer of %llu bytes, %llu needed",
                                        (unsigned long long)buf_size, (unsigned long long)(out.size() + 1));
  return 0;
}
