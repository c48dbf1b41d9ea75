// Contraction order of a tensor network (Sec. "Network", "Setting the
// contraction order"): dynamic programming over subsets of tensors with the
// cost capping of Pfeifer, Haegeman and Verstraete (Phys. Rev. E 90, 033315,
// 2014).  The cost of a pairwise contraction is the product of the dims of
// every index it touches (each index once), the dense multiply-add count.
// The cap bounds the accumulated cost of the subsets kept; it grows until
// the whole network is reached, so the order found is an exact optimum.
#include <cmath>
#include <limits>
#include <vector>

#include "plan.h"

using namespace bst;

extern "C" bst_status bst_network_order(int32_t n, const int32_t* nlegs, const int32_t* legs,
                                        int32_t nid, const int64_t* dims, int32_t* pairs,
                                        double* cost) {
  BST_TRY
  if (n < 1 || n > 16) fail(BST_E_INVALID, "a network holds 1..16 tensors");
  if (nid < 0 || nid > 64) fail(BST_E_INVALID, "at most 64 distinct indices");
  if (!nlegs || (nid > 0 && !dims)) fail(BST_E_INVALID, "null argument");
  // indices of each tensor as a bit set; an index on one tensor only is open
  std::vector<uint64_t> ids(n, 0);
  std::vector<int> count(nid, 0);
  int64_t k = 0;
  for (int t = 0; t < n; ++t) {
    if (nlegs[t] < 0) fail(BST_E_INVALID, "negative leg count");
    if (nlegs[t] > 0 && !legs) fail(BST_E_INVALID, "null argument");
    for (int l = 0; l < nlegs[t]; ++l, ++k) {
      const int32_t id = legs[k];
      if (id < 0 || id >= nid) fail(BST_E_INVALID, "index id out of range");
      if (ids[t] >> id & 1) fail(BST_E_INVALID, "an index appears twice on one tensor");
      ids[t] |= uint64_t(1) << id;
      count[id]++;
    }
  }
  uint64_t open = 0;
  for (int id = 0; id < nid; ++id) {
    if (count[id] > 2) fail(BST_E_INVALID, "an index joins more than two tensors");
    if (dims[id] < 1) fail(BST_E_INVALID, "index dims must be >= 1");
    if (count[id] == 1) open |= uint64_t(1) << id;
  }
  const uint32_t full = (1u << n) - 1u;
  const size_t ns = size_t(1) << n;
  // indices of a subset's tensor: those it holds that are open or reach out
  std::vector<uint64_t> all(ns, 0);
  for (uint32_t s = 1; s < ns; ++s) {
    const int t = __builtin_ctz(s);
    all[s] = all[s & (s - 1)] | ids[t];
  }
  auto legs_of = [&](uint32_t s) { return all[s] & (open | all[full & ~s]); };
  auto dimprod = [&](uint64_t m) {
    double p = 1.0;
    while (m) {
      const int id = __builtin_ctzll(m);
      p *= (double)dims[id];
      m &= m - 1;
    }
    return p;
  };
  const double inf = std::numeric_limits<double>::infinity();
  std::vector<double> best(ns, inf);
  std::vector<uint32_t> split(ns, 0);
  // first cap: the cheapest single pairwise step (at least 1)
  double cap = inf;
  for (int a = 0; a < n; ++a)
    for (int b = a + 1; b < n; ++b)
      cap = std::min(cap, dimprod(legs_of(1u << a) | legs_of(1u << b)));
  if (!(cap >= 1.0)) cap = 1.0;
  while (true) {
    std::fill(best.begin(), best.end(), inf);
    for (int t = 0; t < n; ++t) best[1u << t] = 0.0;
    for (uint32_t s = 1; s < ns; ++s) {
      if ((s & (s - 1)) == 0) continue;
      const uint32_t low = s & (~s + 1);
      // proper subsets a of s holding s's lowest tensor; b = s \ a
      for (uint32_t a = (s - 1) & s; a; a = (a - 1) & s) {
        if (!(a & low)) continue;
        const uint32_t b = s ^ a;
        const double ca = best[a], cb = best[b];
        if (ca == inf || cb == inf) continue;
        const double c = ca + cb + dimprod(legs_of(a) | legs_of(b));
        if (c <= cap && c < best[s]) {
          best[s] = c;
          split[s] = a;
        }
      }
    }
    if (best[full] != inf || n == 1) break;
    cap *= 8.0;
  }
  if (cost) *cost = n == 1 ? 0.0 : best[full];
  if (pairs) {
    // post-order: node ids 0..n-1 are the inputs, n + k the result of step k
    int step = 0;
    std::vector<int32_t> node(ns, -1);
    for (int t = 0; t < n; ++t) node[1u << t] = t;
    std::vector<std::pair<uint32_t, bool>> stack{{full, false}};
    while (!stack.empty()) {
      auto [s, done] = stack.back();
      stack.pop_back();
      if (node[s] >= 0) continue;
      const uint32_t a = split[s], b = s ^ a;
      if (!done) {
        stack.push_back({s, true});
        stack.push_back({b, false});
        stack.push_back({a, false});
        continue;
      }
      pairs[2 * step] = node[a];
      pairs[2 * step + 1] = node[b];
      node[s] = n + step;
      ++step;
    }
  }
  BST_CATCH
}
