// planner.hip -- host-side work ordering for the block GEMM (no device code).
//
// The result blocks of one block row read the B rows k of every stored
// A(i,k); rows whose atoms are close in space share most of those k.  In a
// random atom order (DBCSR permutes rows and columns on purpose for static
// load balance across processes, arXiv:1705.10218 Section 2) consecutive
// rows share nothing, so every B block is fetched from HBM again for each
// of the ~100 rows that need it.  This planner derives a locality order of
// the block rows from the block pattern alone (no coordinates): recursive
// bisection by breadth-first-search distance from a pseudo-peripheral row,
// the coordinate-free analogue of cutting space in halves.  The GEMM then
// walks C in that order and gives each XCD (with its own L2) a contiguous
// piece of it.  The order changes only which C block runs when: every C
// block is computed by one wavefront in the same summation order, so the
// results are bitwise the same in any order.
#include <algorithm>
#include <cstdint>
#include <vector>

#include "internal.h"

namespace bsmm {

namespace {

struct Bisect {
  const std::vector<int64_t> &rp;
  const std::vector<int32_t> &ci;
  std::vector<int32_t> stamp;    // set membership: stamp[v] == cur
  std::vector<int32_t> dist;
  std::vector<int32_t> queue;
  std::vector<int32_t> out;
  int32_t cur = 0;

  Bisect(const std::vector<int64_t> &r, const std::vector<int32_t> &c, int32_t n)
      : rp(r), ci(c), stamp(n, -1), dist(n, -1), queue(n) {
    out.reserve(n);
  }

  // BFS inside the current set from src; returns the last node reached and
  // leaves distances in dist[] (-1 for nodes of the set not reached).
  int32_t bfs(const std::vector<int32_t> &set, int32_t src) {
    for (int32_t v : set) dist[v] = -1;
    int32_t head = 0, tail = 0;
    queue[tail++] = src;
    dist[src] = 0;
    int32_t last = src;
    while (head < tail) {
      int32_t v = queue[head++];
      last = v;
      for (int64_t p = rp[v]; p < rp[v + 1]; p++) {
        int32_t u = ci[p];
        if (u < (int32_t)stamp.size() && stamp[u] == cur && dist[u] < 0) {
          dist[u] = dist[v] + 1;
          queue[tail++] = u;
        }
      }
    }
    return last;
  }

  void order(std::vector<int32_t> &set) {
    if (set.size() <= 32) {
      std::sort(set.begin(), set.end());
      out.insert(out.end(), set.begin(), set.end());
      return;
    }
    cur++;
    for (int32_t v : set) stamp[v] = cur;
    int32_t far = bfs(set, set[0]);
    bfs(set, far);
    // unreached nodes (another component) go last, ties by index
    const int32_t big = INT32_MAX;
    std::vector<std::pair<int32_t, int32_t>> key(set.size());
    for (size_t t = 0; t < set.size(); t++) {
      int32_t v = set[t];
      key[t] = {dist[v] < 0 ? big : dist[v], v};
    }
    std::sort(key.begin(), key.end());
    size_t half = set.size() / 2;
    std::vector<int32_t> s1(half), s2(set.size() - half);
    for (size_t t = 0; t < half; t++) s1[t] = key[t].second;
    for (size_t t = half; t < set.size(); t++) s2[t - half] = key[t].second;
    set.clear();
    set.shrink_to_fit();
    order(s1);
    order(s2);
  }
};

}  // namespace

std::vector<int32_t> locality_order(int32_t n, const std::vector<int64_t> &rp, const std::vector<int32_t> &ci) {
  Bisect b(rp, ci, n);
  std::vector<int32_t> all(n);
  for (int32_t v = 0; v < n; v++) all[v] = v;
  b.order(all);
  return b.out;
}

}  // namespace bsmm
