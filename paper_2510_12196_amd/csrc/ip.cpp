// ip.cpp -- initial partitioning of the coarsest graph on the host.
//
// Section 4.2 runs the initial partitioning on the CPU: the coarsest graph is
// small, so the device would gain nothing.  The method is hierarchical
// multisection (Section 4.1, Algorithm 2): split the graph into a_l pieces,
// each piece into a_{l-1} pieces, and so on; the piece index at level i is
// the level-i mixed-radix digit of the PE id.  The "simple k-way graph
// partitioner" used at every split is a breadth-first split: visit the
// subgraph breadth-first (start at its smallest vertex id, neighbours in
// ascending id, restart at the smallest unvisited id), and cut the visiting
// order into a_i consecutive pieces at the first positions where the
// exclusive running weight reaches ceil(j * c(V') / a_i), j = 1..a_i-1.
#include <algorithm>
#include <vector>

#include "host_ip.h"

namespace pm {

namespace {

struct Task {
  std::vector<int32_t> verts;  // ascending ids
  int level;                   // 1-based hierarchy level to split at
  int64_t base;                // PE id of digit prefix fixed so far
};

}  // namespace

void host_initial_partition(int32_t n, const int64_t *xadj, const int32_t *adj,
                            const int32_t *vwgt, const Hier &h, int32_t *part_ids) {
  // rows sorted ascending once, so that breadth-first visits are canonical
  std::vector<int32_t> sorted(adj, adj + (n ? xadj[n] : 0));
  for (int32_t v = 0; v < n; ++v)
    std::sort(sorted.begin() + xadj[v], sorted.begin() + xadj[v + 1]);

  std::vector<int32_t> stamp(n, -1);
  std::vector<uint8_t> seen(n, 0);
  std::vector<int32_t> order;
  std::vector<int32_t> piece_of(n, 0);
  int32_t next_stamp = 0;

  std::vector<Task> stack;
  Task root;
  root.verts.resize(n);
  for (int32_t v = 0; v < n; ++v) root.verts[v] = v;
  root.level = h.levels;
  root.base = 0;
  stack.push_back(std::move(root));

  while (!stack.empty()) {
    Task t = std::move(stack.back());
    stack.pop_back();
    if (t.verts.empty()) continue;
    const int64_t ai = h.a[t.level - 1];
    const int64_t stride = h.P[t.level - 1];
    const int32_t mark = next_stamp++;
    int64_t wsum = 0;
    for (int32_t v : t.verts) {
      stamp[v] = mark;
      seen[v] = 0;
      wsum += vwgt[v];
    }
    // breadth-first order over the subgraph
    order.clear();
    for (int32_t root_v : t.verts) {
      if (seen[root_v]) continue;
      seen[root_v] = 1;
      size_t head = order.size();
      order.push_back(root_v);
      while (head < order.size()) {
        const int32_t x = order[head++];
        for (int64_t e = xadj[x]; e < xadj[x + 1]; ++e) {
          const int32_t y = sorted[e];
          if (stamp[y] == mark && !seen[y]) {
            seen[y] = 1;
            order.push_back(y);
          }
        }
      }
    }
    // pieces: advance the piece index while the running weight reaches the
    // next proportional threshold
    int64_t running = 0;
    int64_t piece = 0;
    for (int32_t x : order) {
      while (piece + 1 < ai && running >= ((piece + 1) * wsum + ai - 1) / ai) ++piece;
      piece_of[x] = (int32_t)piece;
      running += vwgt[x];
    }
    if (t.level == 1) {
      for (int32_t v : t.verts) part_ids[v] = (int32_t)(t.base + piece_of[v]);
      continue;
    }
    std::vector<Task> children(ai);
    for (int64_t j = 0; j < ai; ++j) {
      children[j].level = t.level - 1;
      children[j].base = t.base + j * stride;
    }
    for (int32_t v : t.verts) children[piece_of[v]].verts.push_back(v);  // stays ascending
    for (int64_t j = ai - 1; j >= 0; --j) stack.push_back(std::move(children[j]));
  }
}

}  // namespace pm
